"""Eshelby verification in 3D (the paper's Sec. 4.1 study).

Sphere case: a
spherical inclusion of radius a with dilatational eigenstrain eps* and its
own isotropic moduli in an isotropic matrix.  The sharp-interface solution
is radial: u = A x inside, u = A a^3 x / r^3 outside, with A = 3 k_i eps* /
(3 k_i + 4 mu_m) from traction continuity at r = a (k_i the inclusion's bulk
modulus, mu_m the matrix shear modulus); it is imposed on every face of
[-1, 1]^3.  The GPU's diffuse-interface solution (tanh profile two cells
wide) approaches it away from the interface as the grid and the interface
width shrink together (65^3, 129^3, 257^3).

Ellipsoid case (the paper's configuration: semi-axes (1, 0.75, 0.5) centred
in [-4, 4]^3, E = 210, nu = 0.3 everywhere, eigenstrain 1e-3 I inside, the
error-function mollification of width 0.1): inside the inclusion the exact
strain is uniform, eps = S : eps* with S the Eshelby tensor of the
ellipsoid (oracle.eshelby, pinned on the CPU), so the interior displacement
is linear.  The tests fit a linear field to the GPU displacement over the
nodes with x^T A x <= 1/2 (away from the diffuse surface) and compare the
fitted strain with S : eps*.  The faces carry the far field of the
equivalent centre of dilatation."""
import numpy as np
import pytest

import synth
from oracle import eshelby

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def emg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_04789_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(emg):
    c = emg.Context(0)
    yield c
    c.close()


def sphere_problem(n, L=1.0, a=0.25, wcells=2.0):
    lam_m, mu_m, lam_i, mu_i, es = 1.5, 1.0, 3.0, 2.0, 1e-3
    p = synth.Problem(dim=3, n=(n, n, n), lo=(-L, -L, -L), hi=(L, L, L), bc=("dirichlet",) * 6, kind="iso",
                      C=np.zeros(0))
    x, y, z = p.coords()
    r = np.sqrt(x ** 2 + y ** 2 + z ** 2)
    eta = 0.5 * (1 - np.tanh((r - a) / (wcells * 2 * L / (n - 1))))
    p.C = np.ascontiguousarray(np.stack([lam_m + (lam_i - lam_m) * eta, mu_m + (mu_i - mu_m) * eta]))
    e = es * eta
    p.eps0 = np.ascontiguousarray(np.stack([e, e, e, 0 * e, 0 * e, 0 * e]))
    k_i = lam_i + 2.0 * mu_i / 3.0
    A = 3.0 * k_i * es / (3.0 * k_i + 4.0 * mu_m)
    fac = np.where(r <= a, A, A * a ** 3 / np.maximum(r, a) ** 3)
    uex = np.stack([fac * x + 0 * y * z, fac * y + 0 * x * z, fac * z + 0 * x * y])
    for f in range(6):
        sl = [slice(None)] * 3
        sl[2 - f // 2] = slice(0, 1) if f % 2 == 0 else slice(n - 1, n)
        p.face[f] = np.ascontiguousarray(uex[(slice(None),) + tuple(sl)])
    return p, uex, np.broadcast_to(r, uex.shape[1:])


def test_eshelby_sphere_closed_form(emg, ctx):
    errs = []
    for n in (65, 129, 257):
        p, uex, r = sphere_problem(n)
        prob = emg.Problem.from_spec(ctx, p)
        st = prob.solve(rtol=1e-10, max_cycles=400, precision="mixed")
        u = prob.displacement()
        prob.close()
        far = np.broadcast_to(np.abs(r - 0.25) > 0.2, uex.shape)
        err = float(np.abs(u - uex)[far].max() / np.abs(uex).max())
        errs.append(err)
        print(f"[gpu] Eshelby sphere n={n}: cycles {st['cycles']} max error away from the interface {err:.3e}",
              flush=True)
        assert st["converged"]
    # measured: 3.1e-2, 5.9e-3, 3.4e-3
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.8 * errs[1]
    assert errs[2] < 1e-2


AXES = (1.0, 0.75, 0.5)


def fitted_strain(ap, prob):
    """Least-squares slope of u_i against x_i (plus a constant) over the
    finest level's nodes with x^T A x <= 1/2, and the relative deviation of
    each slope from Eshelby's interior strain."""
    k = len(ap.boxes)
    if k == 0:
        u = prob.displacement()
        X, Y, Z = np.broadcast_arrays(*ap.base.coords())
    else:
        u = prob.amr_displacement(k)
        X, Y, Z = np.broadcast_arrays(*ap.box_coords(k))
    q = (X / AXES[0]) ** 2 + (Y / AXES[1]) ** 2 + (Z / AXES[2]) ** 2
    m = q <= 0.5
    fit = []
    for i, Xi in enumerate((X, Y, Z)):
        A = np.stack([Xi[m], np.ones(int(m.sum()))], 1)
        c, *_ = np.linalg.lstsq(A, u[i][m], rcond=None)
        fit.append(c[0])
    exact = np.diag(eshelby.interior_strain(AXES, 0.3, 1e-3 * np.eye(3)))
    return np.array(fit), (np.array(fit) - exact) / exact


def test_eshelby_ellipsoid_uniform_grid(emg, ctx):
    """One uniform 129^3 grid (h = 1/16): the fitted interior strain is
    Eshelby's to 1e-3 (measured: 4.5e-4, 1.1e-4, 2.0e-4)."""
    ap = synth.eshelby_ellipsoid_amr(n0=129, levels=1)
    prob = emg.Problem.from_amr(ctx, ap)
    st = prob.solve(rtol=1e-10, max_cycles=300)
    fit, dev = fitted_strain(ap, prob)
    prob.close()
    print(f"[gpu] Eshelby ellipsoid 129^3 uniform: cycles {st['cycles']} interior strain {fit} rel dev {dev}",
          flush=True)
    assert st["converged"]
    assert np.abs(dev).max() < 1e-3


def test_eshelby_ellipsoid_amr_converges(emg, ctx):
    """Two fixed refined boxes ([-2, 2]^3, then [-1.5, 1.5] x [-1.25, 1.25]
    x [-1, 1]) over base grids of 33, 65 and 129 nodes per axis: the
    fitted interior strain approaches Eshelby's at first order in h, the
    order of the coarse/fine rows (their truncation error is O(1) on one
    layer of nodes, as the App. A stencil shows).  Measured max relative
    deviation 3.0e-3, 1.6e-3, 7.8e-4."""
    boxes = [((-2.0,) * 3, (2.0,) * 3), ((-1.5, -1.25, -1.0), (1.5, 1.25, 1.0))]
    errs = []
    for n0 in (33, 65, 129):
        ap = synth.eshelby_ellipsoid_amr(n0=n0, phys_boxes=boxes)
        prob = emg.Problem.from_amr(ctx, ap)
        st = prob.solve(rtol=1e-10, max_cycles=300)
        fit, dev = fitted_strain(ap, prob)
        prob.close()
        errs.append(float(np.abs(dev).max()))
        print(f"[gpu] Eshelby ellipsoid AMR base {n0}^3 + 2 boxes: cycles {st['cycles']} rel dev {dev}", flush=True)
        assert st["converged"]
    assert errs[1] < 0.65 * errs[0] and errs[2] < 0.65 * errs[1]
    assert errs[2] < 1.5e-3


def test_eshelby_ellipsoid_paper_hierarchy(emg, ctx):
    """The paper's hierarchy: base 32^3 cells and five levels, each box the
    bounding box of the nodes tagged by |grad eta| |dx| > 0.01 (finest
    h = 1/64, 2.1 M composite nodes).  The tagged boxes hug the inclusion,
    so the coarse/fine rows sit where the exterior field still varies
    quickly: fitted interior strain within 1.5 % (measured -0.2 %, 0.45 %,
    1.05 %); the paper reports 1.6-2.8 % displacement errors along a line
    through the inclusion for its own comparison."""
    ap = synth.eshelby_ellipsoid_amr(n0=33, levels=5)
    assert len(ap.boxes) == 4
    prob = emg.Problem.from_amr(ctx, ap)
    st = prob.solve(rtol=1e-10, max_cycles=300)
    fit, dev = fitted_strain(ap, prob)
    prob.close()
    print(f"[gpu] Eshelby ellipsoid paper hierarchy {ap.boxes}: composite nodes {ap.composite_nodes()} "
          f"cycles {st['cycles']} rel dev {dev}", flush=True)
    assert st["converged"]
    assert np.abs(dev).max() < 1.5e-2
