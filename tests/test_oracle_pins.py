"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: exactness of
the finite differences on polynomial fields (with the analytic operator built
symbolically in divergence form), rigid-body null spaces, symmetry of the
constant-coefficient operator, the textbook Laplacian it reduces to, the
stress-free eigenstrain, the Eshelby disc closed form, dense direct solves,
invariances under translation and axis exchange, and transfer identities.
"""
import numpy as np
import pytest
import sympy as sp

import oracle
import synth

X = sp.symbols("x y z")


# --------------------------------------------------------------------------
# helpers (test-side constructions, independent of the oracle's code)
# --------------------------------------------------------------------------

def _sym_tensor(rng, scale):
    """Random fourth-order tensor with major and minor symmetry."""
    A = rng.uniform(-1, 1, size=(3, 3, 3, 3))
    T = (A + A.transpose(1, 0, 2, 3) + A.transpose(0, 1, 3, 2) + A.transpose(1, 0, 3, 2))
    T = T + T.transpose(2, 3, 0, 1)
    return scale * T / 8.0


def _q2(rng, dim, scale):
    e = 0
    for a in range(3):
        for b in range(3):
            for c in range(3 if dim == 3 else 1):
                e += scale * rng.uniform(-1, 1) * X[0] ** a * X[1] ** b * X[2] ** c
    return e


def _eval(expr, x, y, z, shape):
    f = sp.lambdify(X, expr, "numpy")
    return np.broadcast_to(np.asarray(f(x, y, z), dtype=float), shape).copy()


def _stored_moduli(Tfield, dim):
    """Moduli arrays in the stored Voigt layout from a per-node full tensor
    field (built with the input-format helpers of ``synth``)."""
    shp = Tfield.shape[4:]
    flat = Tfield.reshape(3, 3, 3, 3, -1)
    comps = []
    for q in range(flat.shape[-1]):
        V = synth.tensor_to_voigt(flat[..., q])
        if dim == 2:
            V = synth.plane_strain_voigt(V)
        comps.append(synth.upper_tri(V))
    return np.array(comps).T.reshape((-1,) + shp)


def _grid(p):
    return oracle.Grid.of(p)


def polynomial_problem(dim, bc, seed, n=(7, 6, 5), lo=(0.1, -0.4, 0.2), hi=(1.3, 0.5, 0.9)):
    """Q2 displacement, Q2 anisotropic moduli and Q2 eigenstrain; body force
    and boundary data from the analytic operator in divergence form."""
    rng = np.random.default_rng(seed)
    d = dim
    n3 = tuple(n[:d]) + (1,) * (3 - d)
    p = synth.Problem(dim=d, n=n3, lo=lo, hi=tuple(hi[a] if a < d else lo[a] for a in range(3)), bc=tuple(bc),
                      kind="aniso", C=np.zeros(0))
    x, y, z = p.coords()
    m = p.m
    shp = (m[2], m[1], m[0])
    T0 = synth.voigt_to_tensor(synth.rotate_voigt(synth.cubic_voigt(*synth.CUBIC), synth.shoemake_rotation(rng.random(3))))
    T1, T2 = _sym_tensor(rng, 0.1), _sym_tensor(rng, 0.1)
    phi1, phi2 = _q2(rng, d, 1.0), _q2(rng, d, 1.0)
    Csym = [[[[T0[i, j, k, l] + phi1 * T1[i, j, k, l] + phi2 * T2[i, j, k, l] for l in range(3)] for k in range(3)]
             for j in range(3)] for i in range(3)]
    E0 = rng.uniform(-1, 1, size=(3, 3)); E0 = 1e-2 * (E0 + E0.T)
    E1 = rng.uniform(-1, 1, size=(3, 3)); E1 = 1e-2 * (E1 + E1.T)
    psi = _q2(rng, d, 1.0)
    eps = [[E0[k, l] + psi * E1[k, l] for l in range(3)] for k in range(3)]
    u = [_q2(rng, d, 0.1) for _ in range(d)]
    sig = [[sum(Csym[i][j][k][l] * (sp.diff(u[k], X[l]) - eps[k][l]) for k in range(d) for l in range(d))
            for j in range(d)] for i in range(d)]
    D = [sum(sp.diff(sig[i][j], X[j]) for j in range(d)) for i in range(d)]

    Tfield = np.empty((3, 3, 3, 3) + shp)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    Tfield[i, j, k, l] = _eval(Csym[i][j][k][l], x, y, z, shp)
    p.C = _stored_moduli(Tfield, d)
    pairs = [(0, 0), (1, 1), (2, 2), (1, 2), (2, 0), (0, 1)] if d == 3 else [(0, 0), (1, 1), (0, 1)]
    p.eps0 = np.stack([_eval(eps[k][l], x, y, z, shp) for k, l in pairs])
    p.b = np.stack([-_eval(D[i], x, y, z, shp) for i in range(d)])
    u_nodal = np.stack([_eval(u[k], x, y, z, shp) for k in range(d)])
    sig_nodal = np.stack([_eval(sig[i][j], x, y, z, shp) for i, j in pairs])
    for f in range(2 * d):
        a = f // 2
        sl = [slice(None)] * 3
        sl[2 - a] = slice(0, 1) if f % 2 == 0 else slice(m[a] - 1, m[a])
        sl = tuple(sl)
        if bc[f] == synth.DIRICHLET:
            p.face[f] = u_nodal[(slice(None),) + sl].copy()
        elif bc[f] == synth.TRACTION:
            nsign = -1.0 if f % 2 == 0 else 1.0
            t = [sum(_eval(sig[i][j], x, y, z, shp)[sl] * (nsign if j == a else 0.0) for j in range(d))
                 for i in range(d)]
            p.face[f] = np.stack(t)
        elif bc[f] == synth.NEUMANN:   # du_i/dx_j n_j (eq. elastic_b3)
            nsign = -1.0 if f % 2 == 0 else 1.0
            p.face[f] = np.stack([nsign * _eval(sp.diff(u[i], X[a]), x, y, z, shp)[sl] for i in range(d)])
    return p, u_nodal, sig_nodal


BC3 = ("dirichlet", "traction", "traction", "traction", "traction", "dirichlet")
BC2 = ("traction", "traction", "dirichlet", "traction", "periodic", "periodic")


@pytest.mark.parametrize("dim,bc,seed", [(3, BC3, 1), (2, BC2, 2),
                                         (3, ("traction", "dirichlet", "dirichlet", "traction", "traction", "traction"), 3),
                                         (3, ("neumann", "traction", "dirichlet", "neumann", "traction", "neumann"), 4),
                                         (2, ("neumann", "neumann", "dirichlet", "traction", "periodic", "periodic"), 5),
                                         (3, ("dirichlet", "neumann", "neumann", "neumann", "traction", "neumann"), 6)])
def test_polynomial_exactness(dim, bc, seed):
    """P1: on Q2 fields every row (interior, traction and Neumann incl.
    edges and corners, Dirichlet) equals the analytic operator or boundary
    condition at the node, so
    rhs - D_H(u) vanishes to rounding; the dense solve returns the nodal u;
    the stress equals the analytic stress at every node."""
    p, u, sig = polynomial_problem(dim, bc, seed)
    g = _grid(p)
    f = oracle.rhs(g, p.C, p.eps0, p.b, p.face)
    Au = oracle.apply(g, p.C, u)
    scale = np.abs(Au).max() + np.abs(f).max()
    assert np.abs(f - Au).max() <= 1e-12 * scale
    us = oracle.dense_solve(p)
    assert np.abs(us - u).max() <= 1e-10 * np.abs(u).max()
    s = oracle.stress(g, p.C, p.eps0, u)
    assert np.abs(s - sig).max() <= 1e-12 * np.abs(sig).max()


@pytest.mark.parametrize("dim,kind", [(2, "iso"), (3, "aniso"), (3, "iso"), (2, "aniso")])
def test_rigid_body_null_space(dim, kind):
    """P2: translations and infinitesimal rotations are in the kernel of
    every interior and traction row, for moduli varying node to node."""
    bc = ("traction", "traction", "dirichlet", "traction", "traction", "traction") if dim == 2 else \
        ("traction", "traction", "traction", "traction", "dirichlet", "traction")
    p = synth.random_problem(dim, (7, 6, 5)[:dim], bc, kind, seed=11, smooth=False)
    g = _grid(p)
    x, y, z = p.coords()
    shp = (p.m[2], p.m[1], p.m[0])
    cls = oracle.row_class(g)
    rng = np.random.default_rng(0)
    W = rng.uniform(-1, 1, size=(3, 3)); W = W - W.T
    pos = [np.broadcast_to(c, shp) for c in (x, y, z)]
    fields = [np.stack([np.full(shp, rng.uniform(-1, 1)) for _ in range(dim)]),
              np.stack([sum(W[k, l] * pos[l] for l in range(dim)) for k in range(dim)])]
    for u in fields:
        Au = oracle.apply(g, p.C, u)
        mask = np.broadcast_to(cls != oracle.ROW_DIRICHLET, Au.shape)
        assert np.abs(Au[mask]).max() <= 1e-12 * np.abs(p.C).max() * np.abs(u).max() / min(p.h[:dim]) ** 2


@pytest.mark.parametrize("dim", [2, 3])
def test_constant_modulus_symmetry(dim):
    """P3: with constant moduli and Dirichlet rows eliminated the operator is
    symmetric and negative definite."""
    rng = np.random.default_rng(5)
    bc = ("dirichlet",) * (2 * dim) + ("periodic",) * (6 - 2 * dim)
    p = synth.random_problem(dim, (6, 5, 5)[:dim], bc, "aniso", seed=3)
    p.C = np.broadcast_to(p.C[:, :1, :1, :1], p.C.shape).copy()
    g = _grid(p)
    A = oracle.dense_matrix(g, p.C)
    keep = ~np.broadcast_to(oracle.row_class(g) == oracle.ROW_DIRICHLET, g.shape(dim)).ravel()
    Ai = A[np.ix_(keep, keep)]
    assert np.abs(Ai - Ai.T).max() <= 1e-12 * np.abs(Ai).max()
    assert np.linalg.eigvalsh(0.5 * (Ai + Ai.T)).max() < 0


@pytest.mark.parametrize("dim", [2, 3])
def test_reduces_to_laplacian(dim):
    """P4: isotropic, constant, lambda = -mu: each component's interior row
    is mu times the textbook 5-/7-point Laplacian (built here from 1D second
    difference matrices with Kronecker products)."""
    import scipy.sparse as sps
    mu = 1.7
    bc = ("dirichlet",) * (2 * dim) + ("periodic",) * (6 - 2 * dim)
    p = synth.random_problem(dim, (7, 6, 5)[:dim], bc, "iso", seed=4, lo=(0, 0, 0), hi=(1.0, 0.8, 1.3))
    p.C = np.stack([np.full(p.C.shape[1:], -mu), np.full(p.C.shape[1:], mu)])
    g = _grid(p)
    m, h = p.m, p.h

    def lap1(n, hh):
        return sps.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1]) / hh ** 2

    I = [sps.identity(m[a]) for a in range(3)]
    L = sps.kron(I[2], sps.kron(I[1], lap1(m[0], h[0]))) + sps.kron(I[2], sps.kron(lap1(m[1], h[1]), I[0]))
    if dim == 3:
        L = L + sps.kron(lap1(m[2], h[2]), sps.kron(I[1], I[0]))
    rng = np.random.default_rng(1)
    u = rng.standard_normal(g.shape(dim))
    Au = oracle.apply(g, p.C, u)
    interior = oracle.row_class(g) == oracle.ROW_INTERIOR
    for k in range(dim):
        ref = (mu * (L @ u[k].ravel())).reshape(u[k].shape)
        assert np.abs((Au[k] - ref)[interior]).max() <= 1e-12 * np.abs(ref).max()


def test_stress_free_eigenstrain():
    """P5: constant moduli, uniform eigenstrain E, traction-free faces and
    u = E x on one face: the solution is u = E x and the stress vanishes."""
    p = synth.random_problem(3, (6, 5, 5), ("dirichlet", "traction", "traction", "traction", "traction", "traction"),
                             "aniso", seed=8, with_eps0=False, with_face_data=False)
    p.C = np.broadcast_to(p.C[:, :1, :1, :1], p.C.shape).copy()
    E = np.array([[1.0, 0.3, -0.2], [0.3, -0.5, 0.4], [-0.2, 0.4, 0.7]]) * 1e-3
    shp = (p.m[2], p.m[1], p.m[0])
    p.eps0 = np.stack([np.full(shp, E[k, l]) for k, l in [(0, 0), (1, 1), (2, 2), (1, 2), (2, 0), (0, 1)]])
    x, y, z = p.coords()
    pos = [np.broadcast_to(c, shp) for c in (x, y, z)]
    uex = np.stack([sum(E[k, l] * pos[l] for l in range(3)) for k in range(3)])
    p.face[0] = uex[:, :, :, :1].copy()
    u = oracle.dense_solve(p)
    assert np.abs(u - uex).max() <= 1e-11 * np.abs(uex).max()
    s = oracle.stress(_grid(p), p.C, p.eps0, u)
    assert np.abs(s).max() <= 1e-10 * np.abs(p.C).max() * np.abs(E).max()


def test_iso_equals_aniso_voigt():
    """Isotropic moduli given as (lambda, mu) and as the textbook Voigt
    matrix (C11 = lambda + 2 mu, C12 = lambda, C44 = mu) give the same
    operator, right-hand side and stress."""
    for dim in (2, 3):
        bc = ("traction", "dirichlet", "traction", "traction", "dirichlet", "traction") if dim == 3 else \
            ("traction", "dirichlet", "traction", "traction", "periodic", "periodic")
        p = synth.random_problem(dim, (7, 6, 5)[:dim], bc, "iso", seed=21)
        lam, mu = p.C
        V = np.zeros((6, 6) + lam.shape)
        for I in range(3):
            for J in range(3):
                V[I, J] = lam + (2 * mu if I == J else 0)
        for I in range(3, 6):
            V[I, I] = mu
        q = synth.Problem(**{**p.__dict__})
        q.kind = "aniso"
        if dim == 3:
            q.C = np.stack([V[I, J] for I in range(6) for J in range(I, 6)])
        else:
            sel = [0, 1, 5]
            q.C = np.stack([V[sel[I], sel[J]] for I in range(3) for J in range(I, 3)])
        g, gq = _grid(p), _grid(q)
        rng = np.random.default_rng(2)
        u = rng.standard_normal(g.shape(dim))
        np.testing.assert_allclose(oracle.apply(gq, q.C, u), oracle.apply(g, p.C, u), rtol=0, atol=1e-12 * 1e3)
        np.testing.assert_allclose(oracle.rhs(gq, q.C, q.eps0, q.b, q.face), oracle.rhs(g, p.C, p.eps0, p.b, p.face),
                                   rtol=0, atol=1e-13)
        np.testing.assert_allclose(oracle.stress(gq, q.C, q.eps0, u), oracle.stress(g, p.C, p.eps0, u),
                                   rtol=0, atol=1e-11)


def test_axis_exchange_equivariance():
    """Exchanging the x and y axes (a reflection, under which the stiffness
    transforms as a tensor) maps the operator's output the same way; pins
    the Voigt index map of every shear slot."""
    p = synth.random_problem(3, (6, 6, 5), ("dirichlet", "traction", "traction", "dirichlet", "traction", "traction"),
                             "aniso", seed=31, smooth=False)
    R = np.array([[0.0, 1, 0], [1, 0, 0], [0, 0, 1]])
    nn = p.C.shape[1:]
    Cq = np.empty_like(p.C)
    for iz in range(nn[0]):
        for iy in range(nn[1]):
            for ix in range(nn[2]):
                V = np.zeros((6, 6))
                k = 0
                for I in range(6):
                    for J in range(I, 6):
                        V[I, J] = V[J, I] = p.C[k, iz, iy, ix]
                        k += 1
                Vr = synth.rotate_voigt(V, R)
                Cq[:, iz, ix, iy] = synth.upper21(Vr)        # node (x,y) -> (y,x)
    q = synth.Problem(**{**p.__dict__})
    q.C = Cq
    q.bc = (p.bc[2], p.bc[3], p.bc[0], p.bc[1], p.bc[4], p.bc[5])
    rng = np.random.default_rng(3)
    u = rng.standard_normal((3,) + nn)
    uq = np.stack([u[1], u[0], u[2]]).transpose(0, 1, 3, 2)
    Au = oracle.apply(_grid(p), p.C, u)
    Aq = oracle.apply(_grid(q), q.C, uq)
    ref = np.stack([Au[1], Au[0], Au[2]]).transpose(0, 1, 3, 2)
    assert np.abs(Aq - ref).max() <= 1e-12 * np.abs(ref).max()


def test_diag_is_operator_diagonal():
    """The Jacobi diagonal equals the operator's own diagonal, read off by
    applying it to unit vectors (interior, faces, edges, corners)."""
    for dim, bc in [(3, ("traction", "traction", "traction", "traction", "dirichlet", "traction")),
                    (2, ("traction", "traction", "dirichlet", "traction", "periodic", "periodic")),
                    (3, ("periodic", "periodic", "traction", "traction", "dirichlet", "dirichlet")),
                    (3, ("neumann", "traction", "neumann", "neumann", "dirichlet", "traction")),
                    (2, ("neumann", "traction", "dirichlet", "neumann", "periodic", "periodic"))]:
        p = synth.random_problem(dim, (8, 6, 5)[:dim], bc, "aniso", seed=12, smooth=False)
        g = _grid(p)
        A = oracle.dense_matrix(g, p.C)
        np.testing.assert_allclose(oracle.diag(g, p.C).ravel(), np.diag(A), rtol=1e-13, atol=0)


@pytest.mark.parametrize("case", ["2d", "3d", "3d_periodic", "2d_iso_traction", "3d_neumann", "2d_neumann"])
def test_vcycle_reaches_dense_solution(case):
    """P7: the V-cycle's fixed point is the dense solution; Jacobi leaves the
    exact solution unchanged."""
    if case == "2d":
        p = synth.random_problem(2, (17, 17), ("traction", "traction", "dirichlet", "traction", "periodic", "periodic"),
                                 "aniso", seed=41)
    elif case == "3d":
        p = synth.random_problem(3, (9, 9, 9), ("dirichlet", "traction", "traction", "traction", "traction", "dirichlet"),
                                 "aniso", seed=42)
    elif case == "3d_periodic":
        p = synth.random_problem(3, (9, 9, 9), ("periodic", "periodic", "periodic", "periodic", "dirichlet", "dirichlet"),
                                 "aniso", seed=43)
    elif case == "2d_iso_traction":
        p = synth.random_problem(2, (17, 17), ("dirichlet", "traction", "traction", "traction", "periodic", "periodic"),
                                 "iso", seed=44, with_body=True)
    elif case == "3d_neumann":
        p = synth.random_problem(3, (9, 9, 9), ("neumann", "traction", "periodic", "periodic", "dirichlet", "neumann"),
                                 "aniso", seed=45)
    else:
        p = synth.random_problem(2, (17, 17), ("neumann", "neumann", "dirichlet", "traction", "periodic", "periodic"),
                                 "iso", seed=46, with_body=True)
    ud = oracle.dense_solve(p)
    res = oracle.solve(p, tol=1e-14, max_cycles=300)
    assert np.abs(res.u - ud).max() <= 1e-11 * np.abs(ud).max()
    g = _grid(p)
    f = oracle.rhs(g, p.C, p.eps0, p.b, p.face)
    np.testing.assert_allclose(oracle.jacobi(g, p.C, ud, f, 2.0 / 3.0), ud, rtol=0, atol=1e-10 * np.abs(ud).max())


def test_periodic_translation_invariance():
    """P9: rolling every input by one node along a periodic axis rolls the
    solution."""
    p = synth.random_problem(3, (9, 9, 9), ("periodic", "periodic", "periodic", "periodic", "dirichlet", "dirichlet"),
                             "aniso", seed=51)
    q = synth.Problem(**{**p.__dict__})
    q.C = np.roll(p.C, 1, axis=3)
    q.eps0 = np.roll(p.eps0, 1, axis=3)
    q.face = {f: np.roll(v, 1, axis=3) for f, v in p.face.items()}
    up, uq = oracle.dense_solve(p), oracle.dense_solve(q)
    assert np.abs(np.roll(up, 1, axis=3) - uq).max() <= 1e-11 * np.abs(up).max()


def test_transfers():
    """P8: interpolation reproduces linear fields; full weighting preserves
    constants on every non-Dirichlet coarse row; interior full weighting is
    2^-d times the transpose of interpolation; coarsened moduli of a linear
    field equal the field at the coarse nodes."""
    for dim, bc in [(3, ("traction", "traction", "periodic", "periodic", "dirichlet", "traction")),
                    (2, ("traction", "dirichlet", "traction", "traction", "periodic", "periodic"))]:
        p = synth.random_problem(dim, (9, 8, 9)[:dim] if dim == 3 else (9, 9), bc, "iso", seed=61)
        if dim == 3:
            p = synth.random_problem(3, (9, 9, 9), bc, "iso", seed=61)
        gf = _grid(p)
        gc = gf.coarse()
        rng = np.random.default_rng(0)
        # linear field on the coarse grid, periodic axes constant
        def lin(g):
            h = g.h
            axes = np.meshgrid(*[np.arange(g.m[a]) * h[a] for a in (2, 1, 0)], indexing="ij")
            coef = [0.0 if g.periodic(a) or a >= dim else rng.uniform(-1, 1) for a in range(3)]
            return lambda c: sum(c[a] * axes[2 - a] for a in range(3))
        coef = [0.0 if gf.periodic(a) or a >= dim else float(a + 1) for a in range(3)]
        def linf(g):
            axes = np.meshgrid(*[np.arange(g.m[a]) * g.h[a] for a in (2, 1, 0)], indexing="ij")
            return sum(coef[a] * axes[2 - a] for a in range(3)) + 0.5
        ec = np.stack([linf(gc)] * dim)
        uf = oracle.prolong_add(gc, gf, ec, np.zeros(gf.shape(dim)))
        nd = np.broadcast_to(oracle.row_class(gf) != oracle.ROW_DIRICHLET, uf.shape)
        ref = np.stack([linf(gf)] * dim)
        assert np.abs((uf - ref)[nd]).max() <= 1e-14
        ones = np.ones(gf.shape(dim))
        fc = oracle.restrict(gf, gc, ones)
        ndc = np.broadcast_to(oracle.row_class(gc) != oracle.ROW_DIRICHLET, fc.shape)
        assert np.abs(fc[ndc] - 1.0).max() <= 1e-15
        # coarse moduli of a linear field
        Cf = np.stack([linf(gf), linf(gf) + 1.0])
        Cc = oracle.coarsen_moduli(gf, gc, Cf)
        np.testing.assert_allclose(Cc, np.stack([linf(gc), linf(gc) + 1.0]), rtol=0, atol=1e-14)
        # interior rows: R = 2^-d P^T
        nF, nC = dim * gf.N, dim * gc.N
        P = np.empty((nF, nC))
        e = np.zeros(nC)
        for q in range(nC):
            e[q] = 1.0
            P[:, q] = oracle.prolong_add(gc, gf, e.reshape(gc.shape(dim)), np.zeros(gf.shape(dim))).ravel()
            e[q] = 0.0
        Rm = np.empty((nC, nF))
        e = np.zeros(nF)
        for q in range(nF):
            e[q] = 1.0
            Rm[:, q] = oracle.restrict(gf, gc, e.reshape(gf.shape(dim))).ravel()
            e[q] = 0.0
        ci = np.broadcast_to(oracle.row_class(gc) == oracle.ROW_INTERIOR, gc.shape(dim)).ravel()
        np.testing.assert_allclose(Rm[ci], (2.0 ** -dim) * P.T[ci], rtol=0, atol=1e-15)


def _disc_problem(n, L, a, w):
    """Plane-strain disc of radius a with dilatational in-plane eigenstrain in
    an isotropic matrix, on [-L, L]^2 with the exact far field imposed on
    every face."""
    lam_m, mu_m, lam_i, mu_i, es = 1.5, 1.0, 3.0, 2.0, 1e-3
    p = synth.Problem(dim=2, n=(n, n, 1), lo=(-L, -L, 0.0), hi=(L, L, 0.0), bc=("dirichlet",) * 4 + ("periodic",) * 2,
                      kind="iso", C=np.zeros(0))
    x, y, _ = p.coords()
    r = np.sqrt(x ** 2 + y ** 2)
    eta = 0.5 * (1 - np.tanh((r - a) / w))
    p.C = np.stack([lam_m + (lam_i - lam_m) * eta, mu_m + (mu_i - mu_m) * eta])
    p.eps0 = np.stack([es * eta, es * eta, 0 * eta])
    A = (lam_i + mu_i) * es / (lam_i + mu_i + mu_m)          # u = A x inside, A a^2 x / r^2 outside
    fac = np.where(r <= a, A, A * a * a / np.maximum(r, a) ** 2)
    uex = np.stack([fac * x, fac * y])
    for f in range(4):
        ax = f // 2
        sl = [slice(None)] * 3
        sl[2 - ax] = slice(0, 1) if f % 2 == 0 else slice(n - 1, n)
        p.face[f] = uex[(slice(None),) + tuple(sl)].copy()
    return p, uex, r


@pytest.mark.slow
def test_eshelby_disc_closed_form():
    """P6: the diffuse-interface solution approaches the sharp-interface
    closed form (u = A x inside, A a^2 x / r^2 outside,
    A = (lambda_i + mu_i) eps* / (lambda_i + mu_i + mu_m)) as h and the
    interface width shrink together; measured away from the interface."""
    errs = []
    for n in (65, 129):
        L, a = 2.0, 0.5
        h = 2 * L / (n - 1)
        p, uex, r = _disc_problem(n, L, a, 2 * h)
        res = oracle.solve(p, tol=1e-10, max_cycles=200)
        far = np.broadcast_to(np.abs(r - a) > 0.25, uex.shape)
        errs.append(np.abs(res.u - uex)[far].max() / np.abs(uex).max())
    assert errs[1] < 0.6 * errs[0]
    assert errs[1] < 0.03


# --------------------------------------------------------------------------
# F-cycle (Sec. 3.1: the paper's solver runs F-cycles)
# --------------------------------------------------------------------------

def _tiny_3level():
    """2D problem whose hierarchy has exactly three levels (17 -> 9 -> 5)."""
    p = synth.random_problem(2, (17, 17), ("neumann", "traction", "dirichlet", "traction", "periodic", "periodic"),
                             "aniso", seed=61)
    H = oracle.Hierarchy(_grid(p), p.C)
    assert len(H.grids) == 3
    return p, H


def _dense_of(fn, n_in, shape_in):
    """Matrix of a linear map given as a function of an array, by unit vectors."""
    cols = []
    e = np.zeros(n_in)
    for q in range(n_in):
        e[q] = 1.0
        cols.append(np.asarray(fn(e.reshape(shape_in))).ravel())
        e[q] = 0.0
    return np.array(cols).T


def test_fcycle_equals_vcycle_on_two_levels():
    """With two levels the coarse F-cycle is the exact coarse solve and the
    V-cycle after it solves the same coarse system again, so an F-cycle is a
    V-cycle bit for bit."""
    p = synth.random_problem(2, (9, 9), ("traction", "traction", "dirichlet", "neumann", "periodic", "periodic"),
                             "iso", seed=62)
    g = _grid(p)
    H = oracle.Hierarchy(g, p.C)
    assert len(H.grids) == 2
    f = oracle.rhs(g, p.C, p.eps0, p.b, p.face)
    x = np.random.default_rng(3).standard_normal(g.shape(2))
    np.testing.assert_array_equal(oracle.fcycle(H, 0, x, f), oracle.vcycle(H, 0, x, f))


def test_fcycle_sweep_counts():
    """Level k (0 = finest, above the bottom) is visited k + 1 times per
    F-cycle (the F-cycle on level l adds one visit of level l to the visits
    of F and V on level l + 1); each visit runs nu1 + nu2 sweeps.  A V-cycle
    visits each level once."""
    p = synth.random_problem(2, (65, 65), ("dirichlet", "traction", "traction", "traction", "periodic", "periodic"),
                             "iso", seed=63)
    g = _grid(p)
    H = oracle.Hierarchy(g, p.C)
    L = len(H.grids)
    assert L >= 4
    f = oracle.rhs(g, p.C, p.eps0, p.b, p.face)
    for nu1, nu2 in ((2, 2), (1, 3)):
        cf, cv = [0] * L, [0] * L
        oracle.fcycle(H, 0, np.zeros(g.shape(2)), f, nu1, nu2, counts=cf)
        oracle.vcycle(H, 0, np.zeros(g.shape(2)), f, nu1, nu2, counts=cv)
        assert cf[:-1] == [(k + 1) * (nu1 + nu2) for k in range(L - 1)]
        assert cv[:-1] == [nu1 + nu2] * (L - 1)


def test_fcycle_without_smoothing_matches_matrix_form():
    """With no smoothing, a 3-level F-cycle from zero is x = P01 (B + B (I -
    A1 B)) R10 f with B = P12 A2^-1 R21: the coarse F-cycle gives B f1 and
    the V-cycle from it adds the coarse correction of its residual.  The
    transfer and operator matrices are read off the oracle's primitives by
    unit vectors; the composition is the textbook one."""
    p, H = _tiny_3level()
    g0, g1, g2 = H.grids
    d = 2
    A1 = oracle.dense_matrix(g1, H.C[1])
    A2 = oracle.dense_matrix(g2, H.C[2])
    R10 = _dense_of(lambda r: oracle.restrict(g0, g1, r), d * g0.N, g0.shape(d))
    R21 = _dense_of(lambda r: oracle.restrict(g1, g2, r), d * g1.N, g1.shape(d))
    P01 = _dense_of(lambda e: oracle.prolong_add(g1, g0, e, np.zeros(g0.shape(d))), d * g1.N, g1.shape(d))
    P12 = _dense_of(lambda e: oracle.prolong_add(g2, g1, e, np.zeros(g1.shape(d))), d * g2.N, g2.shape(d))
    B = P12 @ np.linalg.solve(A2, R21)
    M = P01 @ (B + B @ (np.eye(B.shape[0]) - A1 @ B)) @ R10
    f = np.random.default_rng(5).standard_normal(d * g0.N)
    got = oracle.fcycle(H, 0, np.zeros(g0.shape(d)), f.reshape(g0.shape(d)), 0, 0).ravel()
    ref = M @ f
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # and the V-cycle without smoothing is P01 B R10 f
    gotv = oracle.vcycle(H, 0, np.zeros(g0.shape(d)), f.reshape(g0.shape(d)), 0, 0).ravel()
    refv = P01 @ B @ R10 @ f
    assert np.abs(gotv - refv).max() <= 1e-12 * np.abs(refv).max()


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_fcycle_reaches_dense_solution(case):
    """The F-cycle's fixed point is the dense solution."""
    if case == "2d":
        p, _ = _tiny_3level()
    else:
        p = synth.random_problem(3, (9, 9, 9), ("dirichlet", "neumann", "traction", "traction", "periodic", "periodic"),
                                 "aniso", seed=64)
    ud = oracle.dense_solve(p)
    res = oracle.solve(p, tol=1e-14, max_cycles=300, cycle="F")
    assert np.abs(res.u - ud).max() <= 1e-11 * np.abs(ud).max()


# --------------------------------------------------------------------------
# von Mises stress (Sec. 4.3)
# --------------------------------------------------------------------------

def test_von_mises_closed_forms():
    """Uniaxial stress s gives |s|; pure shear t gives sqrt(3)|t|; a
    hydrostatic state gives 0; equal and opposite normal stresses s, -s give
    sqrt(3)|s|; the value is invariant under rotations of the stress."""
    z = np.zeros(1)
    def voigt(s11=0.0, s22=0.0, s33=0.0, s23=0.0, s31=0.0, s12=0.0):
        return np.array([[s11], [s22], [s33], [s23], [s31], [s12]])
    assert np.isclose(oracle.von_mises(voigt(s11=2.5))[0], 2.5, rtol=1e-15)
    assert np.isclose(oracle.von_mises(voigt(s22=-1.5))[0], 1.5, rtol=1e-15)
    for comp in ("s23", "s31", "s12"):
        assert np.isclose(oracle.von_mises(voigt(**{comp: 0.7}))[0], np.sqrt(3) * 0.7, rtol=1e-15)
    assert abs(oracle.von_mises(voigt(s11=3.0, s22=3.0, s33=3.0))[0]) <= 1e-15
    assert np.isclose(oracle.von_mises(voigt(s11=1.2, s22=-1.2))[0], np.sqrt(3) * 1.2, rtol=1e-15)
    rng = np.random.default_rng(9)
    A = rng.standard_normal((3, 3)); T = A + A.T
    R = synth.shoemake_rotation(rng.random(3))
    TR = R @ T @ R.T
    v = lambda M: np.array([[M[0, 0]], [M[1, 1]], [M[2, 2]], [M[1, 2]], [M[2, 0]], [M[0, 1]]])
    assert np.isclose(oracle.von_mises(v(T))[0], oracle.von_mises(v(TR))[0], rtol=1e-13)
    # the second invariant form: sqrt(1/2 [(s1-s2)^2 + (s2-s3)^2 + (s3-s1)^2]) with principal stresses
    w = np.linalg.eigvalsh(T)
    ref = np.sqrt(0.5 * ((w[0] - w[1]) ** 2 + (w[1] - w[2]) ** 2 + (w[2] - w[0]) ** 2))
    assert np.isclose(oracle.von_mises(v(T))[0], ref, rtol=1e-13)


# --------------------------------------------------------------------------
# Eshelby tensor of an ellipsoid (Sec. 4.1 verification problem)
# --------------------------------------------------------------------------

def test_eshelby_tensor_sphere_values():
    """A sphere gives the textbook values S_1111 = (7-5nu)/(15(1-nu)),
    S_1122 = (5nu-1)/(15(1-nu)), S_1212 = (4-5nu)/(15(1-nu)), the same on
    every axis, and S_1123 = 0."""
    from oracle import eshelby
    for nu in (0.0, 0.25, 0.3, 0.45):
        S = eshelby.eshelby_tensor([0.7, 0.7, 0.7], nu)
        d = 15.0 * (1.0 - nu)
        for i in range(3):
            assert np.isclose(S[i, i, i, i], (7 - 5 * nu) / d, rtol=1e-12, atol=0)
            for j in range(3):
                if j != i:
                    assert np.isclose(S[i, i, j, j], (5 * nu - 1) / d, rtol=1e-11, atol=1e-14)
                    assert np.isclose(S[i, j, i, j], (4 - 5 * nu) / d, rtol=1e-12, atol=0)
                    assert S[i, j, i, j] == S[j, i, i, j]
        assert S[0, 0, 1, 2] == 0.0 and S[0, 1, 2, 2] == 0.0


def test_eshelby_tensor_elliptic_cylinder_limit():
    """a3 -> infinity gives the elliptic cylinder's closed form (semi-axes
    a1, a2 in the cross-section): S_1111 = [(a2^2 + 2 a1 a2)/(a1+a2)^2 +
    (1-2nu) a2/(a1+a2)] / (2(1-nu)), S_1122 = [a2^2/(a1+a2)^2 - (1-2nu)
    a2/(a1+a2)] / (2(1-nu)), S_1212 = [(a1^2+a2^2)/(2(a1+a2)^2) +
    (1-2nu)/2] / (2(1-nu)), S_1133 = nu a2 / ((1-nu)(a1+a2)), S_33kk = 0."""
    from oracle import eshelby
    nu, a1, a2 = 0.3, 1.0, 0.6
    S = eshelby.eshelby_tensor([a1, a2, 1e6], nu)
    k, s = 1.0 / (2.0 * (1.0 - nu)), a1 + a2
    assert np.isclose(S[0, 0, 0, 0], k * ((a2 ** 2 + 2 * a1 * a2) / s ** 2 + (1 - 2 * nu) * a2 / s), rtol=1e-8)
    assert np.isclose(S[1, 1, 1, 1], k * ((a1 ** 2 + 2 * a1 * a2) / s ** 2 + (1 - 2 * nu) * a1 / s), rtol=1e-8)
    assert np.isclose(S[0, 0, 1, 1], k * (a2 ** 2 / s ** 2 - (1 - 2 * nu) * a2 / s), rtol=1e-7)
    assert np.isclose(S[1, 1, 0, 0], k * (a1 ** 2 / s ** 2 - (1 - 2 * nu) * a1 / s), rtol=1e-7)
    assert np.isclose(S[0, 1, 0, 1], k * ((a1 ** 2 + a2 ** 2) / (2 * s ** 2) + (1 - 2 * nu) / 2), rtol=1e-8)
    assert np.isclose(S[0, 0, 2, 2], nu * a2 / ((1 - nu) * s), rtol=1e-8)
    assert np.isclose(S[1, 1, 2, 2], nu * a1 / ((1 - nu) * s), rtol=1e-8)
    assert abs(S[2, 2, 2, 2]) < 1e-8 and abs(S[2, 2, 0, 0]) < 1e-8


def test_eshelby_potential_integrals_prolate_and_identities():
    """Prolate spheroid a1 > a2 = a3: I_2 = I_3 = 2 pi a1 a3^2 /
    (a1^2 - a3^2)^(3/2) [(a1/a3)(a1^2/a3^2 - 1)^(1/2) - arccosh(a1/a3)],
    I_1 = 4 pi - 2 I_2.  Any ellipsoid: I_1 + I_2 + I_3 = 4 pi,
    3 I_11 + I_12 + I_13 = 4 pi / a1^2, and the dilatation inside for a
    dilatational eigenstrain does not depend on the shape:
    S_iikk = (1+nu)/(1-nu)."""
    from oracle import eshelby
    a1, a3 = 2.0, 0.8
    I, II = eshelby.potential_integrals([a1, a3, a3])
    I2 = 2 * np.pi * a1 * a3 ** 2 / (a1 ** 2 - a3 ** 2) ** 1.5 * (
        (a1 / a3) * np.sqrt(a1 ** 2 / a3 ** 2 - 1) - np.arccosh(a1 / a3))
    assert np.isclose(I[1], I2, rtol=1e-12) and np.isclose(I[2], I2, rtol=1e-12)
    assert np.isclose(I[0], 4 * np.pi - 2 * I2, rtol=1e-12)
    for a in ([1.0, 0.75, 0.5], [0.3, 1.7, 0.9]):
        I, II = eshelby.potential_integrals(a)
        assert np.isclose(I.sum(), 4 * np.pi, rtol=1e-12)
        for i in range(3):
            assert np.isclose(3 * II[i, i] + sum(II[i, j] for j in range(3) if j != i), 4 * np.pi / a[i] ** 2,
                              rtol=1e-11)
        for nu in (0.2, 0.3):
            S = eshelby.eshelby_tensor(a, nu)
            assert np.isclose(np.einsum("iikk", S), (1 + nu) / (1 - nu), rtol=1e-12)
