"""Full-size checks of the benchmark's workloads (129^3 and 257^3
polycrystals, the three-level penny-crack AMR problem on a 65^3 base),
through the same C ABI calls and launch configuration as bench.py.

At these sizes the oracle cannot run whole solves in seconds, so it checks:
  * one operator application / residual / Jacobi sweep of the finest level,
    element by element, on a random field (129^3 polycrystal; 257^3
    polycrystal with the sphere);
  * the GPU solutions of FP64 and mixed-precision solves through the
    oracle's own residual: relative residual <= 1.2e-10 (stopping test
    1e-10 plus the rounding of the recomputation), and the mixed solution
    within 1e-8 (relative 2-norm) of a FP64 solution iterated to 1e-13 whose
    oracle residual is itself checked (129^3 polycrystal; 257^3 polycrystal
    with a stiff eigenstrained sphere);
  * the composite residual of the three-level AMR solve on the 65^3 base
    (reading of floor and width as in synth.penny_crack).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import amr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


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


def rel_norm(g, u, f, C):
    """Oracle relative residual of u (reference: the Dirichlet lift)."""
    lift = np.where(oracle.dirichlet_mask(g), f, 0.0)
    r0 = oracle.norm(g, oracle.residual(g, C, lift, f))
    return oracle.norm(g, oracle.residual(g, C, u, f)) / r0


def check_solves(emg, ctx, spec, label):
    g = oracle.Grid.of(spec)
    print(f"[gpu] {label}: oracle rhs", flush=True)
    f = oracle.rhs(g, spec.C, spec.eps0, spec.b, spec.face)
    prob = emg.Problem.from_spec(ctx, spec)
    assert np.abs(prob.rhs() - f).max() <= 1e-12 * np.abs(f).max()
    st_ref = prob.solve(rtol=1e-13, max_cycles=400, precision="fp64", raise_on_error=False)
    u_ref = prob.displacement()
    rel_ref = rel_norm(g, u_ref, f, spec.C)
    print(f"[gpu] {label}: reference cycles={st_ref['cycles']} oracle rel residual={rel_ref:.2e}", flush=True)
    assert rel_ref <= 1e-12
    out = {}
    for prec in ("fp64", "mixed"):
        st = prob.solve(rtol=1e-10, max_cycles=400, precision=prec)
        u = prob.displacement()
        rel = rel_norm(g, u, f, spec.C)
        err = float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))
        print(f"[gpu] {label}: {prec} cycles={st['cycles']} oracle rel residual={rel:.2e} "
              f"error vs FP64 reference={err:.2e}", flush=True)
        assert st["converged"] and rel <= 1.2e-10
        assert err <= 1e-8
        out[prec] = (st, u)
    prob.close()
    return out


@pytest.mark.parametrize("n", [129, 257])
def test_polycrystal_finest_level_steps(emg, ctx, n):
    """Finest-level operator, residual and Jacobi sweep (z-marching columns
    and boundary shell, in the launch configuration the bench times: 4
    chunks per column at 129^3, one 255-plane chunk at 257^3) against the
    oracle, element by element, in FP64 and FP32: the 129^3 polycrystal and
    the 257^3 polycrystal with the stiff eigenstrained sphere."""
    if n == 129:
        spec = synth.polycrystal_3d(n=129, grains=16, seed=2002)
    else:
        print("[gpu] generating the 257^3 polycrystal with a sphere", flush=True)
        spec = synth.polycrystal_3d(n=257, grains=64, seed=2003, inclusion=(3.0, 2e-3))
    g = oracle.Grid.of(spec)
    prob = emg.Problem.from_spec(ctx, spec)
    assert prob.level_zmarch(0, "fp64") == (4 if n == 129 else 1)
    rng = np.random.default_rng(11)
    u = 1e-3 * rng.standard_normal(g.shape(3))
    f = rng.standard_normal(g.shape(3))
    print(f"[gpu] {n}^3 polycrystal level steps: oracle", flush=True)
    ref = {"apply": oracle.apply(g, spec.C, u), "residual": oracle.residual(g, spec.C, u, f),
           "jacobi": oracle.jacobi(g, spec.C, u, f, 2.0 / 3.0)}
    for prec, dt, tol in (("fp64", torch.float64, 1e-12), ("mixed", torch.float32, 2e-5)):
        ud = torch.from_numpy(u).to(DEV, dtype=dt)
        fd = torch.from_numpy(f).to(DEV, dtype=dt)
        out = torch.empty_like(ud)
        for step in ("apply", "residual", "jacobi"):
            if step == "apply":
                prob.level_apply(0, ud, out, precision=prec)
            elif step == "residual":
                prob.level_residual(0, ud, fd, out, precision=prec)
            else:
                prob.level_jacobi(0, ud, fd, out, precision=prec)
            got = out.to("cpu", dtype=torch.float64).numpy()
            err = np.abs(got - ref[step]).max() / np.abs(ref[step]).max()
            print(f"[gpu]   {prec} {step}: max rel error {err:.2e}", flush=True)
            assert err <= tol, (prec, step)
    prob.close()


def test_polycrystal129_solves_full_size(emg, ctx):
    spec = synth.polycrystal_3d(n=129, grains=16, seed=2002)
    res = check_solves(emg, ctx, spec, "129^3 polycrystal")
    assert res["mixed"][0]["cycles"] == res["fp64"][0]["cycles"]


def test_polycrystal257_sphere_solves_full_size(emg, ctx):
    """257^3, 64 grains, stiff eigenstrained sphere: FP32 V-cycles inside
    FP64 refinement against plain FP64, both checked by the oracle."""
    print("[gpu] generating the 257^3 polycrystal with a sphere", flush=True)
    spec = synth.polycrystal_3d(n=257, grains=64, seed=2003, inclusion=(3.0, 2e-3))
    check_solves(emg, ctx, spec, "257^3 polycrystal + sphere")


def test_penny_crack_amr_65_full_size(emg, ctx):
    """The penny crack as benchmarked: 65^3 base, three levels of 16/32-cell
    blocks (40 and 80 boxes) tagged where |grad eta| h > 0.1, diffuse width
    0.01, moduli capped at 1 % inside the crack; FP64 and mixed precision:
    each GPU composite solution satisfies the oracle's composite system to
    1.2e-10; the mixed solution's error against the FP64 one is reported and
    held to 1e-8."""
    ap = synth.penny_crack(n=65, levels=3, floor=1e-2, width=0.01)
    assert [len(ap.level_boxes(k)) for k in (1, 2)] == [40, 80]
    print(f"[gpu] penny crack, 65^3 base: {ap.composite_nodes()} composite nodes", flush=True)
    comp = amr.from_problem(ap)
    r0 = comp.norm(comp.residual(comp.initial()))
    sols = {}
    for precision in ("fp64", "mixed"):
        prob = emg.Problem.from_amr(ctx, ap)
        st = prob.solve(rtol=1e-10, max_cycles=400, precision=precision)
        assert st["converged"]
        u = [prob.displacement()] + [prob.amr_displacement(k) for k in range(1, len(ap.boxes) + 1)]
        prob.close()
        rel = comp.norm(comp.residual(u)) / r0
        print(f"[gpu]   {precision}: cycles={st['cycles']} solve {1e3 * st['solve_seconds']:.1f} ms "
              f"oracle composite rel residual={rel:.2e}", flush=True)
        assert rel <= 1.2e-10
        sols[precision] = u
    num = sum(float(np.sum((a - b) ** 2)) for a, b in zip(sols["mixed"], sols["fp64"]))
    den = sum(float(np.sum(b ** 2)) for b in sols["fp64"])
    diff = np.sqrt(num / den)
    print(f"[gpu]   mixed vs FP64 rel diff {diff:.2e}", flush=True)
    assert diff <= 1e-8
