"""Mixed-precision refinement with several FP32 cycles per FP64 step
(emg_solve_opts.inner_cycles): each step computes one FP64 residual, runs
inner_cycles FP32 cycles on it (the later ones continuing from the
correction) and applies the correction once.  The solution must meet the
same bar as with one cycle per step: relative residual 1e-10 and within
1e-8 of the oracle's (small cases) or of the FP64 GPU solution (a 97^3
polycrystal on the z-marching pass); the cycle count is a multiple of
inner_cycles and close to the one-cycle count, since the FP32 cycles
contract the error as FP64 ones do until FP32 rounding (~1e-7 of the
correction) is reached."""
import numpy as np
import pytest

import oracle
import synth

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


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def check_inner(prob, inner, one):
    st = prob.solve(rtol=1e-10, max_cycles=400, precision="mixed", inner_cycles=inner)
    assert st["converged"] and st["rel_res"] <= 1e-10 and st["fp64_fallback"] == 0
    assert st["cycles"] % inner == 0
    assert one - inner <= st["cycles"] <= one + 2 * inner, (st["cycles"], one)
    return st


@pytest.mark.parametrize("inner", [2, 3])
@pytest.mark.parametrize("case", ["poly17", "incl2d"])
def test_inner_cycles_match_oracle(emg, ctx, case, inner):
    spec = synth.polycrystal_3d(n=17, grains=8, seed=11) if case == "poly17" else synth.inclusion_2d(n=65)
    print(f"[gpu] inner {case} {inner}", flush=True)
    ref = oracle.solve(spec, tol=1e-13, max_cycles=400)
    prob = emg.Problem.from_spec(ctx, spec)
    one = prob.solve(rtol=1e-10, max_cycles=400, precision="mixed")["cycles"]
    check_inner(prob, inner, one)
    u = prob.displacement()
    assert rel(u, ref.u) <= 1e-8
    # eager launches give the graph's result bit for bit
    prob.solve(rtol=1e-10, max_cycles=400, precision="mixed", inner_cycles=inner, use_graph=0)
    assert np.array_equal(prob.displacement(), u)
    prob.close()


def test_inner_cycles_zmarch_polycrystal(emg, ctx):
    spec = synth.polycrystal_3d(n=97, grains=16, seed=5)
    prob = emg.Problem.from_spec(ctx, spec)
    assert prob.level_zmarch(0, "fp64") > 0 and prob.level_zmarch(0, "mixed") > 0
    print("[gpu] inner 97^3", flush=True)
    prob.solve(rtol=1e-13, max_cycles=400, precision="fp64")
    u64 = prob.displacement()
    one = prob.solve(rtol=1e-10, max_cycles=400, precision="mixed")["cycles"]
    st = check_inner(prob, 2, one)
    assert rel(prob.displacement(), u64) <= 1e-8
    # a cap below the converged count stops at a whole step
    st = prob.solve(rtol=1e-10, max_cycles=9, precision="mixed", inner_cycles=2, raise_on_error=False)
    assert st["status"] == emg.EMG_ENOTCONV and st["cycles"] == 10
    prob.close()


def test_inner_cycles_rejected(emg, ctx):
    spec = synth.polycrystal_3d(n=17, grains=8, seed=11)
    prob = emg.Problem.from_spec(ctx, spec)
    for kw in (dict(precision="fp64", inner_cycles=2), dict(precision="mixed", inner_cycles=0),
               dict(precision="mixed", inner_cycles=5)):
        with pytest.raises(emg.EmgError):
            prob.solve(rtol=1e-10, **kw)
    with pytest.raises(emg.EmgError):
        emg.solve_batch([prob], rtol=1e-10, precision="fp64", inner_cycles=2)
    prob.close()


def test_inner_cycles_batch_bitwise_equals_solo(emg, ctx):
    """A ragged batch with two FP32 cycles per step gives every member the
    displacement and cycle count of its own emg_solve, bit for bit."""
    specs = [synth.polycrystal_3d(n=17, grains=8, seed=11), synth.inclusion_3d(n=33, seed=3),
             synth.inclusion_2d(n=65)]
    solo = []
    for sp in specs:
        p = emg.Problem.from_spec(ctx, sp)
        st = p.solve(rtol=1e-10, max_cycles=400, precision="mixed", inner_cycles=2)
        solo.append((st["cycles"], p.displacement()))
        p.close()
    print("[gpu] inner batch", flush=True)
    probs = [emg.Problem.from_spec(ctx, sp) for sp in specs]
    stats = emg.solve_batch(probs, rtol=1e-10, max_cycles=400, precision="mixed", inner_cycles=2)
    for sp, p, st, (c, u) in zip(specs, probs, stats, solo):
        assert st["converged"] and st["rel_res"] <= 1e-10 and st["cycles"] % 2 == 0, sp.name
        assert st["cycles"] == c, (sp.name, st["cycles"], c)
        assert np.array_equal(p.displacement(), u), sp.name
    for p in probs:
        p.close()


def test_inner_cycles_stall_fallback_keeps_cycle_cap(emg, ctx):
    """A forced stall with two FP32 cycles per step: the solve switches to
    FP64 cycles, still reaches 1e-10 with the FP64 solution, and the cap of
    max_cycles counts V-cycles (steps before the fallback count
    inner_cycles each, FP64 cycles one each)."""
    spec = synth.polycrystal_3d(n=17, grains=8, seed=11)
    prob = emg.Problem.from_spec(ctx, spec)
    ref = prob.solve(rtol=1e-10, max_cycles=400, precision="fp64")
    uref = prob.displacement()
    print("[gpu] inner 2 stall fallback", flush=True)
    for use_graph in (1, 0):
        st = prob.solve(rtol=1e-10, max_cycles=400, precision="mixed", inner_cycles=2, check_every=4,
                        stall_iters=4, stall_factor=1e-30, use_graph=use_graph)
        assert st["converged"] and st["fp64_fallback"] == 1 and st["rel_res"] <= 1e-10
        assert rel(prob.displacement(), uref) <= 1e-8
        assert st["cycles"] <= ref["cycles"] + 8
    # a cap that the FP64 cycles after the fallback cannot meet: the solve
    # stops at exactly max_cycles V-cycles (8 steps x 2 before the fallback)
    cap = 30
    st = prob.solve(rtol=1e-14, max_cycles=cap, precision="mixed", inner_cycles=2, check_every=4, stall_iters=4,
                    stall_factor=1e-30, raise_on_error=False)
    assert st["status"] == emg.EMG_ENOTCONV and st["fp64_fallback"] == 1
    assert st["cycles"] == cap, st["cycles"]
    prob.close()


@pytest.mark.parametrize("nu", [(2, 1), (1, 2)])
def test_inner_cycles_odd_sweep_count(emg, ctx, nu):
    """nu1 + nu2 odd: every continuing FP32 cycle leaves the correction in
    the other ping-pong buffer and the step moves it back.  Graph, eager and
    batched solves agree bit for bit, and match the FP64 solution."""
    nu1, nu2 = nu
    spec = synth.polycrystal_3d(n=17, grains=8, seed=11)
    prob = emg.Problem.from_spec(ctx, spec)
    prob.solve(rtol=1e-13, max_cycles=400, precision="fp64", nu1=nu1, nu2=nu2)
    u64 = prob.displacement()
    print(f"[gpu] inner 2 V({nu1},{nu2})", flush=True)
    st = prob.solve(rtol=1e-10, max_cycles=400, precision="mixed", inner_cycles=2, nu1=nu1, nu2=nu2)
    assert st["converged"] and st["rel_res"] <= 1e-10
    u = prob.displacement()
    assert rel(u, u64) <= 1e-8
    st_e = prob.solve(rtol=1e-10, max_cycles=400, precision="mixed", inner_cycles=2, nu1=nu1, nu2=nu2, use_graph=0)
    assert st_e["cycles"] == st["cycles"] and np.array_equal(prob.displacement(), u)
    prob.close()
    probs = [emg.Problem.from_spec(ctx, spec), emg.Problem.from_spec(ctx, synth.inclusion_2d(n=33))]
    stats = emg.solve_batch(probs, rtol=1e-10, max_cycles=400, precision="mixed", inner_cycles=2, nu1=nu1, nu2=nu2)
    assert stats[0]["cycles"] == st["cycles"] and np.array_equal(probs[0].displacement(), u)
    for p in probs:
        p.close()


def test_inner_cycles_batch_bitwise_zmarch(emg, ctx):
    """Batch against solo, bit for bit, with a member whose finest level
    runs the z-marching pass in both precisions (97^3 polycrystal) beside a
    small one, two FP32 cycles per step."""
    specs = [synth.polycrystal_3d(n=97, grains=16, seed=5), synth.polycrystal_3d(n=17, grains=8, seed=11)]
    solo = []
    for sp in specs:
        p = emg.Problem.from_spec(ctx, sp)
        if sp.n[0] == 97:
            assert p.level_zmarch(0, "fp64") > 0 and p.level_zmarch(0, "mixed") > 0
        st = p.solve(rtol=1e-10, max_cycles=400, precision="mixed", inner_cycles=2)
        solo.append((st["cycles"], p.displacement()))
        p.close()
    print("[gpu] inner batch z-march", flush=True)
    probs = [emg.Problem.from_spec(ctx, sp) for sp in specs]
    stats = emg.solve_batch(probs, rtol=1e-10, max_cycles=400, precision="mixed", inner_cycles=2)
    for sp, p, st, (c, u) in zip(specs, probs, stats, solo):
        assert st["converged"] and st["cycles"] == c, (sp.name, st["cycles"], c)
        assert np.array_equal(p.displacement(), u), sp.name
    for p in probs:
        p.close()
