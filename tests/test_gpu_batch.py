"""Ragged batches: problems of different sizes, dimensions and moduli kinds
solved together through emg_solve_batch give, bit for bit, the result each
gives alone (same cycles), in FP64 and mixed precision."""
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


def _mix():
    return [synth.polycrystal_3d(n=17, grains=8, seed=11),
            synth.inclusion_3d(n=33, seed=3),
            synth.polycrystal_3d(n=33, grains=12, seed=12),
            synth.inclusion_3d(n=17, seed=4),
            synth.inclusion_2d(n=65),
            synth.random_problem(2, (65, 33), ("dirichlet", "dirichlet", "traction", "traction", "periodic",
                                               "periodic"), "aniso", seed=10, with_body=True)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_bitwise_equals_solo(emg, ctx, precision):
    specs = _mix()
    print(f"[gpu] batch of {len(specs)} {precision}", flush=True)
    solo = []
    for sp in specs:
        p = emg.Problem.from_spec(ctx, sp)
        st = p.solve(rtol=1e-10, max_cycles=400, precision=precision)
        solo.append((st["cycles"], p.displacement()))
        p.close()
    probs = [emg.Problem.from_spec(ctx, sp) for sp in specs]
    stats = emg.solve_batch(probs, rtol=1e-10, max_cycles=400, precision=precision, check_every=3)
    for sp, p, st, (c, u) in zip(specs, probs, stats, solo):
        assert st["converged"] and st["rel_res"] <= 1e-10, sp.name
        assert st["cycles"] == c, (sp.name, st["cycles"], c)
        assert np.array_equal(p.displacement(), u), sp.name
    for p in probs:
        p.close()


def test_batch_member_matches_oracle(emg, ctx):
    specs = _mix()[:4]
    probs = [emg.Problem.from_spec(ctx, sp) for sp in specs]
    emg.solve_batch(probs, rtol=1e-10, max_cycles=400, precision="mixed")
    ref = oracle.solve(specs[0], tol=1e-13, max_cycles=400)
    u = probs[0].displacement()
    assert np.linalg.norm(u - ref.u) / np.linalg.norm(ref.u) <= 1e-8
    for p in probs:
        p.close()


def test_batch_eager_equals_graph(emg, ctx):
    specs = _mix()[:3]
    res = []
    for g in (1, 0):
        probs = [emg.Problem.from_spec(ctx, sp) for sp in specs]
        emg.solve_batch(probs, rtol=1e-10, use_graph=g)
        res.append([p.displacement() for p in probs])
        for p in probs:
            p.close()
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_batch_rejects_duplicates(emg, ctx):
    p = emg.Problem.from_spec(ctx, synth.inclusion_3d(n=17))
    with pytest.raises(emg.EmgError) as ei:
        emg.solve_batch([p, p])
    assert ei.value.status == emg.EMG_EINVAL
    p.close()
