"""Fused coarse tail (k_tail): the cycle on a problem's coarsest levels runs
as one launch of one workgroup per problem when the tuning table asks for it
(off by default: slower on this GPU).  Solves with the tail (forced through
the EMG_TUNE_CACHE table, at the candidate depth -- the levels below level 0
of at most 1024 nodes -- and at every level below level 0) give, bit for bit,
the displacement and cycle count of the same solves with every pass launched
on its own: 3D anisotropic and isotropic and 2D problems, FP64, mixed
precision, two FP32 cycles per refinement step, V(2,1) smoothing, F-cycles,
graph replay and eager recording.  Batches whose problems have tails starting
at different levels equal the solves without tails, and so do composite (AMR)
solves, whose base hierarchy takes the tail."""
import json

import numpy as np
import pytest

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


def tail_keys(prob, spec, value):
    """Table entries setting the tail of problem `prob` (level 0 of `spec`)
    to `value` levels in both precisions."""
    m = prob.level_shape(0)[0]
    per = sum(1 << a for a in range(3) if a >= spec.dim or spec.periodic[a])   # 2D: the third axis counts as periodic
    iso = "/iso" if spec.kind == "iso" else ""
    return {f"gfx950/{pre}/{m[0]}x{m[1]}x{m[2]}/p{per}{iso}/tail": value for pre in ("fp64", "fp32")}


def candidate(prob):
    """Levels below level 0 with at most 1024 nodes, counted from the bottom."""
    nl = prob.num_levels()
    k = 0
    while k < nl - 1 and np.prod(prob.level_shape(nl - 1 - k)[0]) <= 1024:
        k += 1
    return k


def force(emg, monkeypatch, path, entries):
    path.write_text(json.dumps(entries))
    monkeypatch.setenv("EMG_TUNE_CACHE", str(path))
    emg.autotune_reset()


CASES = {
    "poly65": lambda: synth.polycrystal_3d(n=65, grains=8, seed=7),   # ... 8x8x9, 4x4x5 fused
    "incl33": lambda: synth.inclusion_3d(n=33, seed=3),               # ... 9^3, 5^3 fused
    "incl2d": lambda: synth.inclusion_2d(n=65),                       # 17^2, 9^2, 5^2, 3^2 fused
}
VARIANTS = [dict(precision="fp64"), dict(precision="mixed"), dict(precision="mixed", inner_cycles=2),
            dict(precision="fp64", nu1=2, nu2=1), dict(precision="mixed", nu1=2, nu2=1, inner_cycles=2),
            dict(precision="fp64", cycle="F"), dict(precision="mixed", cycle="F")]


@pytest.mark.parametrize("name", list(CASES))
def test_tail_bitwise(emg, ctx, tmp_path, monkeypatch, name):
    spec = CASES[name]()
    prob = emg.Problem.from_spec(ctx, spec)
    cache = tmp_path / "tune.json"
    emg.autotune_reset()
    try:
        nl = prob.num_levels()
        k = candidate(prob)
        assert 2 <= k < nl, (k, nl)
        assert prob.tail_levels("fp64") == 0 and prob.tail_levels("mixed") == 0   # default: no fusion
        ref = []
        for v in VARIANTS:
            print(f"[gpu] tail {name} {v}", flush=True)
            st = prob.solve(rtol=1e-10, max_cycles=400, **v)
            u = prob.displacement().copy()
            st0 = prob.solve(rtol=1e-10, max_cycles=400, use_graph=0, **v)
            assert st0["cycles"] == st["cycles"], v
            np.testing.assert_array_equal(prob.displacement(), u)
            ref.append((st["cycles"], u))
        for depth in (k, nl - 1):   # the candidate levels fused; every level below 0 fused
            force(emg, monkeypatch, cache, tail_keys(prob, spec, depth))
            assert prob.tail_levels("fp64") == depth and prob.tail_levels("mixed") == depth
            for v, (c, u) in zip(VARIANTS if depth == k else VARIANTS[:2], ref):
                print(f"[gpu] tail {name} depth {depth} {v}", flush=True)
                st = prob.solve(rtol=1e-10, max_cycles=400, use_graph=0, **v)
                assert st["cycles"] == c, (depth, v, st["cycles"], c)
                np.testing.assert_array_equal(prob.displacement(), u)
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()
        prob.close()


def _batch_mix():
    return [synth.polycrystal_3d(n=17, grains=8, seed=11),   # tail from level 1
            synth.inclusion_3d(n=33, seed=3),
            synth.polycrystal_3d(n=33, grains=12, seed=12),
            synth.inclusion_2d(n=65),
            synth.random_problem(2, (65, 33), ("dirichlet", "dirichlet", "traction", "traction", "periodic",
                                               "periodic"), "aniso", seed=10, with_body=True)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tail_in_batches(emg, ctx, tmp_path, monkeypatch, precision):
    specs = _batch_mix()
    cache = tmp_path / "tune.json"
    emg.autotune_reset()
    probs = [emg.Problem.from_spec(ctx, sp) for sp in specs]
    try:
        assert all(p.tail_levels(precision) == 0 for p in probs)
        stats = emg.solve_batch(probs, rtol=1e-10, max_cycles=400, precision=precision, check_every=3)
        got = [(st["cycles"], p.displacement().copy()) for st, p in zip(stats, probs)]
        depths = [candidate(p) for p in probs]
        assert all(d >= 2 for d in depths[:4]), depths
        assert len({p.num_levels() - d for p, d in zip(probs, depths)}) > 1   # tails start at different levels
        entries = {}
        for p, sp, d in zip(probs, specs, depths):
            entries.update(tail_keys(p, sp, d))
        force(emg, monkeypatch, cache, entries)
        assert [p.tail_levels(precision) for p in probs] == depths
        print(f"[gpu] tail batch {precision} depths {depths}", flush=True)
        stats = emg.solve_batch(probs, rtol=1e-10, max_cycles=400, precision=precision, check_every=3)
        for sp, st, p, (c, u) in zip(specs, stats, probs, got):
            assert st["cycles"] == c, sp.name
            np.testing.assert_array_equal(p.displacement(), u)
        for sp, p, (c, u) in zip(specs, probs, got):
            st = p.solve(rtol=1e-10, max_cycles=400, precision=precision, use_graph=0)
            assert st["cycles"] == c, sp.name
            np.testing.assert_array_equal(p.displacement(), u)
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()
        for p in probs:
            p.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_tail_under_amr(emg, ctx, tmp_path, monkeypatch, dim):
    ap = synth.smooth_amr(dim=dim, levels=2, n=17, kind="aniso")   # base 17^d: 9^d and 5^d (2D: and 3^2) fused
    prob = emg.Problem.from_amr(ctx, ap)
    cache = tmp_path / "tune.json"
    emg.autotune_reset()
    try:
        k = candidate(prob)
        assert k >= 2
        ref = {}
        for prec in ("fp64", "mixed"):
            st = prob.solve(rtol=1e-10, max_cycles=400, precision=prec)
            ref[prec] = (st["cycles"], prob.displacement().copy())
        force(emg, monkeypatch, cache, tail_keys(prob, ap.base, k))
        assert prob.tail_levels("fp64") == k
        for prec in ("fp64", "mixed"):
            st = prob.solve(rtol=1e-10, max_cycles=400, precision=prec, use_graph=0)
            assert st["cycles"] == ref[prec][0]
            np.testing.assert_array_equal(prob.displacement(), ref[prec][1])
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()
        prob.close()


def test_tail_in_server(emg, ctx, tmp_path, monkeypatch):
    """Served requests (3 slots, admission at cycle boundaries) whose batched
    cycles run the fused tail, forced for every domain of the stream, give
    the displacement and cycle count of their solo solves without it."""
    specs = [synth.polycrystal_3d(n=17, grains=8, seed=21),
             synth.inclusion_3d(n=33, seed=5),
             synth.inclusion_2d(n=65),
             synth.polycrystal_3d(n=17, grains=8, seed=22),
             synth.polycrystal_3d(n=33, grains=12, seed=23),
             synth.inclusion_3d(n=17, seed=6)]
    opts = dict(rtol=1e-10, max_cycles=400, precision="mixed", check_every=2)
    cache = tmp_path / "tune.json"
    emg.autotune_reset()
    solo, entries = [], {}
    for sp in specs:
        p = emg.Problem.from_spec(ctx, sp)
        st = p.solve(**opts)
        solo.append((st["cycles"], p.displacement()))
        entries.update(tail_keys(p, sp, candidate(p)))
        p.close()
    try:
        force(emg, monkeypatch, cache, entries)
        print(f"[gpu] tail server {len(specs)} requests", flush=True)
        srv = emg.Server(ctx, max_slots=3, **opts)
        tickets = [srv.submit(sp) for sp in specs]
        for sp, t, (c, u) in zip(specs, tickets, solo):
            got, info = srv.wait(t)
            assert info["done"] and info["status"] == emg.EMG_OK, (sp.name, info)
            assert info["cycles"] == c, (sp.name, info["cycles"], c)
            assert np.array_equal(got.reshape(u.shape), u), sp.name
        srv.close()
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()
