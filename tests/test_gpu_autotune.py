"""The autotuner (emg_autotune) picks by measurement, per level: the
stencil pass (the tile kernel in tiles of 64x4, 64x2, 128x2 or 32x8 nodes,
or the z-marching pass with some number of chunks per column), and the tile
shapes of the restriction from the level and of the interpolation onto it;
per problem, whether the cycle on its smallest levels runs fused.
Every variant computes the same values node by node, so tuning changes
timing only.  On a 65^3 polycrystal (periodic x and y: levels 64x64x65 and
coarser), solves after tuning, and with every variant forced through the
EMG_TUNE_CACHE file, give bit-identical displacements and the same cycle
counts in FP64 and mixed precision; the recorded choices are what
emg_level_zmarch / emg_level_tiles report, and the file restores them after
the table is emptied."""
import json

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRECS = ("fp64", "mixed")


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


def plans(prob):
    return {p: [prob.level_zmarch(l, p) for l in range(prob.num_levels())] for p in PRECS}


def test_autotune_changes_timing_only(emg, ctx, tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("EMG_TUNE_CACHE", str(cache))
    emg.autotune_reset()
    try:
        spec = synth.polycrystal_3d(n=65, grains=8, seed=7)
        prob = emg.Problem.from_spec(ctx, spec)
        nlev = prob.num_levels()
        print("[gpu] autotune: reference solves", flush=True)
        ref = {}
        for p in PRECS:
            st = prob.solve(rtol=1e-10, max_cycles=300, precision=p)
            ref[p] = (st["cycles"], prob.displacement().copy())
        print("[gpu] autotune: tuning", flush=True)
        tuned = {p: prob.autotune(p, reps=5) for p in PRECS}
        assert tuned == {"fp64": nlev, "mixed": nlev}   # every level has variants
        assert prob.autotune("fp64", reps=5) == 0      # already in the table
        after = plans(prob)
        tiles = {p: [prob.level_tiles(l, p) for l in range(nlev)] for p in PRECS}
        table = json.loads(cache.read_text())
        assert len(table) == 2 * (3 * nlev - 2 + 1)   # + the fused-tail choice per precision
        for key, v in table.items():
            parts = key.split("/")
            arch, prec, shape, per = parts[:4]
            assert arch.startswith("gfx") and per == "p3"
            p = "fp64" if prec == "fp64" else "mixed"
            lev = [prob.level_shape(l)[0] for l in range(nlev)].index(tuple(int(x) for x in shape.split("x")))
            if parts[4:] == ["tail"]:    # 8x8x9 and 4x4x5 fused, or not
                assert lev == 0 and v in (0, 2) and prob.tail_levels(p) == v
            elif len(parts) == 4:        # stencil pass
                if v > 0:
                    assert after[p][lev] == v and tiles[p][lev][0] == 0
                else:
                    assert after[p][lev] == 0 and tiles[p][lev][0] == -v
            else:                        # restriction / interpolation tile shape
                assert parts[4] in ("r", "i") and 0 <= v <= 3
                assert tiles[p][lev][1 if parts[4] == "r" else 2] == v
        print(f"[gpu] autotune: table {table}", flush=True)
        for p in PRECS:
            st = prob.solve(rtol=1e-10, max_cycles=300, precision=p)
            assert st["cycles"] == ref[p][0]
            np.testing.assert_array_equal(prob.displacement(), ref[p][1])

        # every variant, forced through the table file, solves identically
        def forced(entries, p):
            cache.write_text(json.dumps(entries))
            emg.autotune_reset()
            st = prob.solve(rtol=1e-10, max_cycles=300, precision=p, use_graph=0)
            assert st["cycles"] == ref[p][0], entries
            np.testing.assert_array_equal(prob.displacement(), ref[p][1])
        for p in PRECS:
            pre = "fp64" if p == "fp64" else "fp32"
            k0 = [k for k in table if f"/{pre}/64x64x65/p3" in k and k.count("/") == 3][0]
            k1 = [k for k in table if f"/{pre}/32x32x33/p3" in k and k.count("/") == 3][0]
            for v in list(range(-3, 0)) + list(range(0, 63 // 8 + 1)):
                forced({k0: v}, p)
                if v <= 0:
                    assert prob.level_zmarch(0, p) == 0 and prob.level_tiles(0, p)[0] == -v
                else:
                    assert prob.level_zmarch(0, p) == v
            for s in range(4):
                forced({k1: -s, k0 + "/r": s, k0 + "/i": s, k1 + "/r": s, k1 + "/i": s}, p)
                assert prob.level_tiles(0, p)[1:] == (s, s) and prob.level_tiles(1, p) == (s, s, s)
        # the file alone restores the table
        cache.write_text(json.dumps(table))
        emg.autotune_reset()
        assert plans(prob) == after
        assert {p: [prob.level_tiles(l, p) for l in range(nlev)] for p in PRECS} == tiles
        # out-of-range entries are ignored (the cost model's plan is used)
        cache.write_text(json.dumps({k: 99 for k in table}))
        emg.autotune_reset()
        monkeypatch.delenv("EMG_TUNE_CACHE")
        base = plans(prob)
        monkeypatch.setenv("EMG_TUNE_CACHE", str(cache))
        emg.autotune_reset()
        assert plans(prob) == base
        assert all(prob.level_tiles(l, p)[0] == 0 for l in range(nlev) for p in PRECS)
        prob.close()
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()


def test_autotune_2d_and_errors(emg, ctx):
    """2D levels have the tile-shape variants; a tuned 2D solve is
    bit-identical to the untuned one."""
    spec = synth.inclusion_2d(n=65)
    prob = emg.Problem.from_spec(ctx, spec)
    try:
        st0 = prob.solve(rtol=1e-10, max_cycles=300)
        u0 = prob.displacement()
        assert prob.autotune("fp64", reps=5) == prob.num_levels()
        st1 = prob.solve(rtol=1e-10, max_cycles=300)
        assert st1["cycles"] == st0["cycles"]
        np.testing.assert_array_equal(prob.displacement(), u0)
        with pytest.raises(emg.EmgError):
            prob.autotune("fp64", reps=0)
    finally:
        prob.close()
        emg.autotune_reset()


def test_tuned_plan_reaches_batches(emg, ctx, tmp_path, monkeypatch):
    """A table entry also steers the batched plans (one launch per cycle
    step over several problems): with the 64x64x65 level forced to the
    z-marching pass (3 chunks per column, which the cost model never picks
    there), a batch of two 65^3 polycrystals gives each problem the
    displacement and cycle count of its own solve under the cost model."""
    cache = tmp_path / "tune.json"
    emg.autotune_reset()
    try:
        specs = [synth.polycrystal_3d(n=65, grains=g, seed=s) for g, s in ((8, 7), (12, 9))]
        probs = [emg.Problem.from_spec(ctx, sp) for sp in specs]
        ref = {}
        for p in PRECS:
            for i, pr in enumerate(probs):
                st = pr.solve(rtol=1e-10, max_cycles=300, precision=p)
                ref[p, i] = (st["cycles"], pr.displacement().copy())
        assert probs[0].level_zmarch(0, "fp64") == 0 and probs[0].level_zmarch(0, "mixed") == 0
        cache.write_text(json.dumps({"gfx950/fp64/64x64x65/p3": 3, "gfx950/fp32/64x64x65/p3": 3}))
        monkeypatch.setenv("EMG_TUNE_CACHE", str(cache))
        emg.autotune_reset()
        arch_ok = probs[0].level_zmarch(0, "fp64") == 3
        if not arch_ok:
            pytest.skip("device architecture is not gfx950")
        assert probs[0].level_zmarch(0, "mixed") == 3
        for p in PRECS:
            print(f"[gpu] tuned batch {p}", flush=True)
            sts = emg.solve_batch(probs, rtol=1e-10, max_cycles=300, precision=p)
            for i, pr in enumerate(probs):
                assert sts[i]["cycles"] == ref[p, i][0]
                np.testing.assert_array_equal(pr.displacement(), ref[p, i][1])
        for pr in probs:
            pr.close()
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()
