"""The autotuner (emg_autotune) picks each level's stencil pass by
measurement: the tile kernel or the z-marching pass with some number of
chunks per column.  Every variant computes the same rows with the same
arithmetic, so tuning must change timing only.  On a 65^3 polycrystal
(periodic x and y: levels 64x64x65 and coarser), where the cost model keeps
the tile kernel on the finest level, solves after tuning give bit-identical
displacements and the same cycle counts in FP64 and mixed precision; the
recorded choices are what emg_level_zmarch reports; the EMG_TUNE_CACHE file
holds them and restores them after the table is emptied."""
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
        print("[gpu] autotune: reference solves", flush=True)
        ref = {}
        for p in PRECS:
            st = prob.solve(rtol=1e-10, max_cycles=300, precision=p)
            ref[p] = (st["cycles"], prob.displacement().copy())
        print("[gpu] autotune: tuning", flush=True)
        tuned = {p: prob.autotune(p, reps=5) for p in PRECS}
        assert tuned == {"fp64": 1, "mixed": 1}   # only the 64x64x65 level is wide enough
        assert prob.autotune("fp64", reps=5) == 0  # already in the table
        after = plans(prob)
        table = json.loads(cache.read_text())
        assert len(table) == 2
        for key, chunks in table.items():
            arch, prec, shape, per = key.split("/")
            assert arch.startswith("gfx") and per == "p3" and shape == "64x64x65"
            assert after["fp64" if prec == "fp64" else "mixed"][0] == chunks
            assert 0 <= chunks <= 63 // 8
        print(f"[gpu] autotune: table {table}", flush=True)
        for p in PRECS:
            st = prob.solve(rtol=1e-10, max_cycles=300, precision=p)
            assert st["cycles"] == ref[p][0]
            np.testing.assert_array_equal(prob.displacement(), ref[p][1])
        # every variant, forced through the table file, solves identically
        for p in PRECS:
            for chunks in range(0, 63 // 8 + 1):
                key = [k for k in table if ("/fp64/" in k) == (p == "fp64")][0]
                cache.write_text(json.dumps({key: chunks}))
                emg.autotune_reset()
                assert prob.level_zmarch(0, p) == chunks
                st = prob.solve(rtol=1e-10, max_cycles=300, precision=p, use_graph=0)
                assert st["cycles"] == ref[p][0]
                np.testing.assert_array_equal(prob.displacement(), ref[p][1])
        # the file alone restores the table
        cache.write_text(json.dumps(table))
        emg.autotune_reset()
        assert plans(prob) == after
        # out-of-range entries are ignored (the cost model's plan is used)
        cache.write_text(json.dumps({k: 99 for k in table}))
        emg.autotune_reset()
        monkeypatch.delenv("EMG_TUNE_CACHE")
        base = plans(prob)
        monkeypatch.setenv("EMG_TUNE_CACHE", str(cache))
        emg.autotune_reset()
        assert plans(prob) == base
        prob.close()
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()


def test_autotune_argument_errors(emg, ctx):
    spec = synth.inclusion_2d(n=33)
    prob = emg.Problem.from_spec(ctx, spec)
    assert prob.autotune("fp64") == 0   # 2D: one variant
    with pytest.raises(emg.EmgError):
        prob.autotune("fp64", reps=0)
    prob.close()


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
