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
