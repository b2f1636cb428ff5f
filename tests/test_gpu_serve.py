"""Continuous-batching server: requests of mixed sizes, dimensions and
moduli kinds submitted while others run (fewer slots than requests, so
admission happens at cycle boundaries) give, bit for bit, the displacement
and cycle count each gives alone through emg_solve; resident hierarchies
are reused for repeated domains and evicted under an HBM budget."""
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


def _requests():
    return [synth.polycrystal_3d(n=17, grains=8, seed=21),
            synth.inclusion_3d(n=33, seed=5),
            synth.inclusion_2d(n=65),
            synth.polycrystal_3d(n=17, grains=8, seed=22),      # same domain as the first: pooled hierarchy
            synth.random_problem(2, (33, 65), ("dirichlet", "traction", "periodic", "periodic", "periodic",
                                               "periodic"), "aniso", seed=7, with_body=True),
            synth.polycrystal_3d(n=33, grains=12, seed=23),
            synth.inclusion_3d(n=17, seed=6),
            synth.polycrystal_3d(n=17, grains=8, seed=24)]


def _solo(emg, ctx, specs, **opts):
    out = []
    for sp in specs:
        p = emg.Problem.from_spec(ctx, sp)
        st = p.solve(**opts)
        out.append((st["cycles"], p.displacement()))
        p.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_served_bitwise_equals_solo(emg, ctx, precision):
    specs = _requests()
    opts = dict(rtol=1e-10, max_cycles=400, precision=precision, check_every=2)
    print(f"[gpu] serve {len(specs)} requests {precision}", flush=True)
    solo = _solo(emg, ctx, specs, **opts)
    srv = emg.Server(ctx, max_slots=3, **opts)
    tickets = [srv.submit(sp) for sp in specs]
    for sp, t, (c, u) in zip(specs, tickets, solo):
        got, info = srv.wait(t)
        assert info["done"] and info["status"] == emg.EMG_OK, (sp.name, info)
        assert info["converged"] and info["rel_res"] <= 1e-10, sp.name
        assert info["cycles"] == c, (sp.name, info["cycles"], c)
        assert info["t_submit"] <= info["t_admit"] <= info["t_done"]
        assert np.array_equal(got.reshape(u.shape), u), sp.name
    srv.close()


def test_served_under_budget_and_late_arrivals(emg, ctx):
    """A budget that holds about two of the hierarchies forces eviction of
    idle pooled problems and admission only as memory frees up; requests
    submitted after earlier ones finished reuse the server."""
    specs = _requests()[:4]
    solo = _solo(emg, ctx, specs, rtol=1e-10, max_cycles=400)
    sizes = []
    for sp in specs:
        p = emg.Problem.from_spec(ctx, sp)
        sizes.append(p.footprint())
        p.close()
    small = emg.Context(0, hbm_budget_bytes=int(1.3 * max(sizes)))
    srv = emg.Server(small, max_slots=4, rtol=1e-10, max_cycles=400)
    t0 = srv.submit(specs[0])
    u0, i0 = srv.wait(t0)
    assert i0["status"] == emg.EMG_OK and np.array_equal(u0.reshape(solo[0][1].shape), solo[0][1])
    tickets = [srv.submit(sp) for sp in specs[1:]]
    for t, (c, u) in zip(tickets, solo[1:]):
        got, info = srv.wait(t)
        assert info["status"] == emg.EMG_OK and info["cycles"] == c
        assert np.array_equal(got.reshape(u.shape), u)
    srv.close()
    small.close()


def test_request_larger_than_budget_fails_cleanly(emg):
    tiny = emg.Context(0, hbm_budget_bytes=1 << 20)
    srv = emg.Server(tiny, max_slots=2)
    t = srv.submit(synth.inclusion_3d(n=33, seed=1))
    _, info = srv.wait(t)
    assert info["done"] and info["status"] == emg.EMG_ENOMEM
    t2 = srv.submit(synth.inclusion_2d(n=17))
    _, info2 = srv.wait(t2)
    assert info2["status"] in (emg.EMG_OK, emg.EMG_ENOMEM)
    srv.close()
    tiny.close()


def test_served_trace_matches_solo_and_oracle(emg, ctx):
    """A stretch of the served stream (96 requests of the Poisson trace, all
    sizes and both problem types, submitted at once so they queue and join
    running batches): every result equals, bit for bit, the solo solve of
    its input, and one sampled input is checked against the oracle."""
    import oracle
    trace = synth.serving_trace(count=96, seed=2005)
    keys = sorted({(r.kind, r.n, r.variant) for r in trace})
    print(f"[gpu] served trace: {len(trace)} requests over {len(keys)} inputs", flush=True)
    specs = {k: synth.serving_problem(*k) for k in keys}
    opts = dict(rtol=1e-10, max_cycles=400, precision="mixed")
    solo = {k: u for k, (_, u) in zip(keys, _solo(emg, ctx, [specs[k] for k in keys], **opts))}
    srv = emg.Server(ctx, max_slots=16, **opts)
    tickets = [(srv.submit(specs[(r.kind, r.n, r.variant)]), (r.kind, r.n, r.variant)) for r in trace]
    for t, k in tickets:
        got, info = srv.wait(t)
        assert info["status"] == emg.EMG_OK and info["converged"], (k, info)
        assert np.array_equal(got.reshape(solo[k].shape), solo[k]), k
    srv.close()
    small = [k for k in keys if k[1] == 33]
    k = small[0]
    ref = oracle.solve(specs[k], tol=1e-13, max_cycles=400)
    err = float(np.linalg.norm(solo[k] - ref.u) / np.linalg.norm(ref.u))
    print(f"[gpu] served {k} vs oracle: rel error {err:.2e}", flush=True)
    assert err <= 1e-8
