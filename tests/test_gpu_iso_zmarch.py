"""The z-marching stencil pass on isotropic levels (Lame moduli, two per
node): forced through the EMG_TUNE_CACHE table at several chunk counts, the
finest-level operator, residual and Jacobi sweep equal the tile kernel's bit
for bit and the oracle element by element (FP64 to 1e-12, FP32 to 2e-5 of
the output's magnitude), on grids with non-periodic, ragged x and y,
Neumann and traction faces, periodic x and z, and periodic x and y.  Solves (FP64, mixed,
two FP32 cycles per refinement step, F-cycles) and ragged batches whose
isotropic finest levels take the z-marching pass give the displacement and
cycle count of the same solves on the tile kernel; so do composite (AMR)
solves whose base level takes it, isotropic or anisotropic."""
import json

import numpy as np
import pytest

import oracle
import synth

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


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


def host(t):
    return t.detach().to("cpu", dtype=torch.float64).numpy()


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def stencil_key(prob, spec, level, pre):
    m = prob.level_shape(level)[0]
    per = sum(1 << a for a in range(3) if spec.periodic[a])
    return f"gfx950/{pre}/{m[0]}x{m[1]}x{m[2]}/p{per}/iso"


def force(emg, monkeypatch, path, entries):
    path.write_text(json.dumps(entries))
    monkeypatch.setenv("EMG_TUNE_CACHE", str(path))
    emg.autotune_reset()


CASES = {
    # non-periodic x and y (ragged 64 x 4 tiles in both), Dirichlet / traction / Neumann faces
    "iso_nonperiodic": dict(n=(97, 97, 65), bc=("dirichlet", "traction", "neumann", "traction", "traction", "neumann")),
    # periodic x (96 stored nodes: a ragged second column) and z (64 planes, wrapped), non-periodic y
    "iso_periodic_xz": dict(n=(97, 97, 65), bc=("periodic", "periodic", "dirichlet", "traction", "periodic", "periodic")),
    # periodic x and y (96 stored nodes each: ragged second column, wrapped halo rows), Dirichlet z
    "iso_periodic_xy": dict(n=(97, 97, 65), bc=("periodic", "periodic", "periodic", "periodic", "dirichlet", "dirichlet")),
}


@pytest.mark.parametrize("name", list(CASES))
def test_iso_zmarch_level_steps(emg, ctx, tmp_path, monkeypatch, name):
    c = CASES[name]
    spec = synth.random_problem(3, c["n"], c["bc"], "iso", seed=23, with_body=True,
                                lo=(0.0, -0.2, 0.1), hi=(1.0, 0.8, 0.8))
    g = oracle.Grid.of(spec)
    prob = emg.Problem.from_spec(ctx, spec)
    cache = tmp_path / "tune.json"
    rng = np.random.default_rng(8)
    u = rng.standard_normal(g.shape(3))
    f = rng.standard_normal(g.shape(3))
    print(f"[gpu] iso z-march level steps {name} m={spec.m}: oracle", flush=True)
    ref = {"apply": oracle.apply(g, spec.C, u), "residual": oracle.residual(g, spec.C, u, f),
           "jacobi": oracle.jacobi(g, spec.C, u, f, 2.0 / 3.0)}
    try:
        for prec, pre, dt, tol in (("fp64", "fp64", torch.float64, 1e-12), ("mixed", "fp32", torch.float32, 2e-5)):
            ud, fd = dev(u, dt), dev(f, dt)
            key = stencil_key(prob, spec, 0, pre)
            tile = None
            for v in (0, 1, 2, 7):   # the tile kernel, then 1, 2 and 7 chunks per column
                force(emg, monkeypatch, cache, {key: v})
                assert prob.level_zmarch(0, prec) == v, (prec, v)
                got = {}
                for step in ("apply", "residual", "jacobi"):
                    out = torch.empty_like(ud)
                    out.fill_(float("nan"))   # every node must be written
                    if step == "apply":
                        prob.level_apply(0, ud, out, precision=prec)
                    elif step == "residual":
                        prob.level_residual(0, ud, fd, out, precision=prec)
                    else:
                        prob.level_jacobi(0, ud, fd, out, precision=prec)
                    got[step] = host(out)
                    err = rel_err(got[step], ref[step])
                    print(f"[gpu]   {prec} chunks {v} {step}: max rel error {err:.2e}", flush=True)
                    assert err <= tol, (prec, v, step)
                if tile is None:
                    tile = got
                else:
                    for step in got:
                        np.testing.assert_array_equal(got[step], tile[step], err_msg=f"{prec} {v} {step}")
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()
        prob.close()


VARIANTS = [dict(precision="fp64"), dict(precision="mixed"), dict(precision="mixed", inner_cycles=2),
            dict(precision="fp64", cycle="F")]


def test_iso_zmarch_solves(emg, ctx, tmp_path, monkeypatch):
    spec = synth.inclusion_3d(n=97, seed=4)   # 97^3 isotropic, traction and Dirichlet faces
    prob = emg.Problem.from_spec(ctx, spec)
    cache = tmp_path / "tune.json"
    keys = [stencil_key(prob, spec, 0, pre) for pre in ("fp64", "fp32")]
    try:
        force(emg, monkeypatch, cache, {k: 0 for k in keys})
        ref = []
        for v in VARIANTS:
            st = prob.solve(rtol=1e-10, max_cycles=400, **v)
            ref.append((st["cycles"], prob.displacement().copy()))
        for nzc in (1, 4):
            force(emg, monkeypatch, cache, {k: nzc for k in keys})
            assert prob.level_zmarch(0, "fp64") == nzc and prob.level_zmarch(0, "mixed") == nzc
            for v, (c, u) in zip(VARIANTS, ref):
                print(f"[gpu] iso z-march solve chunks {nzc} {v}", flush=True)
                for graph in (1, 0):
                    st = prob.solve(rtol=1e-10, max_cycles=400, use_graph=graph, **v)
                    assert st["cycles"] == c, (nzc, v, graph)
                    np.testing.assert_array_equal(prob.displacement(), u)
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()
        prob.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_iso_zmarch_in_batches(emg, ctx, tmp_path, monkeypatch, precision):
    specs = [synth.inclusion_3d(n=97, seed=4),
             synth.polycrystal_3d(n=65, grains=8, seed=7),
             synth.random_problem(3, (97, 97, 65), ("periodic", "periodic", "dirichlet", "traction", "periodic",
                                                    "periodic"), "iso", seed=24, with_body=True),
             synth.inclusion_3d(n=33, seed=5)]   # too small for the z-marching pass
    cache = tmp_path / "tune.json"
    probs = [emg.Problem.from_spec(ctx, sp) for sp in specs]
    pre = "fp64" if precision == "fp64" else "fp32"
    iso = [(probs[i], specs[i]) for i in (0, 2)]
    try:
        force(emg, monkeypatch, cache, {stencil_key(p, sp, 0, pre): 0 for p, sp in iso})
        solo = []
        for p in probs:
            st = p.solve(rtol=1e-10, max_cycles=400, precision=precision)
            solo.append((st["cycles"], p.displacement().copy()))
        force(emg, monkeypatch, cache, {stencil_key(p, sp, 0, pre): 2 for p, sp in iso})
        assert all(p.level_zmarch(0, precision) == 2 for p, _ in iso)
        print(f"[gpu] iso z-march batch {precision}", flush=True)
        stats = emg.solve_batch(probs, rtol=1e-10, max_cycles=400, precision=precision, check_every=2)
        for sp, st, p, (c, u) in zip(specs, stats, probs, solo):
            assert st["cycles"] == c, sp.name
            np.testing.assert_array_equal(p.displacement(), u)
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()
        for p in probs:
            p.close()


@pytest.mark.parametrize("kind", ["iso", "aniso"])
def test_zmarch_under_amr(emg, ctx, tmp_path, monkeypatch, kind):
    """A composite (AMR) solve whose 97^3 base level takes the z-marching
    pass equals, bit for bit and in cycle count, the same solve on the tile
    kernel, in FP64 and mixed precision (base level and refined box)."""
    ap = synth.smooth_amr(dim=3, levels=2, n=97, kind=kind)
    prob = emg.Problem.from_amr(ctx, ap)
    cache = tmp_path / "tune.json"
    iso = "/iso" if kind == "iso" else ""
    shapes = [prob.level_shape(0)[0]] + [tuple(prob.amr_level_shape(k)) for k in range(1, prob.amr_num_levels())]

    def entries(v):
        return {f"gfx950/{pre}/{m[0]}x{m[1]}x{m[2]}/p0{iso}": v for m in shapes for pre in ("fp64", "fp32")}
    try:
        force(emg, monkeypatch, cache, entries(0))
        ref = {}
        for prec in ("fp64", "mixed"):
            st = prob.solve(rtol=1e-10, max_cycles=400, precision=prec)
            ref[prec] = (st["cycles"], prob.displacement().copy(), prob.amr_displacement(1).copy())
        for nzc in (1, 3):
            force(emg, monkeypatch, cache, entries(nzc))
            for prec in ("fp64", "mixed"):
                assert prob.level_zmarch(0, prec) == nzc
                print(f"[gpu] z-march under AMR {kind} chunks {nzc} {prec}", flush=True)
                st = prob.solve(rtol=1e-10, max_cycles=400, precision=prec)
                assert st["cycles"] == ref[prec][0], (nzc, prec)
                np.testing.assert_array_equal(prob.displacement(), ref[prec][1])
                np.testing.assert_array_equal(prob.amr_displacement(1), ref[prec][2])
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()
        prob.close()


def test_autotune_isotropic_levels(emg, ctx, tmp_path, monkeypatch):
    """emg_autotune measures the isotropic z-marching pass beside the tile
    shapes: on a 97^3 inclusion every level is tuned, the level-0 entries
    (keyed ".../iso") hold a valid variant that emg_level_zmarch reports, and
    the tuned solves equal the untuned ones bit for bit."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("EMG_TUNE_CACHE", str(cache))
    emg.autotune_reset()
    spec = synth.inclusion_3d(n=97, seed=4)
    prob = emg.Problem.from_spec(ctx, spec)
    try:
        ref = {}
        for p in ("fp64", "mixed"):
            st = prob.solve(rtol=1e-10, max_cycles=400, precision=p)
            ref[p] = (st["cycles"], prob.displacement().copy())
        print("[gpu] autotune isotropic 97^3", flush=True)
        for p in ("fp64", "mixed"):
            assert prob.autotune(p, reps=5) == prob.num_levels()
        table = json.loads(cache.read_text())
        for p, pre in (("fp64", "fp64"), ("mixed", "fp32")):
            v = table[stencil_key(prob, spec, 0, pre)]
            assert -3 <= v <= 95 // 8, v
            assert prob.level_zmarch(0, p) == max(v, 0)
            st = prob.solve(rtol=1e-10, max_cycles=400, precision=p)
            assert st["cycles"] == ref[p][0]
            np.testing.assert_array_equal(prob.displacement(), ref[p][1])
        assert all("/iso" in k for k in table)
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()
        prob.close()


def test_iso_zmarch_mixed_periodic(emg, ctx, tmp_path, monkeypatch):
    """Mixed-precision solves on a grid periodic in x (ragged second column)
    and z, where the FP64 residual pass of each refinement step also writes
    the FP32 cycle's zero-start sweep on the z-marching pass: equal, bit for
    bit and in cycle count, to the solves on the tile kernel (which runs that
    sweep as a pass of its own)."""
    c = CASES["iso_periodic_xz"]
    spec = synth.random_problem(3, c["n"], c["bc"], "iso", seed=23, with_body=True,
                                lo=(0.0, -0.2, 0.1), hi=(1.0, 0.8, 0.8))
    prob = emg.Problem.from_spec(ctx, spec)
    cache = tmp_path / "tune.json"
    keys = [stencil_key(prob, spec, 0, pre) for pre in ("fp64", "fp32")]
    variants = [dict(precision="mixed"), dict(precision="mixed", inner_cycles=2)]
    try:
        force(emg, monkeypatch, cache, {k: 0 for k in keys})
        ref = []
        for v in variants:
            st = prob.solve(rtol=1e-10, max_cycles=400, **v)
            ref.append((st["cycles"], prob.displacement().copy()))
        for nzc in (2, 7):
            force(emg, monkeypatch, cache, {k: nzc for k in keys})
            assert prob.level_zmarch(0, "fp64") == nzc
            for v, (cyc, u) in zip(variants, ref):
                print(f"[gpu] iso z-march mixed periodic chunks {nzc} {v}", flush=True)
                st = prob.solve(rtol=1e-10, max_cycles=400, **v)
                assert st["cycles"] == cyc, (nzc, v)
                np.testing.assert_array_equal(prob.displacement(), u)
    finally:
        monkeypatch.delenv("EMG_TUNE_CACHE", raising=False)
        emg.autotune_reset()
        prob.close()
