"""GPU parity of the reflux-free AMR composite solve (Sec. 3.2, App. A)
against the oracle's composite system, through the C ABI."""
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


CASES = {"2d_2L": (2, 2, 17), "2d_3L": (2, 3, 17), "3d_2L": (3, 2, 9), "3d_2L_17": (3, 2, 17),
         # anisotropic moduli (21 / 6 stored constants) on every level
         "2d_3L_aniso": (2, 3, 33, 5, "aniso"), "3d_2L_aniso": (3, 2, 17, 5, "aniso"),
         # two boxes per refined level (L-shaped unions with reentrant corners)
         "2d_3L_Lshape": (2, 3, 17, 2, "iso", "L"), "3d_3L_Lshape": (3, 3, 17, 2, "iso", "L"),
         "3d_3L_Lshape_aniso": (3, 3, 17, 2, "aniso", "L")}


def _state(prob, comp, u):
    prob.set_displacement(u[0])
    for k in range(1, len(u)):
        prob.amr_set_displacement(k, u[k])


def _gpu_solution(prob, nlev):
    return [prob.displacement()] + [prob.amr_displacement(k) for k in range(1, nlev)]


def _rel(u, ref, comp):
    """Relative 2-norm difference over base nodes and valid box nodes."""
    num = float(np.sum((u[0] - ref[0]) ** 2))
    den = float(np.sum(ref[0] ** 2))
    for k in range(1, len(u)):
        v = comp.fines[k - 1].valid_full()
        num += float(np.sum(((u[k] - ref[k]) ** 2)[v]))
        den += float(np.sum((ref[k] ** 2)[v]))
    return np.sqrt(num / den)


@pytest.mark.parametrize("name", list(CASES))
def test_composite_residual_matches_oracle(emg, ctx, name):
    ap = synth.smooth_amr(*CASES[name])
    print(f"[gpu] amr residual {name} boxes={ap.boxes}", flush=True)
    comp = amr.from_problem(ap)
    prob = emg.Problem.from_amr(ctx, ap)
    rng = np.random.default_rng(1)
    u = [1e-3 * rng.standard_normal(comp.grid(k).shape(ap.base.dim)) for k in range(len(ap.boxes) + 1)]
    # Dirichlet rows of the base carry their prescribed values in both
    f0 = comp.f[0]
    u[0] = np.where(oracle.dirichlet_mask(comp.g0), f0, u[0])
    _state(prob, comp, u)
    ref = comp.residual(u)
    masks = comp.unknown_masks()
    gnorm = None
    for k in range(len(u)):
        out = torch.empty(comp.grid(k).shape(ap.base.dim), dtype=torch.float64, device=DEV)
        gnorm = prob.amr_residual(k, out)
        got = out.cpu().numpy()
        m = masks[k]
        scale = np.abs(ref[k][m]).max()
        assert np.abs(got[m] - ref[k][m]).max() <= 1e-12 * scale, k
    assert gnorm == pytest.approx(comp.norm(ref), rel=1e-12)
    prob.close()


_REF = {}


def _reference(name):
    if name not in _REF:
        ap = synth.smooth_amr(*CASES[name])
        comp = amr.from_problem(ap)
        u, hist = comp.solve(tol=1e-13, max_cycles=300)
        _, hist10 = comp.solve(tol=1e-10, max_cycles=300)
        _REF[name] = (ap, comp, u, len(hist10) - 1)
    return _REF[name]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_composite_solve_matches_oracle(emg, ctx, name, precision):
    """FP64 composite cycles, or FP32 composite corrections inside FP64
    refinement: the solution equals the oracle's composite solution to 1e-8
    and satisfies its composite system to 1.2e-10, in the oracle's cycle
    count (mixed: within two)."""
    ap, comp, uref, cycles10 = _reference(name)
    print(f"[gpu] amr solve {name} {precision}", flush=True)
    prob = emg.Problem.from_amr(ctx, ap)
    st = prob.solve(rtol=1e-10, max_cycles=300, precision=precision)
    assert st["converged"] and st["rel_res"] <= 1e-10
    assert abs(st["cycles"] - cycles10) <= (1 if precision == "fp64" else 2)
    u = _gpu_solution(prob, len(ap.boxes) + 1)
    err = _rel(u, uref, comp)
    print(f"[gpu]   cycles={st['cycles']} (oracle {cycles10}) rel_err={err:.2e}", flush=True)
    assert err <= 1e-8
    # the oracle's composite residual of the GPU solution
    r0 = comp.norm(comp.residual(comp.initial()))
    assert comp.norm(comp.residual(u)) / r0 <= 1.2e-10
    nodes = ap.composite_nodes() - ap.base.dirichlet_count()
    assert st["dofs"] == ap.base.dim * nodes
    prob.close()


def test_penny_crack_three_levels(emg, ctx):
    """Diffuse penny crack, 3 levels, on a 33^3 base,
    FP64 and mixed precision: each GPU solution satisfies the oracle's
    composite system to 1e-10, and the two agree to 1e-8."""
    ap = synth.penny_crack(n=33, levels=3, floor=1e-2, width=0.05)
    print(f"[gpu] penny crack 33^3, boxes per level {[len(ap.level_boxes(k)) for k in (1, 2)]}", flush=True)
    comp = amr.from_problem(ap)
    r0 = comp.norm(comp.residual(comp.initial()))
    sols = {}
    for precision in ("fp64", "mixed"):
        prob = emg.Problem.from_amr(ctx, ap)
        st = prob.solve(rtol=1e-10, max_cycles=400, precision=precision)
        assert st["converged"]
        u = _gpu_solution(prob, 3)
        prob.close()
        rel = comp.norm(comp.residual(u)) / r0
        print(f"[gpu]   {precision}: cycles={st['cycles']} oracle rel residual={rel:.2e}", flush=True)
        assert rel <= 1.2e-10
        sols[precision] = u
    diff = _rel(sols["mixed"], sols["fp64"], comp)
    print(f"[gpu]   mixed vs FP64 composite solution: rel diff {diff:.2e}", flush=True)
    assert diff <= 1e-8


def test_amr_rejects_bad_boxes(emg, ctx):
    ap = synth.smooth_amr(2, 1, 17)
    prob = emg.Problem.from_spec(ctx, ap.base)
    for lo, hi in [((2, 8, 0), (24, 24, 0)),      # too close to the domain boundary
                   ((7, 8, 0), (24, 24, 0)),      # odd bound
                   ((8, 8, 0), (8, 24, 0))]:      # empty
        with pytest.raises(emg.EmgError) as ei:
            prob.amr_add_level(lo, hi)
        assert ei.value.status == emg.EMG_EINVAL
    prob.amr_add_level((8, 8, 0), (24, 24, 0))
    st = prob.solve(raise_on_error=False)
    assert st["status"] == emg.EMG_ESTATE          # refined level without moduli
    with pytest.raises(emg.EmgError) as ei:        # levels are added in order
        prob.set_level_boxes(3, [((20, 20, 0), (28, 28, 0))])
    assert ei.value.status == emg.EMG_ESTATE
    prob.close()
    # several boxes: a level-2 box reaching into the notch of an L-shaped level 1
    prob = emg.Problem.from_spec(ctx, ap.base)
    prob.set_level_boxes(1, [((8, 8, 0), (24, 16, 0)), ((8, 16, 0), (16, 24, 0))])
    mask, nvalid = prob.amr_level_valid(1)
    assert nvalid == 17 * 9 + 9 * 9 - 9 and int(mask.sum()) == nvalid
    with pytest.raises(emg.EmgError) as ei:
        prob.set_level_boxes(2, [((24, 24, 0), (36, 36, 0))])
    assert ei.value.status == emg.EMG_EINVAL
    prob.set_level_boxes(2, [((20, 20, 0), (28, 28, 0)), ((36, 20, 0), (44, 28, 0))])
    prob.close()


@pytest.mark.parametrize("name", ["3d_2L_aniso", "3d_3L_Lshape_aniso", "2d_3L_Lshape"])
def test_stress_on_refined_levels(emg, ctx, name):
    """emg_get_stress on every level: from the oracle's composite solution
    (set on every level, ghosts included) the GPU stress equals
    oracle.stress on the level's array at every valid node (1e-12); after a
    GPU solve, within 1e-7 of it."""
    ap, comp, uref, _ = _reference(name)
    d = ap.base.dim
    prob = emg.Problem.from_amr(ctx, ap)
    prob.solve(rtol=1e-10, max_cycles=300)
    after = [prob.stress(level=k) for k in range(len(uref))]
    _state(prob, comp, uref)
    print(f"[gpu] stress on refined levels {name}", flush=True)
    for k in range(len(uref)):
        g = comp.grid(k)
        E = comp.E0 if k == 0 else comp.fines[k - 1].eps0
        ref = oracle.stress(g, comp.C(k), E, uref[k])
        got = prob.stress(level=k)
        v = np.ones(ref.shape[1:], dtype=bool) if k == 0 else comp.fines[k - 1].valid_mask
        scale = np.abs(ref[:, v]).max()
        assert np.abs(got[:, v] - ref[:, v]).max() <= 1e-12 * scale, k
        assert np.abs(after[k][:, v] - ref[:, v]).max() <= 1e-7 * scale, k
    prob.close()


@pytest.mark.parametrize("base", ["V", "F"])
@pytest.mark.parametrize("case", [(2, 3, 65, 4), (3, 2, 17, 2), (3, 2, 17, 5, "aniso"), (2, 3, 17, 2, "iso", "L"),
                                  (3, 3, 17, 2, "aniso", "L")])
def test_composite_cycle_iterates_match_oracle(emg, ctx, case, base):
    """Element by element: after 1, 2 and 5 composite cycles from the
    initial state, the GPU's composite unknowns (valid fine nodes, uncovered
    coarse nodes) equal the oracle's composite cycle iterates (base grid
    corrected by a V- or an F-cycle; one box per level, or two boxes per
    level forming an L)."""
    dim, levels, n, seed = case[:4]
    ap = synth.smooth_amr(dim=dim, levels=levels, n=n, seed=seed, kind=case[4] if len(case) > 4 else "iso",
                          shape=case[5] if len(case) > 5 else "box")
    comp = amr.from_problem(ap)
    masks = comp.unknown_masks()
    u = comp.initial()
    done = 0
    for ncyc in (1, 2, 5):
        while done < ncyc:
            u = comp.cycle(u, base=base)
            done += 1
        prob = emg.Problem.from_amr(ctx, ap)
        st = prob.solve(rtol=1e-30, max_cycles=ncyc, cycle=base, raise_on_error=False, check_every=1)
        assert st["cycles"] == ncyc
        ug = _gpu_solution(prob, len(ap.boxes) + 1)
        prob.close()
        scale = max(float(np.abs(b).max()) for b in u)
        diff = max(float(np.abs(np.where(m, a - b, 0.0)).max()) for a, b, m in zip(ug, u, masks)) / scale
        print(f"[gpu] composite iterate {case} base {base} after {ncyc} cycles: max rel diff {diff:.2e}", flush=True)
        assert diff <= 1e-11


@pytest.mark.parametrize("base", ["V", "F"])
def test_ellipsoid_eigenstrain_iterates_match_oracle(emg, ctx, base):
    """3D composite system with eigenstrain on every level (the Sec. 4.1
    ellipsoid on [-2, 2]^3, base 17^3, two fixed boxes, far-field Dirichlet
    faces): after 1, 2 and 5 composite cycles the GPU's composite unknowns
    equal the oracle's iterates element by element."""
    ap = synth.eshelby_ellipsoid_amr(n0=17, L=2.0, phys_boxes=[((-1.5,) * 3, (1.5,) * 3),
                                                               ((-1.25, -1.0, -0.75), (1.25, 1.0, 0.75))])
    comp = amr.from_problem(ap)
    masks = comp.unknown_masks()
    u = comp.initial()
    done = 0
    for ncyc in (1, 2, 5):
        while done < ncyc:
            u = comp.cycle(u, base=base)
            done += 1
        prob = emg.Problem.from_amr(ctx, ap)
        st = prob.solve(rtol=1e-30, max_cycles=ncyc, cycle=base, raise_on_error=False, check_every=1)
        assert st["cycles"] == ncyc
        ug = _gpu_solution(prob, len(ap.boxes) + 1)
        prob.close()
        scale = max(float(np.abs(b).max()) for b in u)
        diff = max(float(np.abs(np.where(m, a - b, 0.0)).max()) for a, b, m in zip(ug, u, masks)) / scale
        print(f"[gpu] ellipsoid composite iterate base {base} after {ncyc} cycles: max rel diff {diff:.2e}",
              flush=True)
        assert diff <= 1e-11


def test_eshelby_amr_efficiency_case(emg, ctx):
    """AMR-efficiency input (2D disc, base 33^2, two refined boxes; finest
    resolution that of a uniform 129^2 grid): the GPU composite solution
    satisfies the oracle's composite system, in the oracle's cycle count, and
    its base-grid values match the uniform finest-grid GPU solution to 2 %
    while solving 5x fewer nodes."""
    ap = synth.eshelby_amr_2d(n0=33, levels=3)
    comp = amr.from_problem(ap)
    _, hist = comp.solve(tol=1e-10, max_cycles=300)
    prob = emg.Problem.from_amr(ctx, ap)
    st = prob.solve(rtol=1e-10, max_cycles=300)
    u = _gpu_solution(prob, len(ap.boxes) + 1)
    prob.close()
    rel = comp.norm(comp.residual(u)) / comp.norm(comp.residual(comp.initial()))
    assert st["converged"] and rel <= 1.2e-10 and abs(st["cycles"] - (len(hist) - 1)) <= 1
    pu = synth.eshelby_uniform_2d(n0=33, levels=3)
    pf = emg.Problem.from_spec(ctx, pu)
    pf.solve(rtol=1e-10, max_cycles=300)
    uf = pf.displacement()[:, :, ::4, ::4]
    pf.close()
    diff = float(np.abs(u[0] - uf).max() / np.abs(uf).max())
    print(f"[gpu] eshelby AMR: cycles {st['cycles']} composite nodes {ap.composite_nodes()} vs {pu.nodes}, "
          f"base diff vs uniform {diff:.3e}", flush=True)
    assert diff <= 2e-2 and 5 * ap.composite_nodes() <= pu.nodes


def test_microstructure_amr_efficiency_case(emg, ctx):
    """Microstructure half of the AMR study at a small size (finest 129^2,
    base 33^2, two levels of blocks along the grain boundaries): the GPU
    composite solution satisfies the oracle's composite system to 1.2e-10 in
    the oracle's cycle count, and its base-grid values stay within 5 % of
    the uniform finest-grid GPU solution."""
    ap = synth.microstructure_amr_2d(129, 3)
    assert all(len(ap.level_boxes(k)) > 1 for k in (1, 2))
    comp = amr.from_problem(ap)
    _, hist = comp.solve(tol=1e-10, max_cycles=300)
    prob = emg.Problem.from_amr(ctx, ap)
    st = prob.solve(rtol=1e-10, max_cycles=300)
    u = _gpu_solution(prob, len(ap.boxes) + 1)
    prob.close()
    rel = comp.norm(comp.residual(u)) / comp.norm(comp.residual(comp.initial()))
    print(f"[gpu] microstructure AMR: boxes {[len(ap.level_boxes(k)) for k in (1, 2)]} cycles {st['cycles']} "
          f"(oracle {len(hist) - 1}) oracle rel residual {rel:.2e}", flush=True)
    assert st["converged"] and rel <= 1.2e-10 and abs(st["cycles"] - (len(hist) - 1)) <= 1
    pu = synth.microstructure_uniform_2d(129)
    pf = emg.Problem.from_spec(ctx, pu)
    pf.solve(rtol=1e-10, max_cycles=300)
    uf = pf.displacement()[:, :, ::4, ::4]
    pf.close()
    diff = float(np.abs(u[0] - uf).max() / np.abs(uf).max())
    print(f"[gpu] microstructure AMR vs uniform 129^2: base diff {diff:.3e}, nodes {ap.composite_nodes()} vs "
          f"{pu.nodes}", flush=True)
    assert diff <= 5e-2
