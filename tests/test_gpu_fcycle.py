"""F-cycles on the GPU (Sec. 3.1: the paper's solver cycle) against the
oracle's F-cycle: the FP64 solve takes the same number of cycles as the
oracle's and equals its iterate to 1e-10; FP64 and mixed solutions match the
oracle's converged solution to 1e-8 at residual 1e-10 (1e-11 with Neumann
faces, whose boundary rows the residual norm weighs little); graph replay
equals eager launches bit for bit; the composite AMR cycle with an F-cycle
on the base grid satisfies the oracle's composite system; batched and
served solves refuse F-cycles."""
import numpy as np
import pytest

import oracle
import synth
from oracle import amr

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


RTOL = {"random3d_neumann": 1e-11, "random2d_neumann_129": 1e-11}
CASES = {
    "inclusion2d_65": lambda: synth.inclusion_2d(n=65),
    "polycrystal_17": lambda: synth.polycrystal_3d(n=17, grains=8, seed=2002),
    "random3d_neumann": lambda: synth.random_problem(3, (17, 17, 17), ("neumann", "traction", "dirichlet", "neumann",
                                                                       "traction", "neumann"), "aniso", seed=11),
    "random2d_neumann_129": lambda: synth.random_problem(2, (129, 129), ("neumann", "neumann", "dirichlet", "traction",
                                                                         "periodic", "periodic"), "iso", seed=12,
                                                         with_body=True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fcycle_solve_matches_oracle(emg, ctx, name):
    spec = CASES[name]()
    print(f"[gpu] F-cycle {name} m={spec.m}", flush=True)
    ref10 = oracle.solve(spec, tol=1e-10, max_cycles=400, cycle="F")
    ref = oracle.solve(spec, tol=1e-13, max_cycles=400, cycle="F")
    g = oracle.Grid.of(spec)
    lift = np.where(oracle.dirichlet_mask(g), ref.rhs, 0.0)
    r0 = oracle.norm(g, oracle.residual(g, spec.C, lift, ref.rhs))
    prob = emg.Problem.from_spec(ctx, spec)
    st = prob.solve(rtol=1e-10, max_cycles=400, cycle="F")
    u = prob.displacement()
    it = float(np.linalg.norm(u - ref10.u) / np.linalg.norm(ref10.u))
    print(f"[gpu]   fp64 rtol 1e-10: cycles={st['cycles']} (oracle {ref10.cycles}) iterate diff={it:.2e}", flush=True)
    assert st["converged"] and st["cycles"] == ref10.cycles and it <= 1e-10
    rtol = RTOL.get(name, 1e-10)
    for prec in ("fp64", "mixed"):
        st = prob.solve(rtol=rtol, max_cycles=400, precision=prec, cycle="F")
        u = prob.displacement()
        err = float(np.linalg.norm(u - ref.u) / np.linalg.norm(ref.u))
        rel = oracle.norm(g, oracle.residual(g, spec.C, u, ref.rhs)) / r0
        print(f"[gpu]   {prec} rtol {rtol:.0e}: cycles={st['cycles']} rel_res={rel:.2e} err={err:.2e}", flush=True)
        assert st["converged"] and rel <= 1.2 * rtol and err <= 1e-8
    prob.close()


def test_fcycle_graph_and_eager_agree_bitwise(emg, ctx):
    spec = synth.random_problem(2, (65, 65), ("neumann", "neumann", "dirichlet", "traction", "periodic", "periodic"),
                                "iso", seed=12, with_body=True)
    out = []
    for use_graph in (1, 0):
        for prec in ("fp64", "mixed"):
            prob = emg.Problem.from_spec(ctx, spec)
            st = prob.solve(rtol=1e-10, use_graph=use_graph, check_every=3, precision=prec, cycle="F")
            out.append((st["cycles"], prob.displacement()))
            prob.close()
    for a, b in ((0, 2), (1, 3)):
        assert out[a][0] == out[b][0] and np.array_equal(out[a][1], out[b][1])


def test_amr_with_fcycle_base(emg, ctx):
    """Three-level AMR (two nested boxes over a 65^2 base with five
    multigrid levels) with an F-cycle on the base grid: the composite
    solution satisfies the oracle's composite system, in as many cycles as
    the oracle's composite cycle with the same base cycle."""
    ap = synth.smooth_amr(dim=2, levels=3, n=65, seed=4)
    comp = amr.from_problem(ap)
    prob = emg.Problem.from_amr(ctx, ap)
    for base in ("V", "F"):
        _, hist = comp.solve(tol=1e-10, max_cycles=300, base=base)
        st = prob.solve(rtol=1e-10, max_cycles=400, cycle=base)
        print(f"[gpu] AMR 65^2 + 2 boxes, base {base}: cycles={st['cycles']} (oracle {len(hist) - 1})", flush=True)
        assert st["converged"] and abs(st["cycles"] - (len(hist) - 1)) <= 1
    u = [prob.displacement()] + [prob.amr_displacement(k) for k in range(1, len(ap.boxes) + 1)]
    rel = comp.norm(comp.residual(u)) / comp.norm(comp.residual(comp.initial()))
    print(f"[gpu] AMR F base: cycles={st['cycles']} composite rel residual={rel:.2e}", flush=True)
    assert rel <= 1.2e-10
    # the same with the composite correction in FP32 (mixed precision)
    st = prob.solve(rtol=1e-10, max_cycles=400, cycle="F", precision="mixed")
    u = [prob.displacement()] + [prob.amr_displacement(k) for k in range(1, len(ap.boxes) + 1)]
    rel = comp.norm(comp.residual(u)) / comp.norm(comp.residual(comp.initial()))
    print(f"[gpu] AMR F base, mixed: cycles={st['cycles']} composite rel residual={rel:.2e}", flush=True)
    assert st["converged"] and abs(st["cycles"] - (len(hist) - 1)) <= 2 and rel <= 1.2e-10
    prob.close()


def test_batch_and_server_refuse_fcycles(emg, ctx):
    spec = synth.inclusion_2d(n=33)
    p = emg.Problem.from_spec(ctx, spec)
    with pytest.raises(emg.EmgError) as ei:
        emg.solve_batch([p], cycle="F")
    assert ei.value.status == emg.EMG_EINVAL
    p.close()
    with pytest.raises(emg.EmgError) as ei:
        emg.Server(ctx, max_slots=2, cycle="F")
    assert ei.value.status == emg.EMG_EINVAL
