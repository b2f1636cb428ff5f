"""Benchmark: solve DoF/s of the multigrid elasticity solve on one MI355X.

Workload (the headline): 3D Voronoi polycrystal, 257^3 nodes on [0,1]^3
(256 x 256 x 257 stored nodes, periodic x/y), 64 grains (seed 2003) with
uniformly random orientations of a cubic crystal (C11=1.68, C12=1.21,
C44=0.75), grain boundaries smoothed over about two cells, plus a stiff
sphere of radius 0.25 at the centre (moduli x3, isotropic eigenstrain 2e-3,
tanh edge over two cells); u=0 on z=0 and u=(0,0,1e-3) on z=1; plain FP64
V-cycles (damped Jacobi omega=2/3, 2 pre + 2 post sweeps) to relative
residual 1e-10, 50.1 M DoF.

A step is one whole solve with every input already resident in HBM: moduli,
eigenstrain and face data copied device-to-device into the problem (which
invalidates its hierarchy), hierarchy setup (coarse moduli, coarsest-level
inverse), right-hand side, V-cycles to 1e-10, and the stress field.  `value`
is DoF x steps / wall time of the timed steps.  The same steps are repeated
with the mixed-precision solve (FP32 V-cycle inside FP64 refinement, one and
two FP32 cycles per refinement step) and reported under "mixed" and
"mixed_inner2".  "accuracy" gives each result's relative displacement error
against an FP64 solve to 1e-13 whose residual the CPU oracle recomputes (in
the cpu_baseline leg).

Roofline: the dominant kernel is the finest-level FP64 Jacobi sweep; its
average duration is measured with HIP events on the problem's stream
(emg_kernel_time) right after the timed steps; its algorithmic bytes are
240 B per node (read u 3x8, C 21x8, f 3x8; write u 3x8).  `traffic` is the
HBM bytes per launch from the committed rocprofv3 counter summary, reported
only while the kernel sources are the ones the counters were taken on.

polycrystal129: the 129^3, 16-grain polycrystal (seed 2002) in FP64 and
mixed precision, with its variants: V(4,4) smoothing, F-cycles, two FP32
cycles per step, autotuned stencil passes and a phase-field style coupling
loop of warm-started re-solves.

inclusion257: the isotropic workload, a spherical inclusion (lambda, mu
doubled, eigenstrain 1e-3) in an isotropic matrix, 257^3 nodes, z = 0
clamped and the other faces traction-free, FP64 and mixed precision; its
finest-level sweep moves 88 B per node (u, lambda, mu, f, out) and runs on
the isotropic z-marching pass.

serving: a stream of 512 independent solve requests (3D spherical
inclusions and 8-32-grain polycrystals, 33^3 to 129^3 nodes, log-uniform
sizes, Poisson arrivals at 200 requests/s, seed 2005), each with an input of
its own seeded from its id, is submitted to a fresh continuous-batching
server (mixed precision to 1e-10): the cold pass allocates hierarchies and
captures graphs while it runs, the warm pass replays the arrivals on the
same server; reported are p50/p99 latency (submit to result), solves/s and
solve-DoF/s over the stream.

cpu_baseline: the CPU oracle (plain FP64 C + OpenMP, gcc -O3) on this host,
on a bounded sample of the headline workload: hierarchy setup, right-hand
side and one V-cycle on all host threads, the solve time scaled to the GPU's
cycle count (same algorithm, same count); the one-thread figure scales that
by the ratio of one fine-level Jacobi sweep over 16 planes of the workload
on one thread and on all threads.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=257, help="nodes per axis of the headline polycrystal")
    ap.add_argument("--grains", type=int, default=64)
    ap.add_argument("--seed", type=int, default=2003)
    ap.add_argument("--no-sphere", action="store_true", help="leave out the stiff eigenstrained sphere")
    ap.add_argument("--cpu", type=int, default=1, help="run the CPU-oracle baseline leg (0 = skip)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--small", type=int, default=1, help="run the 129^3 polycrystal block (0 = skip)")
    ap.add_argument("--small-steps", type=int, default=10)
    ap.add_argument("--serve-requests", type=int, default=512, help="served stream length (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-slots", type=int, default=32, help="concurrent requests on the GPU")
    ap.add_argument("--serve-light-rate", type=float, default=40.0,
                    help="arrival rate of a second, shorter served stream below the GPU's capacity (0 = skip)")
    ap.add_argument("--serve-light-requests", type=int, default=160)
    ap.add_argument("--serve-nu", type=int, default=6, help="pre/post Jacobi sweeps per level of the served solves "
                    "(the served stream fixes no sweep count; V(6,6) serves the most solves/s of V(3,3) to "
                    "V(10,10))")
    ap.add_argument("--serve-inner", type=int, default=2, help="FP32 cycles per FP64 refinement step of the "
                    "served solves")
    ap.add_argument("--serve-check-every", type=int, default=1,
                    help="refinement steps per graph replay of the served batch (admission and retirement "
                         "happen between replays)")
    ap.add_argument("--amr", type=int, default=1, help="run the AMR blocks (0 = skip)")
    ap.add_argument("--amr-blocks", default="efficiency,microstructure,penny",
                    help="which AMR blocks to run (comma list of efficiency, microstructure, penny)")
    ap.add_argument("--iso", type=int, default=257, help="nodes per axis of the isotropic-inclusion block (0 = skip)")
    ap.add_argument("--iso-steps", type=int, default=5)
    ap.add_argument("--headline", type=int, default=1,
                    help="run the headline polycrystal (0: only the other blocks asked for, e.g. to profile them)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only set up the workload, time the finest-level sweeps and a 512 MiB device copy "
                         "(used for hardware-counter runs)")
    return ap.parse_args()


def _sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("emg_device.hpp", "emg_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2001_04789_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sweep_traffic(name):
    """HBM bytes per launch of the finest-level FP64 sweep from the committed
    rocprofv3 counter summary profiles/<name> (FETCH_SIZE/WRITE_SIZE scaled by
    a 512 MiB copy), or None when the kernel sources changed since the
    counters were taken."""
    prof = os.path.join(ROOT, "profiles", name)
    vals = {}
    if os.path.exists(prof):
        for line in open(prof):
            k, _, v = line.strip().partition(": ")
            if k in ("sources_sha256", "fp64_sweep_traffic_bytes"):
                vals[k] = v
    if vals.get("sources_sha256") != _sources_sha() or "fp64_sweep_traffic_bytes" not in vals:
        return None
    return int(vals["fp64_sweep_traffic_bytes"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, gpu_cycles, u_ref=None):
    """The oracle on this host's cores, on a bounded sample of the headline
    workload: hierarchy setup, right-hand side and one V-cycle with every
    thread (solve time = setup + rhs + cycles x one cycle), and one
    fine-level Jacobi sweep over 16 planes of the workload with one thread
    and with every thread (the one-thread estimate scales the all-thread
    cycle by that ratio).  With u_ref, the oracle's relative residual of that
    displacement (the accuracy reference of the GPU results)."""
    import numpy as np
    import oracle
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    g = oracle.Grid.of(spec)
    H = oracle.Hierarchy(g, spec.C)
    f = oracle.rhs(g, H.C[0], spec.eps0, spec.b, spec.face)
    u = np.where(oracle.dirichlet_mask(g), f, 0.0)
    t1 = time.perf_counter()
    r0 = oracle.norm(g, oracle.residual(g, H.C[0], u, f))
    t2 = time.perf_counter()
    u = oracle.vcycle(H, 0, u, f)
    t3 = time.perf_counter()
    per_cycle = (t3 - t2) + (t2 - t1)          # a cycle plus its convergence check
    est = (t1 - t0) + gpu_cycles * per_cycle
    out = {"value": spec.dofs() / est, "unit": "DoF/s", "cores": threads, "kind": "oracle",
           "sample": f"hierarchy setup + rhs + 1 V-cycle + residual norm of the full {spec.n[0]}^3 workload on "
                     f"{threads} threads ({t3 - t0:.1f} s), solve time scaled to the GPU's {gpu_cycles} cycles; "
                     f"one-thread figure from a fine-level Jacobi sweep over 16 planes on 1 and {threads} threads",
           "cpu_model": cpu_model(), "build": "gcc " + " ".join(oracle.build_flags()),
           "seconds_per_cycle": per_cycle, "setup_seconds": t1 - t0}
    # one fine-level sweep over a 16-plane slab, 1 thread vs all threads
    nz = 16
    gs = oracle.Grid(g.dim, (g.m[0], g.m[1], nz), g.h, g.bc, g.kind)
    Cs = np.ascontiguousarray(H.C[0][:, :nz])
    fs = np.ascontiguousarray(f[:, :nz])
    us = np.ascontiguousarray(u[:, :nz])
    t = {}
    for th in (threads, 1):
        oracle.set_threads(th)
        ta = time.perf_counter()
        oracle.jacobi(gs, Cs, us, fs, 2.0 / 3.0)
        t[th] = time.perf_counter() - ta
    oracle.set_threads(threads)
    ratio = t[1] / t[threads]
    est1 = est * ratio
    out["one_thread"] = {"value": spec.dofs() / est1, "unit": "DoF/s", "cores": 1,
                         "sweep_ratio_1_vs_all": ratio, "slab_sweep_seconds": {"1": t[1], str(threads): t[threads]}}
    if u_ref is not None:
        ta = time.perf_counter()
        rr = oracle.norm(g, oracle.residual(g, H.C[0], u_ref, f))
        out["reference_check"] = {"oracle_rel_res_of_reference": rr / r0, "seconds": time.perf_counter() - ta}
    return out


def solve_block(emg, torch, ctx, args, spec, steps, warmup, with_variants):
    """FP64 and mixed-precision timed steps (inputs resident in HBM) of one
    3D workload (anisotropic polycrystal or isotropic inclusion), the
    finest-level sweep timings, and optionally the variants (V(4,4),
    F-cycles, autotuning, coupling loop)."""
    import numpy as np
    import synth
    dev = "cuda:0"
    prob = emg.Problem(ctx, spec.dim, spec.n, spec.lo, spec.hi, spec.bc, spec.kind)
    C_d = torch.from_numpy(spec.C).to(dev)
    E_d = None if spec.eps0 is None else torch.from_numpy(spec.eps0).to(dev)
    faces_d = {f: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for f, v in spec.face.items()}
    sigma_d = torch.empty((6,) + spec.C.shape[1:], dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def step(precision, **kw):
        prob.set_moduli(C_d)
        prob.set_eigenstrain(E_d)
        for f in (4, 5):
            prob.set_face(f, faces_d.get(f))
        st = prob.solve(rtol=1e-10, max_cycles=400, precision=precision, **kw)
        prob.stress(out=sigma_d)
        return st

    def timed(precision, **kw):
        for _ in range(warmup):
            step(precision, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = [step(precision, **kw) for _ in range(steps)]
        torch.cuda.synchronize()
        return time.perf_counter() - t0, stats

    def summary(dt, sts, dofs):
        return {"value": dofs * steps / dt, "ms_per_step": 1e3 * dt / steps,
                "cycles": sts[-1]["cycles"], "rel_res": sts[-1]["rel_res"], "conv_factor": sts[-1]["conv_factor"],
                "solve_only_dofs_per_s": dofs / np.mean([s["solve_seconds"] for s in sts]),
                "solve_ms": 1e3 * float(np.mean([s["solve_seconds"] for s in sts])),
                "setup_ms": 1e3 * float(np.mean([s["setup_seconds"] for s in sts]))}

    out = {}
    dt64, st64 = timed("fp64")
    dofs = st64[0]["dofs"]
    u64 = prob.displacement()
    out["fp64"] = summary(dt64, st64, dofs)
    out["dofs"] = dofs
    out["nodes"] = spec.nodes
    out["levels"] = prob.num_levels()
    ms = prob.kernel_time(0, level=0, precision="fp64", reps=args.kernel_reps)
    nzc = prob.level_zmarch(0, "fp64")
    # algorithmic bytes per node of a sweep: read u, C, f, write u (FP64)
    bpn = 240 if spec.kind == "aniso" else 88
    kind = "ANISO" if spec.kind == "aniso" else "ISO"
    out["sweep"] = {"kernel": ("k_stencil_zm<double,JACOBI,%s> finest level (z-marching pass, %d chunks per column)"
                               % (kind, nzc) if nzc else "k_stencil<3,%s,double,JACOBI> finest level" % kind),
                    "fp64_ms": ms, "fp64_bytes": bpn * spec.nodes}
    sols = {"fp64": u64}
    if not args.no_mixed:
        out["sweep"]["fp32_ms"] = prob.kernel_time(0, level=0, precision="mixed", reps=args.kernel_reps)
        out["sweep"]["fp32_bytes"] = bpn // 2 * spec.nodes
        out["sweep"]["fp32_gbs"] = bpn // 2 * spec.nodes / (out["sweep"]["fp32_ms"] * 1e-3) / 1e9
        dt32, st32 = timed("mixed")
        out["mixed"] = summary(dt32, st32, dofs)
        out["mixed"]["speedup_vs_fp64_step"] = dt64 / dt32
        sols["mixed"] = prob.displacement()
        dti, sti = timed("mixed", inner_cycles=2)
        out["mixed_inner2"] = summary(dti, sti, dofs)
        out["mixed_inner2"]["speedup_vs_fp64_step"] = dt64 / dti
        sols["mixed_inner2"] = prob.displacement()
    # accuracy reference: FP64 to 1e-13 (its oracle residual is taken in the cpu_baseline leg)
    prob.set_moduli(C_d)
    prob.set_eigenstrain(E_d)
    ref = prob.solve(rtol=1e-13, max_cycles=600, precision="fp64")
    u_ref = prob.displacement()
    nrm = float(np.linalg.norm(u_ref))
    out["accuracy"] = {"reference": "FP64 GPU solve to rel. residual 1e-13 (%d cycles, %.2e)" % (ref["cycles"],
                                                                                              ref["rel_res"]),
                       "rel_err_vs_reference": {k: float(np.linalg.norm(v - u_ref)) / nrm for k, v in sols.items()}}
    if not with_variants:
        prob.close()
        return out, u_ref
    # the same FP64 step with the inputs handed over from host memory (PCIe-inclusive)
    def host_step():
        prob.set_moduli(spec.C)
        prob.set_eigenstrain(spec.eps0)
        for f in (4, 5):
            prob.set_face(f, spec.face.get(f))
        st = prob.solve(rtol=1e-10, max_cycles=400, precision="fp64")
        prob.stress(out=sigma_d)
        return st
    host_step()
    torch.cuda.synchronize()
    th = time.perf_counter()
    for _ in range(2):
        host_step()
    torch.cuda.synchronize()
    out["fp64"]["host_inputs_ms_per_step"] = 1e3 * (time.perf_counter() - th) / 2
    precs = ("fp64",) + (() if args.no_mixed else ("mixed",))

    def solve_twice(prec, **kw):
        sts = []
        for _ in range(2):
            prob.set_moduli(C_d)
            sts.append(prob.solve(rtol=1e-10, max_cycles=400, precision=prec, **kw))
        return {"cycles": sts[-1]["cycles"], "solve_ms": 1e3 * sts[-1]["solve_seconds"],
                "solve_only_dofs_per_s": dofs / sts[-1]["solve_seconds"]}
    out["smoothing_v44"] = {p: solve_twice(p, nu1=4, nu2=4) for p in precs}
    out["fcycle"] = {p: solve_twice(p, cycle="F") for p in precs}
    nlev = prob.num_levels()
    tun = {"plans_cost_model": {p: [prob.level_zmarch(l, p) for l in range(nlev)] for p in precs}}
    t0 = time.perf_counter()
    tun["levels_tuned"] = {p: prob.autotune(p, reps=10, retune=True) for p in precs}
    tun["tune_seconds"] = time.perf_counter() - t0
    tun["plans_tuned"] = {p: [prob.level_zmarch(l, p) for l in range(nlev)] for p in precs}
    tun["tiles_tuned"] = {p: [list(prob.level_tiles(l, p)) for l in range(nlev)] for p in precs}
    tun["tile_codes"] = "per level [stencil, restriction, interpolation]: 0 = 64x4, 1 = 64x2, 2 = 128x2, 3 = 32x8"
    for p in precs:
        tun[p] = solve_twice(p)
    emg.autotune_reset()
    out["autotuned"] = tun
    # phase-field style coupling loop: a precipitate grows over 6 steps; each
    # step re-sets moduli and eigenstrain and solves warm-started from the
    # previous displacement, beside a cold solve of the same step
    loop = {"steps": 6, "precision": "fp64", "warm_cycles": [], "cold_cycles": [], "warm_ms": 0.0, "cold_ms": 0.0,
            "von_mises_max": []}
    vm_d = torch.empty((1,) + spec.C.shape[1:], dtype=torch.float64, device=dev)
    u_prev = None
    for t in range(6):
        sp = synth.precipitate_step(spec, t, 6)
        Ct = torch.from_numpy(sp.C).to(dev)
        Et = torch.from_numpy(sp.eps0).to(dev)
        for warm in (0, 1):
            if warm and t:
                prob.set_displacement(u_prev)
            prob.set_moduli(Ct)
            prob.set_eigenstrain(Et)
            st = prob.solve(rtol=1e-10, max_cycles=400, warm_start=warm if t else 0)
            key = "warm" if warm else "cold"
            loop[key + "_cycles"].append(st["cycles"])
            loop[key + "_ms"] += 1e3 * st["solve_seconds"]
        u_prev = torch.from_numpy(prob.displacement()).to(dev)
        prob.von_mises(out=vm_d)
        loop["von_mises_max"].append(float(vm_d.max()))
        del Ct, Et
    loop["warm_over_cold_time"] = loop["warm_ms"] / loop["cold_ms"]
    out["coupling_loop"] = loop
    prob.close()
    return out, u_ref


def iso_block(emg, torch, ctx, args, synth):
    """The isotropic workload: a spherical inclusion with eigenstrain in an
    isotropic matrix, FP64 and mixed precision (finest level on the
    isotropic z-marching pass)."""
    spec = synth.inclusion_3d(n=args.iso, seed=2004)
    blk, _ = solve_block(emg, torch, ctx, args, spec, args.iso_steps, 1, with_variants=False)
    blk["workload"] = (f"isotropic spherical inclusion {args.iso}^3 nodes (seed 2004): matrix lambda 1.5, mu 1; "
                       f"inclusion r=0.25 with lambda 3, mu 2 and eigenstrain 1e-3; z=0 clamped, other faces "
                       f"traction-free; V(2,2) to rel. residual 1e-10")
    sw = blk["sweep"]
    blk["roofline_frac"] = sw["fp64_bytes"] / (sw["fp64_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS
    return blk


def serving_pool(torch, count):
    """Device-resident inputs of the served stream: every request's own input
    (seeded from its id), generated in parallel on the host and uploaded."""
    import types
    import numpy as np
    import synth
    trace = synth.serving_trace(count=count, seed=2005, rate=200.0, variants=0)
    dev = "cuda:0"
    pool = {}
    t0 = time.perf_counter()
    for key, sp in synth.serving_inputs(trace, workers=min(16, os.cpu_count() or 1)):
        d = types.SimpleNamespace(dim=sp.dim, n=sp.n, lo=sp.lo, hi=sp.hi, bc=sp.bc, kind=sp.kind, m=sp.m,
                                  C=torch.from_numpy(sp.C).to(dev),
                                  eps0=None if sp.eps0 is None else torch.from_numpy(sp.eps0).to(dev),
                                  b=None if sp.b is None else torch.from_numpy(sp.b).to(dev),
                                  face={f: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
                                        for f, v in (sp.face or {}).items() if v is not None})
        pool[key] = (d, sp.dofs())
    torch.cuda.synchronize()
    return pool, time.perf_counter() - t0


def serve(emg, torch, ctx, args, count, rate, pool, gen_s):
    """Served stream (continuous batching) of `count` requests with inputs of
    their own, on a fresh server: the first pass is cold (every domain shape's
    hierarchy allocated and its batch graphs captured while the stream runs),
    the second replays the same arrivals on the same server (hierarchies
    resident, graphs cached).  Latencies from the server's clock."""
    import numpy as np
    import synth
    trace = synth.serving_trace(count=count, seed=2005, rate=rate, variants=0)
    dev = "cuda:0"

    def out_for(d):
        return torch.empty((d.dim,) + tuple(d.m[::-1]), dtype=torch.float64, device=dev)

    outs = [out_for(pool[(r.kind, r.n, r.variant)][0]) for r in trace]
    torch.cuda.synchronize()
    srv = emg.Server(ctx, max_slots=args.serve_slots, rtol=1e-10, max_cycles=400, precision="mixed",
                     nu1=args.serve_nu, nu2=args.serve_nu, inner_cycles=args.serve_inner,
                     check_every=args.serve_check_every)
    passes = {}
    for name in ("cold", "warm"):
        base = srv.now()
        tickets = []
        for i, r in enumerate(trace):
            while srv.now() - base < r.t:
                time.sleep(min(1e-4, max(0.0, r.t - (srv.now() - base))))
            tickets.append(srv.submit(pool[(r.kind, r.n, r.variant)][0], out=outs[i]))
        infos = [srv.wait(t)[1] for t in tickets]
        bad = [i for i in infos if i["status"] != 0 or not i["converged"]]
        lat = np.array([i["t_done"] - i["t_submit"] for i in infos])
        qwait = np.array([i["t_admit"] - i["t_submit"] for i in infos])
        prep = np.array([i["t_ready"] - i["t_admit"] for i in infos])
        span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
        dofs = sum(pool[(r.kind, r.n, r.variant)][1] for r in trace)
        passes[name] = {"failed": len(bad), "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                        "p99_ms": 1e3 * float(np.percentile(lat, 99)), "mean_ms": 1e3 * float(lat.mean()),
                        "queue_p50_ms": 1e3 * float(np.percentile(qwait, 50)),
                        "prep_mean_ms": 1e3 * float(prep.mean()), "prep_max_ms": 1e3 * float(prep.max()),
                        "solves_per_s": len(trace) / span, "served_dofs_per_s": dofs / span, "span_s": span,
                        "mean_cycles": float(np.mean([i["cycles"] for i in infos]))}
    srv.close()
    out = {"requests": len(trace), "rate_req_per_s": rate, "slots": args.serve_slots, "precision": "mixed",
           "smoothing": f"V({args.serve_nu},{args.serve_nu})", "inner_cycles": args.serve_inner,
           "check_every": args.serve_check_every,
           "offered_span_s": trace[-1].t,
           "inputs": f"{len(trace)} distinct inputs seeded from the request ids, resident in HBM "
                     f"(pool generated in {gen_s:.0f} s on the host)",
           "domain_shapes": len({(r.kind, r.n) for r in trace})}
    out.update(passes["cold"])
    out["warm"] = passes["warm"]
    return out


def amr_efficiency(emg, ctx, synth, n0=129, levels=(2, 3, 4, 5, 6)):
    """AMR against the uniform grid of the same finest resolution (the 2D
    disc of inclusion_2d, refined boxes around it): composite and uniform node
    counts, FP64 solve times to 1e-10 (second solve of each, after setup),
    and the largest difference of the AMR base-grid displacement from the
    uniform solution at the same points."""
    import numpy as np
    rows = []
    for L in levels:
        ap = synth.eshelby_amr_2d(n0, L)
        pu = synth.eshelby_uniform_2d(n0, L)
        pa = emg.Problem.from_amr(ctx, ap)
        pf = emg.Problem.from_spec(ctx, pu)
        sa = [pa.solve(rtol=1e-10, max_cycles=400) for _ in range(2)][-1]
        su = [pf.solve(rtol=1e-10, max_cycles=400) for _ in range(2)][-1]
        s = 2 ** (L - 1)
        ub, uf = pa.displacement(), pf.displacement()[:, :, ::s, ::s]
        rows.append({"levels": L, "finest_nodes_per_axis": pu.n[0], "composite_nodes": ap.composite_nodes(),
                     "uniform_nodes": pu.nodes, "node_ratio": ap.composite_nodes() / pu.nodes,
                     "amr_cycles": sa["cycles"], "uniform_cycles": su["cycles"],
                     "amr_solve_ms": 1e3 * sa["solve_seconds"], "uniform_solve_ms": 1e3 * su["solve_seconds"],
                     "speedup": su["solve_seconds"] / sa["solve_seconds"],
                     "base_rel_diff_vs_uniform": float(np.abs(ub - uf).max() / np.abs(uf).max())})
        pa.close()
        pf.close()
    return {"workload": f"2D disc r=0.1 (inclusion_2d moduli), base {n0}^2, boxes around the disc", "rows": rows}


def amr_microstructure(emg, ctx, synth, n_finest=2049, levels=(2, 3, 4, 5)):
    """The microstructure half of the AMR performance study: a 10-grain 2D
    polycrystal, refined where some |grad eta| |dx| > 0.1 with 16/32-cell
    blocks at a fixed finest resolution of n_finest nodes per axis, against
    the uniform grid at that resolution (levels = 1).  FP64 solves to 1e-10
    (second solve of each, after setup): nodes, cycles, solve times, and the
    largest difference of the AMR base-grid displacement from the uniform
    solution at the same points."""
    import numpy as np
    pu = synth.microstructure_uniform_2d(n_finest)
    pf = emg.Problem.from_spec(ctx, pu)
    su = [pf.solve(rtol=1e-10, max_cycles=400) for _ in range(2)][-1]
    uu = pf.displacement()
    pf.close()
    rows = []
    for L in levels:
        ap = synth.microstructure_amr_2d(n_finest, L)
        pa = emg.Problem.from_amr(ctx, ap)
        sa = [pa.solve(rtol=1e-10, max_cycles=400) for _ in range(2)][-1]
        s = 2 ** (L - 1)
        ub, uf = pa.displacement(), uu[:, :, ::s, ::s]
        rows.append({"levels": L, "base_nodes_per_axis": ap.base.n[0],
                     "boxes_per_level": [len(ap.level_boxes(k)) for k in range(1, len(ap.boxes) + 1)],
                     "composite_nodes": ap.composite_nodes(), "uniform_nodes": pu.nodes,
                     "node_ratio": ap.composite_nodes() / pu.nodes, "amr_cycles": sa["cycles"],
                     "uniform_cycles": su["cycles"], "amr_solve_ms": 1e3 * sa["solve_seconds"],
                     "uniform_solve_ms": 1e3 * su["solve_seconds"],
                     "speedup": su["solve_seconds"] / sa["solve_seconds"],
                     "base_rel_diff_vs_uniform": float(np.abs(ub - uf).max() / np.abs(uf).max())})
        pa.close()
    return {"workload": f"2D 10-grain cubic polycrystal (seed 2010), GB width 4 finest cells, finest "
                        f"{n_finest}^2, bottom clamped, top sheared 1e-3", "rows": rows}


def amr_penny_crack(emg, ctx, synth):
    """The diffuse penny crack on a 65^3 base, three levels of 16/32-cell
    blocks where |grad eta| h > 0.1 (reflux-free composite system), FP64 and
    mixed precision to 1e-10 (second solve of each, after setup); composite
    DoF/s and the mixed solution's difference from the FP64 one."""
    import numpy as np
    ap = synth.penny_crack(n=65, levels=3, floor=1e-2, width=0.01)
    prob = emg.Problem.from_amr(ctx, ap)
    out = {"workload": "penny crack R=0.2, width 0.01, moduli floor 1e-2 (the 1 % cap), base 65^3 nodes, "
                       "3 levels of 16/32-cell blocks tagged where |grad eta| h > 0.1",
           "boxes_per_level": [len(ap.level_boxes(k)) for k in range(1, len(ap.boxes) + 1)],
           "bounding_boxes": [[list(lo), list(hi)] for lo, hi in ap.boxes], "composite_nodes": ap.composite_nodes()}
    sols = {}
    for prec in ("fp64", "mixed"):
        st = [prob.solve(rtol=1e-10, max_cycles=400, precision=prec) for _ in range(2)][-1]
        sols[prec] = [prob.displacement()] + [prob.amr_displacement(k) for k in range(1, len(ap.boxes) + 1)]
        out[prec] = {"cycles": st["cycles"], "rel_res": st["rel_res"], "solve_ms": 1e3 * st["solve_seconds"],
                     "dofs": st["dofs"], "dofs_per_s": st["dofs"] / st["solve_seconds"]}
    num = sum(float(np.sum((a - b) ** 2)) for a, b in zip(sols["mixed"], sols["fp64"]))
    den = sum(float(np.sum(b ** 2)) for b in sols["fp64"])
    out["mixed_rel_diff_vs_fp64"] = float(np.sqrt(num / den))
    out["mixed_speedup"] = out["fp64"]["solve_ms"] / out["mixed"]["solve_ms"]
    prob.close()
    return out


def amr_blocks(emg, ctx, synth, args):
    pick = set(args.amr_blocks.split(","))
    out = {}
    if "efficiency" in pick:
        out["amr_efficiency"] = amr_efficiency(emg, ctx, synth)
    if "microstructure" in pick:
        out["amr_microstructure"] = amr_microstructure(emg, ctx, synth)
    if "penny" in pick:
        out["amr_penny_crack"] = amr_penny_crack(emg, ctx, synth)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solve is single-GPU", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import synth
    import paper_2001_04789_amd as emg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if not args.headline:
        ctx = emg.Context(0)
        out = {"headline": "skipped"}
        if args.iso:
            out[f"inclusion{args.iso}"] = iso_block(emg, torch, ctx, args, synth)
        if args.amr:
            out.update(amr_blocks(emg, ctx, synth, args))
        ctx.close()
        print(json.dumps(out), flush=True)
        return
    t_gen = time.perf_counter()
    spec = synth.polycrystal_3d(n=args.n, grains=args.grains, seed=args.seed,
                                inclusion=None if args.no_sphere else (3.0, 2e-3))
    gen_s = time.perf_counter() - t_gen
    print(f"[bench] input {spec.name}: {spec.nodes} nodes, generated in {gen_s:.1f} s", file=sys.stderr, flush=True)
    ctx = emg.Context(0)
    dev = "cuda:0"

    if args.kernel_only:
        prob = emg.Problem.from_spec(ctx, spec)
        st = prob.solve(rtol=1e-10, max_cycles=400, precision="mixed")
        ms64 = prob.kernel_time(0, level=0, precision="fp64", reps=args.kernel_reps)
        ms32 = prob.kernel_time(0, level=0, precision="mixed", reps=args.kernel_reps)
        src = torch.empty(64 * 2 ** 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(args.kernel_reps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only": True, "workload": spec.name, "cycles": st["cycles"], "sweep_fp64_ms": ms64,
                          "sweep_fp32_ms": ms32, "nodes": spec.nodes, "copy_bytes": 2 * src.numel() * 8,
                          "copy_reps": args.kernel_reps}))
        return

    head, u_ref = solve_block(emg, torch, ctx, args, spec, args.steps, args.warmup, with_variants=False)
    print(f"[bench] headline done: FP64 {head['fp64']['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)
    dofs = head["dofs"]
    sw = head["sweep"]
    achieved = sw["fp64_bytes"] / (sw["fp64_ms"] * 1e-3) / 1e9
    sphere = "" if args.no_sphere else " + stiff sphere r=0.25 (moduli x3, eigenstrain 2e-3)"
    out = {
        "metric": "solve DoF/s at rel. residual 1e-10 (FP64 vs mixed); served p50/p99 latency",
        "value": head["fp64"]["value"],
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["fp64"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"polycrystal {args.n}^3 nodes, {args.grains} grains (seed {args.seed}){sphere}, "
                               f"periodic x/y, uniaxial z displacement 1e-3, FP64 V(2,2) damped Jacobi to rel. "
                               f"residual 1e-10; mixed = FP32 V-cycles in FP64 refinement",
                   "nodes": head["nodes"], "dofs": dofs, "levels": head["levels"],
                   "step": "setup + rhs + solve + stress, inputs resident in HBM",
                   "input_generation_s": gen_s},
        "fp64": head["fp64"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": sweep_traffic(f"jacobi_sweep_polycrystal{args.n}_counters.md"),
                     "kernel": sw["kernel"], "avg_ms": sw["fp64_ms"], "bytes_per_launch": sw["fp64_bytes"]},
    }
    for k in ("mixed", "mixed_inner2", "accuracy"):
        if k in head:
            out[k] = head[k]
    if "fp32_ms" in sw:
        out["fp32_sweep"] = {"avg_ms": sw["fp32_ms"], "gbs": sw["fp32_gbs"], "bytes_per_launch": sw["fp32_bytes"]}
    if args.small:
        small = synth.polycrystal_3d(n=129, grains=16, seed=2002)
        blk, _ = solve_block(emg, torch, ctx, args, small, args.small_steps, 2, with_variants=True)
        blk["workload"] = "polycrystal 129^3 nodes, 16 grains (seed 2002), periodic x/y, uniaxial z 1e-3"
        blk["roofline_frac"] = blk["sweep"]["fp64_bytes"] / (blk["sweep"]["fp64_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS
        blk["traffic"] = sweep_traffic("jacobi_sweep_polycrystal129_counters.md")
        out["polycrystal129"] = blk
        print("[bench] 129^3 block done", file=sys.stderr, flush=True)
    if args.iso:
        out[f"inclusion{args.iso}"] = iso_block(emg, torch, ctx, args, synth)
        print("[bench] isotropic block done", file=sys.stderr, flush=True)
    if args.amr:
        out.update(amr_blocks(emg, ctx, synth, args))
        print("[bench] AMR blocks done", file=sys.stderr, flush=True)
    nserve = max(args.serve_requests, args.serve_light_requests if args.serve_light_rate > 0 else 0)
    if nserve > 0:
        pool, gen_s = serving_pool(torch, nserve)
        if args.serve_requests > 0:
            out["serving"] = serve(emg, torch, ctx, args, args.serve_requests, args.serve_rate, pool, gen_s)
        if args.serve_light_rate > 0 and args.serve_light_requests > 0:
            # the same request mix offered below the GPU's capacity: latency without the queue
            out["serving_light"] = serve(emg, torch, ctx, args, args.serve_light_requests, args.serve_light_rate,
                                         pool, gen_s)
        del pool
    print("[bench] serving done", file=sys.stderr, flush=True)
    ctx.close()
    if args.cpu:
        out["cpu_baseline"] = cpu_baseline(spec, out["fp64"]["cycles"], u_ref)
        chk = out["cpu_baseline"].pop("reference_check", None)
        if chk and "accuracy" in out:
            out["accuracy"]["reference_oracle_rel_res"] = chk["oracle_rel_res_of_reference"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
