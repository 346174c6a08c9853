"""Benchmark: Picard-step linear solve to an exact relative residual of 1e-8.

Workload (default): the 64x192 symmetric-step grid (h = 1/16, n_u = 50,368,
n_p = 6,641), m = 4 uniform random variables with coefficients 1/k^2,
Legendre chaos of degree 3 (n_xi = 35), n_t = 128 backward-Euler steps of
tau = 0.05 -- 255.4 M unknowns in the all-at-once system.  One step = one
sgtt_solve of the first Picard-step system (the Stokes system of Alg. 3.1)
to ||b - L x|| <= 1e-8 ||b||, inputs resident on the GPU.

Prints ONE JSON line.  value = solves per second (whole job, one GPU).
One profiled solve after the warm-up gives the per-class and per-phase
breakdown and the dominant kernel class (largest event time).  During the
timed steps only that class is evented; the roofline object reports its
algorithmic bytes (or flops) per launch divided by its average launch
duration over the timed region.  cpu_baseline times the CPU oracle on a bounded
sample of the same solve (the first outer iterations within a time budget),
scaled to solves per second with the GPU's outer-iteration count.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (and FP64 matrix) peak


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--outer-explicit", type=int, default=1,
                    help="1: Alg. 4.2 literally (z_k, s_k every outer iteration); 0: least-squares estimate")
    ap.add_argument("--restart", type=int, default=20)
    ap.add_argument("--relax", type=int, default=1,
                    help="1: relaxed truncation of late Krylov vectors (inexact Krylov); 0: fixed eps of Alg. 4.2")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU baseline budget: the oracle stops after the first outer iteration that ends past it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", type=int, default=0)
    ap.add_argument("--precision", type=int, default=0, choices=[0, 1, 2, 3],
                    help="velocity block: 0 FP64, 1 FP32, 2 BF16, 3 FP32 where the residual allows it")
    ap.add_argument("--inner-mode", type=int, default=1,
                    help="velocity block of the preconditioner: 1 time-stepped mean solve on the full tensor, "
                         "0 inner low-rank GMRES with M (eq. 5.22-5.23)")
    ap.add_argument("--inner-rhs-eps", type=float, default=1e-2,
                    help="truncation of the inner GMRES right-hand side (inner mode 0)")
    ap.add_argument("--batch", type=int, default=0,
                    help="N > 0: instead, time N independent problems (batch_configs) on --contexts streams")
    ap.add_argument("--contexts", type=int, default=8)
    ap.add_argument("--batch-small", action="store_true", help="coarse grids / short horizons for the batch")
    ap.add_argument("--jsonl", default="",
                    help="append one JSON line per timed solve (stats, residual and rank history) to this file")
    ap.add_argument("--event-sample", type=int, default=8,
                    help="in the timed region, bracket one scope of the dominant kernel class in every N with "
                         "HIP events (a scope is one launch, or one spatial solve's passes)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="M > 0: before the timed solves, one device-to-device copy of M MiB (a plain copy kernel "
                         "of known size for scaling memory counters)")
    ap.add_argument("--progress", action="store_true", help="one line on stderr per solve")
    ap.add_argument("--system", default="stokes", choices=("stokes", "picard1"),
                    help="stokes: the first Picard system (w = 0, Alg. 3.1 line 1); picard1: the system of "
                         "Picard step 1, assembled around the Stokes solution (untimed) as the prior iterate")
    ap.add_argument("--compare", default="mixed_relaxed,graph",
                    help="comma list of solver variants timed after the main measurement with the same steps "
                         f"(names: {', '.join(sorted(VARIANTS))}; empty for none); the default times the "
                         "mixed-precision solve the metric compares with the plain FP64 one, and the plain "
                         "solve with the mean solve's time loop as a captured graph")
    ap.add_argument("--picard", type=int, default=0,
                    help="N > 0: instead, run Picard's method (Alg. 3.1) for N steps after the Stokes solve and print "
                         "the per-step record")
    ap.add_argument("--sweep", default="", choices=("",) + tuple(SWEEPS),
                    help="instead, run Picard's method with the paper's tolerances (Table 6.2) on the Table 6.1 "
                         "sizes, varying one parameter (sec. 6.3), and print ranks, storage ratio and times")
    return ap.parse_args(argv)


# the paper's stopping and truncation tolerances (Table 6.2, sec. 6.2):
# inexact Picard with tol_gmres = 1e-1, eps_gmres = 1e-3 for the outer and the
# inner (preconditioner) solves, eps_soln = 1e-7, eps_conv = 1e-3,
# tol_picard = 1e-5
PAPER_TOLERANCES = dict(solve=dict(tol=1e-1, eps_krylov=1e-3, tol_cycle=1e-1, inner_tol=1e-1, inner_eps=1e-3,
                                   max_cycles=4, restart=30, relax=0, outer_explicit=1, inner_mode=0),
                        eps_soln=1e-7, eps_conv=1e-3, eps_rhs=1e-3, tol_picard=1e-5, max_steps=10,
                        # the update truncated, the sum kept exact: the Gram-based rounding of the sum
                        # itself (update_mode 0, eq. 4.8 as written) leaves the nonlinear residual
                        # level at about 1.1e-5, just above tol_picard (the "floor" sweep)
                        update_mode=1)

# one-parameter variations of the Table 6.1 problem (sec. 6.3, Figs. 6.5-6.6);
# sigma is this build's relative viscosity amplitude nu_coef, h keeps the
# domain, tau keeps t_f = 1
SWEEPS = {
    "paper": [{}],
    "sigma": [dict(nu_coef=v) for v in (0.01, 0.03, 0.1)],
    "nu0": [dict(nu0=v) for v in (1 / 25, 1 / 50, 1 / 100)],
    "h": [dict(h=v) for v in (1 / 4, 1 / 8, 1 / 16)],
    "tau": [dict(tau=1 / n, nt=n) for n in (32, 64, 128)],
    # the paper's own problem: KL viscosity (sec. 6.1), Table 6.1 and 6.2
    "kl": [dict(base="paper_kl")],
    # Table 6.3: tighter GMRES tolerances with eps_gmres = 1e-2 tol_gmres
    "kl_tol": [dict(base="paper_kl", solve=dict(tol=t, tol_cycle=t, eps_krylov=1e-2 * t, inner_eps=1e-2 * t),
                    eps_rhs=1e-2 * t) for t in (1e-1, 1e-2, 1e-3)],
    # eq. 4.8 as written (the updated iterate rounded, update_mode 0): the
    # nonlinear residual levels off near 1.1e-5 whatever the truncation of
    # the iterate or of the convection field
    "floor": [dict(base="paper_kl", update_mode=0, eps_soln=e) for e in (1e-7, 1e-9)]
             + [dict(base="paper_kl", update_mode=0, eps_conv=1e-5)],
}


def storage_ratio(nt, nxi, n, ranks):
    """eq. 6.6: entries of a TT with ranks (k1, k2) over those of the full tensor."""
    k1, k2 = ranks
    return (nt * k1 + nxi * k1 * k2 + n * k2) / (nt * nxi * n)


def sweep_main(args):
    from paper_1906_06785_amd import sgtt
    from synthetic_inputs import CONFIGS

    ctx = sgtt.Context(0)
    tol = PAPER_TOLERANCES
    runs = []
    for over in SWEEPS[args.sweep]:
        over = dict(over)
        base = over.pop("base", "paper")
        solve = dict(tol["solve"], **over.pop("solve", {}))
        eps_rhs = over.pop("eps_rhs", tol["eps_rhs"])
        eps_soln = over.pop("eps_soln", tol["eps_soln"])
        eps_conv = over.pop("eps_conv", tol["eps_conv"])
        update_mode = over.pop("update_mode", tol["update_mode"])
        cfg = dict(CONFIGS[base], **over)
        hp = sgtt.HostProblem(cfg)
        t0 = time.perf_counter()
        x, st, rc = sgtt.picard(ctx, cfg, steps=tol["max_steps"], tol_picard=tol["tol_picard"],
                                eps_soln=eps_soln, eps_conv=eps_conv, eps_rhs=eps_rhs,
                                caps=OUT_CAPS, update_mode=update_mode, **solve)
        over.update(base=base, solve=solve, eps_rhs=eps_rhs, eps_soln=eps_soln, eps_conv=eps_conv,
                    update_mode=update_mode)
        el = time.perf_counter() - t0
        # ranks of the final iterate rounded at eps_soln (eq. 4.8); with
        # update_mode 1 the stored exact sum has the larger stored ranks
        ru, rp = tuple(st["rank_u"][-1]), tuple(st["rank_p"][-1])
        runs.append({"params": over, "n_t": hp.nt, "n_xi": hp.n_xi, "n_u": hp.n_u, "n_p": hp.n_p, "status": rc,
                     "picard_steps": st["steps"], "nonlinear_residual": st["nonlinear_residual"],
                     "gmres_iters": st["outer_iters"], "inner_iters": st["inner_iters"],
                     "rank_u": ru, "rank_p": rp, "rank_u_per_step": st["rank_u"], "rank_p_per_step": st["rank_p"],
                     "stored_rank_u": tuple(x.ranks[0]), "stored_rank_p": tuple(x.ranks[1]),
                     "storage_ratio_u": storage_ratio(hp.nt, hp.n_xi, hp.n_u, ru),
                     "storage_ratio_p": storage_ratio(hp.nt, hp.n_xi, hp.n_p, rp),
                     "seconds": el, "solve_seconds": st["solve_seconds"]})
        print(f"[sweep] {args.sweep} {over}: {st['steps']} Picard steps, ranks u {ru} p {rp}, {el:.1f} s",
              file=sys.stderr, flush=True)
    print(json.dumps({"metric": f"Picard's method with the paper's tolerances, {args.sweep} sweep",
                      "config": {"workload": "Table 6.1 sizes (h=1/4, m=3, degree 3, t_f=1, tau=1/64, nu0=1/50); "
                                             "base 'paper': this build's viscosity law, 'paper_kl': the KL "
                                             "viscosity of sec. 6.1 (b=4, sigma=0.01); one parameter varied",
                                 "tolerances": tol},
                      "runs": runs}), flush=True)


# solver variants that --compare can time next to the main configuration:
# option overrides of solve_options
VARIANTS = {
    "exact_mean": dict(inner_mode=1),
    "minv": dict(inner_mode=2),
    "inner_gmres": dict(inner_mode=0),
    "inner_gmres_f32": dict(inner_mode=0, precision=1),
    "inner_gmres_bf16": dict(inner_mode=0, precision=2),
    "pcd": dict(schur=1),
    "mixed_f32": dict(precision=1),
    "mixed_relaxed": dict(precision=3),
    "graph": dict(graph=1),
    "mixed_relaxed_graph": dict(precision=3, graph=1),
}

VELOCITY_BLOCK = {0: "inner low-rank GMRES on (F_0 + C) preconditioned by M (eq. 5.22-5.23)",
                  1: "time-stepped mean solve (F_0 + C)^-1 on the full velocity tensor, then TT-SVD",
                  2: "M^-1 of eq. 5.23 applied once (prefix sum in time, one F_avg solve on core 3)"}
PRECISION = {0: "f64", 1: "f64 (inner-solve products f32 on MFMA, f32 accumulate)",
             2: "f64 (inner-solve products bf16 on MFMA, f32 accumulate)"}


def workload_name(cfg, system):
    """Workload label from the configuration's own sizes."""
    grid = f"{round(4 / cfg['h'])}x{round(12 / cfg['h'])}"
    what = "Stokes (w = 0) Picard-step system" if system == "stokes" else \
        "Picard step-1 system (prior iterate = the Stokes solution)"
    return (f"{what}, {grid} grid (h=1/{round(1 / cfg['h'])}), m={cfg['m']}, p={cfg['p']}, nt={cfg['nt']}, "
            f"tau={cfg['tau']:g}, nu0={cfg['nu0']:g}, tol 1e-8, Krylov TT eps 1e-6")


def dtype_name(opts):
    if opts["precision"] == 0:
        return "f64"
    if opts["inner_mode"] == 0:
        return PRECISION[opts["precision"]]
    if opts["inner_mode"] == 1 and opts["precision"] == 3:
        return ("f64 (time-stepped mean solve of the preconditioner in f32 on MFMA, f32 accumulate, in the outer "
                "iterations whose residual is below 0.05 tol / 1e-5; f64 before)")
    if opts["inner_mode"] == 1:
        return "f64 (time-stepped mean solve of the preconditioner in f32 on MFMA, f32 accumulate)"
    return "f64"


def solve_options(args=None):
    """Options of the timed solve; the defaults are the configuration bench.py times."""
    if args is None:
        args = parse([])
    return dict(restart=args.restart, outer_explicit=args.outer_explicit, verbose=args.verbose, relax=args.relax,
                precision=args.precision, inner_mode=args.inner_mode, inner_rhs_eps=args.inner_rhs_eps)


# HBM traffic of the dominant kernel, measured with rocprofv3 counters
# (FETCH_SIZE and WRITE_SIZE runs, scaled by the same counters on a device copy
# of known size): bytes per launch, valid while the kernel source it was
# measured on is unchanged (digest of the block cyclic reduction section of
# kernels.hip and of the host factorization).  None until measured.
TRAFFIC_RECORD = {"kernel_src_sha256": "ab4b6e22b1a3b4b6ee52d6c7e0cc1ef1bfcd899b158baaafde10bb28332e78bb",
                  "bytes_per_launch": 14435093, "fetch_bytes_per_launch": 11849973, "write_bytes_per_launch": 2585120,
                  "summary": "profiles/k_bcr_c2_stokes_traffic.md"}


def bcr_source_digest():
    """Digest of what the pass traffic depends on: the block cyclic reduction
    pass kernels (their section of kernels.hip), the host side that launches
    them (variant table, XCD grid padding, tuning and the choice of a variant
    per pass, from struct BcrVariant to bcr_solve_variant), the device
    layout of a factor (upload_bcr and factor_bcr in solver.hip: fragment
    order, descriptors, padding), the callers that set the layout of the
    passes' right-hand sides (the time loop of the mean solve, not the graph
    capture around it, and the time-stepped mean solves in solver.hip) and
    the host factorization (bcr_factor in host_setup.cpp: block sizes,
    levels, dropped zeros)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1906_06785_amd", "csrc")
    src = open(os.path.join(csrc, "kernels.hip")).read()
    head = "// " + "-" * 66 + " block cyclic reduction"
    i0 = src.index(head)
    i1 = src.index("// " + "-" * 66, i0 + len(head))
    k0 = src.index("struct BcrVariant {")
    k1 = src.index("\n}\n", src.index("void bcr_solve_variant(")) + 3
    sol = open(os.path.join(csrc, "solver.hip")).read()
    s0 = sol.index("BcrDev upload_bcr(")
    s1 = sol.index("\n}\n", sol.index("BcrDev factor_bcr(")) + 3
    l0 = sol.index("void mean_time_loop(")
    l1 = sol.index("\n}\n", l0) + 3
    m0 = sol.index("TT exact_mean_solve32(")
    m1 = sol.index("\n}\n", sol.index("TT exact_mean_solve(")) + 3
    host = open(os.path.join(csrc, "host_setup.cpp")).read()
    j0 = host.index("void bcr_factor(")
    j1 = host.index("void bcr_apply_host(")
    return hashlib.sha256((src[i0:i1] + src[k0:k1] + sol[s0:s1] + sol[l0:l1] + sol[m0:m1] +
                           host[j0:j1]).encode()).hexdigest()


def recorded_traffic(dom_name):
    rec = TRAFFIC_RECORD
    if dom_name != "k_bcr" or not rec or rec.get("kernel_src_sha256") != bcr_source_digest():
        return None
    return rec["bytes_per_launch"]


# kernel classes of the profiler -> the kernels they stand for
KERNEL_LABELS = {
    "k_bcr": "k_bcr_split<*> + k_bcr_tile<*> + k_bcr_stream<*> (block cyclic reduction passes, kernel variant "
             "tuned per pass; one event pair per spatial solve, so the average includes the dispatch gaps between "
             "its passes)",
}

OUT_CAPS = (512, 8192)   # output TT capacity (core-1 rank, core-2 rank) of the solution: the exact sum of the
#                          refinement cycles' corrections, whose ranks add
BATCH_CAPS = (128, 2048)  # per problem of a batch (many problems share the GPU's memory)


ORACLE_VELOCITY = {0: "inner", 1: "exact", 2: "minv"}


def cpu_baseline(cfg, budget, gpu_outer_per_solve, inner_mode=1, system=None):
    """The oracle's low-rank FGMRES (oracle.solver.solve_tt, numpy/scipy FP64)
    on the same system with the same velocity block of the preconditioner as
    the GPU line, timed for a bounded number of outer iterations (until the
    budget is spent), all BLAS threads and then one thread; solves/s scaled
    by the GPU's outer-iteration count."""
    import numpy as np  # noqa: F401
    from oracle.solver import solve_tt
    from oracle.system import Problem
    if system is not None:
        raise ValueError("the CPU baseline covers the Stokes system (the Picard step-1 system needs the prior "
                         "iterate on the host)")
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    P = Problem(cfg)
    b = P.rhs()
    velocity = ORACLE_VELOCITY[inner_mode]

    def sample():
        t0 = time.perf_counter()
        _, st = solve_tt(P, b, max_seconds=budget, velocity=velocity)
        dt = time.perf_counter() - t0
        return dt, max(st["outer"], 1)

    dt, outer = sample()
    per_solve = dt / outer * max(gpu_outer_per_solve, 1)
    res = {"value": 1.0 / per_solve, "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": (f"first {outer} outer low-rank FGMRES iteration(s) of the same {cfg_name(cfg)} Stokes solve "
                      f"with the same preconditioner velocity block ({velocity}), {dt:.1f} s with {threads} BLAS "
                      f"threads (numpy/scipy FP64), scaled to the GPU's {gpu_outer_per_solve} outer iterations "
                      f"per solve; host cpu_count={os.cpu_count()}, affinity={len(os.sched_getaffinity(0))}")}
    if threadpool_limits is not None and threads > 1 and dt <= 2 * budget:
        with threadpool_limits(limits=1):
            dt1, outer1 = sample()
        res["single_thread_value"] = 1.0 / (dt1 / outer1 * max(gpu_outer_per_solve, 1))
        res["sample"] += f"; one BLAS thread: {outer1} iteration(s) in {dt1:.1f} s"
    elif threads > 1:
        res["sample"] += ("; no one-thread sample: a single outer iteration already took more than twice the "
                          f"{budget:.0f} s budget")
    return res


def c1_whole_solves(sgtt, ctx, opts, reps=3):
    """Whole solves of the C1 Stokes system (h = 1/4, 207,180 unknowns), where
    the oracle finishes in seconds: the oracle's low-rank FGMRES with the same
    preconditioner velocity block as the GPU line, one warm-up and the median
    of reps with all BLAS threads, one solve with one thread; the library's
    solve of the same system with the same options on the GPU, one warm-up and
    the median of reps (wall time around sgtt_solve, which returns after its
    stream is done)."""
    import statistics

    import torch

    from oracle.solver import solve_tt
    from oracle.system import Problem
    from synthetic_inputs import CONFIGS
    cfg = CONFIGS["C1"]
    velocity = ORACLE_VELOCITY[opts["inner_mode"]]
    P = Problem(cfg)
    bo = P.rhs()
    cpu, outer_cpu = [], 0
    for i in range(reps + 1):
        t0 = time.perf_counter()
        _, st = solve_tt(P, bo, velocity=velocity)
        if i:
            cpu.append(time.perf_counter() - t0)
        outer_cpu = st["outer"]
    one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            solve_tt(P, bo, velocity=velocity)
            one = time.perf_counter() - t0
    except ImportError:
        pass
    S1 = sgtt.System(ctx, cfg)
    b1 = S1.rhs()
    x1 = S1.pair(*OUT_CAPS)
    S1.solve(b1, x1, **opts)   # warm-up: tunes the spatial solves of this system
    gpu, st1 = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st1, _ = S1.solve(b1, x1, **opts)
        torch.cuda.synchronize()
        gpu.append(time.perf_counter() - t0)
    med_cpu, med_gpu = statistics.median(cpu), statistics.median(gpu)
    return {"workload": f"Stokes system at C1 ({cfg_name(cfg)}, {int(P.nt * P.n_xi * (P.n_u + P.n_p))} "
                        f"unknowns), tol 1e-8, same preconditioner velocity block ({velocity})",
            "oracle_seconds_median": med_cpu, "oracle_seconds": cpu, "oracle_single_thread_seconds": one,
            "oracle_outer_iters": outer_cpu, "gpu_seconds_median": med_gpu, "gpu_seconds": gpu,
            "gpu_outer_iters": st1["outer_iters"], "gpu_rel_residual": st1["rel_residual"],
            "gpu_speedup_vs_oracle": med_cpu / med_gpu}


def cfg_name(cfg):
    return f"h={cfg['h']:g} m={cfg['m']} p={cfg['p']} nt={cfg['nt']}"


def batch_main(args):
    """Aggregate throughput of independent problems solved concurrently."""
    import torch

    from paper_1906_06785_amd import sgtt
    from synthetic_inputs import batch_configs

    cfgs = batch_configs(args.batch, seed=0, small=args.batch_small)
    K = max(1, args.contexts)
    ctxs = [sgtt.Context(0) for _ in range(K)]
    systems = [sgtt.System(ctxs[i % K], c) for i, c in enumerate(cfgs)]
    bs = [S.rhs() for S in systems]
    xs = [S.pair(*BATCH_CAPS) for S in systems]
    opts = solve_options(args)
    for _ in range(args.warmup):
        sgtt.solve_batched(systems, bs, xs, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats, status = sgtt.solve_batched(systems, bs, xs, **opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    n = len(cfgs) * args.steps
    print(json.dumps({
        "metric": "independent Picard-step systems solved to 1e-8 exact rel. residual, concurrently",
        "value": n / el, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(cfgs)} independent Stokes Picard-step systems (batch_configs seed 0"
                               f"{', small' if args.batch_small else ''}), {K} contexts",
                   "problems": cfgs},
        "solve": {"worst_rel_residual": max(s["rel_residual"] for s in stats), "status": status,
                  "outer_iters": [s["outer_iters"] for s in stats]}}), flush=True)


# kernel classes reported against their rooflines, with what they stand for
ROOFLINE_CLASSES = {
    "k_spmm": "CSR sparse products of the operator (k_spmm, k_spmm_short<32>)",
    "k_ell_spmm": "ELL mass product of the time-stepped mean solve (k_ell_grouped: row groups staged in LDS)",
    "k_gram": "tall-skinny core-3 Gram products of truncations and inner products (k_gemm<0, 1>)",
    "k_proj": "projections of core 3 onto the kept ranks (k_gemm<0, 2>)",
    "k_gemm": "other FP64 products: full-tensor expansion, small core products (k_gemm<0, 0>)",
    "k_bcr": "block cyclic reduction passes",
}


def class_rooflines(classes):
    out = {}
    for name, what in ROOFLINE_CLASSES.items():
        v = classes.get(name)
        if not v or not v["launches"] or v["seconds"] <= 0:
            continue
        by, fl, sec, nl = v["bytes"], v["flops"], v["seconds"], v["launches"]
        hbm = by > 0 and fl / by < PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
        ach = by / sec / 1e9 if hbm else fl / sec / 1e12
        peak = PEAK_HBM_GBS if hbm else PEAK_FP64_TFLOPS
        out[name] = {"bound": "hbm" if hbm else "mfma", "achieved": ach, "peak": peak,
                     "unit": "GB/s" if hbm else "TFLOP/s", "frac": ach / peak, "launches": nl,
                     "avg_launch_us": sec / nl * 1e6, "algorithmic_bytes_per_launch": by / nl,
                     "algorithmic_flops_per_launch": fl / nl, "kernels": what}
    return out


def build_system(sgtt, ctx, cfg, system, opts, progress):
    """The timed system and its right-hand side; for picard1 the Stokes
    system is solved first (untimed) and its solution is the prior iterate
    (Alg. 3.1: u^(0) from the Stokes solve, then the residual equation
    eq. 3.14 around it)."""
    S = sgtt.System(ctx, cfg)
    b = S.rhs()
    if system == "stokes":
        return S, b, None
    x0 = S.pair(*OUT_CAPS)
    _, st0, _ = S.solve(b, x0, **opts)
    progress("Stokes solve for the prior iterate")
    S1 = sgtt.System(ctx, cfg, prior=x0, eps_conv=1e-3, eps_rhs=1e-6)
    b1 = S1.rhs(S1.pair(128, 1024))
    info = {"prior_ranks": x0.ranks, "prior_rel_residual": st0["rel_residual"],
            "convection_ranks": (S1.info.conv_r1, S1.info.conv_r2),
            "rhs_ranks": b1.ranks, "rhs_norm_over_f": S1.info.rhs_norm / S.info.rhs_norm}
    return S1, b1, info


def time_solves(S, b, out, opts, steps, progress, stream, jsonl=None, label=""):
    """Times `steps` solves; with jsonl (an open file) each solve appends one
    JSON line: its stats and its per-iteration history (residuals and ranks
    of every outer iteration and refinement cycle; a host-side copy, no
    device work)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(steps):
        _, st, rc = S.solve(b, out, **opts)
        stats.append(st)
        if jsonl is not None:
            jsonl.write(json.dumps({"solve": i, "label": label, "status": rc, "stats": st,
                                    "history": S.history()}) + "\n")
        progress("timed solve")
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats


def picard_main(args):
    """Picard's method on the device: Stokes solve, then args.picard steps
    (Alg. 3.1 with eq. 4.8); one JSON line with the per-step record."""
    from paper_1906_06785_amd import sgtt
    from synthetic_inputs import CONFIGS

    cfg = CONFIGS[args.config]
    ctx = sgtt.Context(0)
    opts = solve_options(args)
    x, st, rc = sgtt.picard(ctx, cfg, steps=args.picard, tol_picard=1e-12, eps_soln=1e-10, eps_conv=1e-3,
                            eps_rhs=1e-6, caps=OUT_CAPS, **opts)
    print(json.dumps({"metric": "Picard's method (Alg. 3.1) on the device: per-step record",
                      "config": {"workload": workload_name(cfg, "stokes").replace(
                          "Stokes (w = 0) Picard-step system", f"Stokes solve + {args.picard} Picard steps"),
                                 "eps_conv": 1e-3, "eps_rhs": 1e-6, "eps_soln": 1e-10,
                                 "preconditioner_velocity_block": VELOCITY_BLOCK[opts["inner_mode"]]},
                      "status": rc, "picard": st}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(independent Picard systems would shard one per GPU with no communication)"}))
        sys.exit(2)
    if args.batch > 0:
        batch_main(args)
        return
    if args.picard > 0:
        picard_main(args)
        return
    if args.sweep:
        sweep_main(args)
        return
    import torch

    from paper_1906_06785_amd import sgtt
    from synthetic_inputs import CONFIGS

    cfg = CONFIGS[args.config]
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = sgtt.Context(0, use_torch_stream=True)
    opts = solve_options(args)
    t_setup = time.perf_counter()

    def progress(what):
        if args.progress:
            print(f"[bench] {what} done at {time.perf_counter() - t_setup:.1f} s", file=sys.stderr, flush=True)

    S, b, sys_info = build_system(sgtt, ctx, cfg, args.system, opts, progress)
    setup_s = time.perf_counter() - t_setup
    out = S.pair(*OUT_CAPS)

    for _ in range(args.warmup):
        S.solve(b, out, **opts)
        progress("warm-up solve")
    torch.cuda.synchronize()
    # breakdown solve (outside the timed region): every kernel class and
    # phase, and the dominant class by event time
    ctx.profile(True)
    S.solve(b, out, **opts)
    progress("breakdown solve")
    breakdown = ctx.profile_read()
    phases = ctx.profile_regions()
    ctx.profile(False)
    dom_name = max(breakdown.items(), key=lambda kv: kv[1]["seconds"])[0]
    if args.copy_calibration_mb > 0:
        # a plain copy of known size just before the timed region (also marks
        # where the timed solves begin in a kernel trace)
        n = args.copy_calibration_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # timed region: events on the dominant class only, on one of its scopes
    # in every --event-sample (evenly spread over the timed solves)
    ctx.profile(True, classes=[dom_name])
    ctx.profile_sample(args.event_sample)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    jsonl = open(args.jsonl, "a") if args.jsonl else None
    elapsed, stats = time_solves(S, b, out, opts, args.steps, progress, stream, jsonl, "plain")
    ev1.record(stream)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.profile_sample(1)
    ev_s = ev0.elapsed_time(ev1) * 1e-3
    dom = prof[dom_name]
    by, fl, sec, nl = dom["bytes"], dom["flops"], dom["seconds"], dom["launches"]
    intensity = fl / by if by > 0 else 0.0
    if by > 0 and intensity < PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9):
        ach = by / sec / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS}
    else:
        ach = fl / sec / 1e12 if sec > 0 else 0.0
        roof = {"bound": "mfma", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_FP64_TFLOPS}
    roof.update({"kernel": KERNEL_LABELS.get(dom_name, dom_name), "launches": nl,
                 "avg_launch_us": sec / max(nl, 1) * 1e6,
                 "algorithmic_bytes_per_launch": by / max(nl, 1), "algorithmic_flops_per_launch": fl / max(nl, 1),
                 # launches and seconds cover the sampled scopes: one in every
                 # event_sample_period, so the class's share of the timed
                 # region is about period times the sampled seconds
                 "event_sample_period": args.event_sample,
                 "share_of_timed_region": sec * args.event_sample / ev_s if ev_s > 0 else None,
                 "traffic": recorded_traffic(dom_name) if args.system == "stokes" and args.config == "C2" else None})
    outer = int(round(sum(s["outer_iters"] for s in stats) / len(stats)))
    worst = max(s["rel_residual"] for s in stats)
    # the metric compares learned/mixed-precision solves with the plain FP64
    # one at equal accuracy: value is the plain FP64 solver; variants named
    # with --compare are timed the same way and reported beside it
    comparison = {}
    for name in [v for v in args.compare.split(",") if v]:
        vopts = dict(opts, **VARIANTS[name])
        vout = S.pair(*OUT_CAPS)
        S.solve(b, vout, **vopts)   # warm-up (tuning of the spatial solves for new column counts)
        progress(f"warm-up solve of {name}")
        v_el, v_stats = time_solves(S, b, vout, vopts, args.steps, progress, stream, jsonl, name)
        v_worst = max(s["rel_residual"] for s in v_stats)
        ctx.profile(True)   # one profiled solve of the variant for its breakdown
        _, vp_st, _ = S.solve(b, vout, **vopts)
        v_breakdown = ctx.profile_read()
        ctx.profile(False)
        comparison[name] = {
            "solves_per_s": args.steps / v_el, "ms_per_step": v_el / args.steps * 1e3,
            "speedup_vs_value": (args.steps / v_el) / (args.steps / elapsed), "dtype": dtype_name(vopts),
            "preconditioner_velocity_block": VELOCITY_BLOCK[vopts["inner_mode"]],
            "outer_iters": int(round(sum(s["outer_iters"] for s in v_stats) / len(v_stats))),
            "inner_iters": v_stats[-1]["inner_iters"], "max_rel_residual": v_worst, "converged": v_worst <= 1e-8,
            "max_krylov_rank_u": v_stats[-1]["max_rank_krylov_u"],
            "f32_applications": v_stats[-1]["f32_applications"],
            "graph_launches": v_stats[-1]["graph_launches"],
            "kernels_note": ("the mean solve's time loop ran as graph launches, which the per-class breakdown does "
                             "not attribute (its mass products and BCR passes are missing below)")
            if vp_st["graph_launches"] else None,
            "kernels": {k: {"ms": v["seconds"] * 1e3, "launches": v["launches"]} for k, v in v_breakdown.items()
                        if v["launches"]}}
    res = {
        "metric": "Picard-step solve time to 1e-8 rel. residual: learned/mixed vs plain FP64",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name(opts),
        "data": "synthetic (step-domain flow generated by the library's own mesh/assembly; no dataset)",
        "config": {"workload": workload_name(cfg, args.system),
                   "unknowns": int(S.nt * S.nxi * (S.nu + S.np)),
                   "solver": ("Alg. 4.2 (explicit residual each outer iteration)" if args.outer_explicit
                              else "Alg. 4.2 cycles stopped on the least-squares estimate"),
                   "restart": args.restart, "relaxed_truncation": bool(args.relax),
                   "preconditioner_velocity_block": VELOCITY_BLOCK[opts["inner_mode"]],
                   "system": sys_info},
        "solve": {"outer_iters": outer, "cycles": stats[-1]["cycles"], "inner_iters": stats[-1]["inner_iters"],
                  "max_rel_residual": worst, "converged": worst <= 1e-8,
                  "max_krylov_rank_u": stats[-1]["max_rank_krylov_u"], "setup_s": setup_s},
        "roofline": roof,
        "learned_mixed": (comparison if comparison else
                          {"measured": False, "reason": "no variant named with --compare; value is the plain "
                                                        "FP64 solver"}),
        # per-class and per-phase event times of one profiled solve after the
        # warm-up (every class evented, so it runs slower than a timed step)
        "kernels": {k: {"ms": v["seconds"] * 1e3, "launches": v["launches"]} for k, v in breakdown.items()
                    if v["launches"]},
        # the same solve's kernel classes against their rooflines: algorithmic
        # bytes (flops above the ridge) per launch over the event-timed launch
        "rooflines": class_rooflines(breakdown),
        "phases_ms": {r: {k: round(v * 1e3, 1) for k, v in row.items()} for r, row in phases.items()},
    }
    if not args.no_cpu_baseline:
        try:
            res["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds, outer, opts["inner_mode"],
                                               None if args.system == "stokes" else "picard1")
        except Exception as e:  # the baseline is informative only
            res["cpu_baseline"] = {"error": repr(e)}
        if args.config == "C2" and args.system == "stokes":
            # like for like at a size both sides solve whole
            try:
                res["cpu_baseline"]["c1_whole_solves"] = c1_whole_solves(sgtt, ctx, opts)
            except Exception as e:
                res["cpu_baseline"]["c1_whole_solves"] = {"error": repr(e)}
            progress("C1 whole solves on both sides")
    if jsonl is not None:
        jsonl.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
