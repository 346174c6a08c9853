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
    ap.add_argument("--precision", type=int, default=0, help="inner-solve products: 0 FP64, 1 FP32, 2 BF16")
    ap.add_argument("--inner-mode", type=int, default=1,
                    help="velocity block of the preconditioner: 1 time-stepped mean solve on the full tensor, "
                         "0 inner low-rank GMRES with M (eq. 5.22-5.23)")
    ap.add_argument("--inner-rhs-eps", type=float, default=1e-2,
                    help="truncation of the inner GMRES right-hand side (inner mode 0)")
    ap.add_argument("--batch", type=int, default=0,
                    help="N > 0: instead, time N independent problems (batch_configs) on --contexts streams")
    ap.add_argument("--contexts", type=int, default=8)
    ap.add_argument("--batch-small", action="store_true", help="coarse grids / short horizons for the batch")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="M > 0: before the timed solves, one device-to-device copy of M MiB (a plain copy kernel "
                         "of known size for scaling memory counters)")
    ap.add_argument("--progress", action="store_true", help="one line on stderr per solve")
    return ap.parse_args(argv)


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
TRAFFIC_RECORD = {"kernel_src_sha256": "12eb2c4c70deb575f017698bb4d7b98b56ab3dc6b5ed67aab8c86a749f5e63ac",
                  "bytes_per_launch": 32953178, "fetch_bytes_per_launch": 30163588, "write_bytes_per_launch": 2789590,
                  "summary": "profiles/k_bcr_c2_stokes_traffic.md"}


def bcr_source_digest():
    """Digest of what the pass traffic depends on: the block cyclic reduction
    section of kernels.hip (the pass kernels) and the host factorization
    (bcr_factor in host_setup.cpp: block sizes, levels, dropped zeros)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1906_06785_amd", "csrc")
    src = open(os.path.join(csrc, "kernels.hip")).read()
    head = "// " + "-" * 66 + " block cyclic reduction"
    i0 = src.index(head)
    i1 = src.index("// " + "-" * 66, i0 + len(head))
    host = open(os.path.join(csrc, "host_setup.cpp")).read()
    j0 = host.index("void bcr_factor(")
    j1 = host.index("void bcr_apply_host(")
    return hashlib.sha256((src[i0:i1] + host[j0:j1]).encode()).hexdigest()


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

OUT_CAPS = (128, 4096)   # output TT capacity (core-1 rank, core-2 rank) of the solution


def cpu_baseline(cfg, budget, gpu_outer_per_solve):
    import numpy as np  # noqa: F401
    from oracle.solver import solve_tt
    from oracle.system import Problem
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    P = Problem(cfg)
    b = P.rhs()
    t0 = time.perf_counter()
    _, st = solve_tt(P, b, max_seconds=budget)
    dt = time.perf_counter() - t0
    outer = max(st["outer"], 1)
    per_iter = dt / outer
    per_solve = per_iter * max(gpu_outer_per_solve, 1)
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"first {st['outer']} outer low-rank FGMRES iteration(s) of the same {cfg_name(cfg)} solve "
                       f"({dt:.1f} s, numpy/scipy FP64), scaled to the GPU's {gpu_outer_per_solve} outer "
                       f"iterations per solve; host cpu_count={os.cpu_count()}, "
                       f"affinity={len(os.sched_getaffinity(0))}")}


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
    xs = [S.pair(*OUT_CAPS) for S in systems]
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


def main():
    args = parse()
    if args.batch > 0 and args.gpus == 1:
        batch_main(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(independent Picard systems would shard one per GPU with no communication)"}))
        sys.exit(2)
    import torch

    from paper_1906_06785_amd import sgtt
    from synthetic_inputs import CONFIGS

    cfg = CONFIGS[args.config]
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = sgtt.Context(0, use_torch_stream=True)
    t_setup = time.perf_counter()
    S = sgtt.System(ctx, cfg)
    b = S.rhs()
    setup_s = time.perf_counter() - t_setup
    opts = solve_options(args)
    out = S.pair(*OUT_CAPS)
    def progress(what):
        if args.progress:
            print(f"[bench] {what} done at {time.perf_counter() - t_setup:.1f} s", file=sys.stderr, flush=True)

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
    # timed region: events on the dominant class only
    ctx.profile(True, classes=[dom_name])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    stats = []
    for _ in range(args.steps):
        _, st, rc = S.solve(b, out, **opts)
        stats.append(st)
        progress("timed solve")
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    elapsed = t1 - t0
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
                 "share_of_timed_region": sec / ev_s if ev_s > 0 else None,
                 "traffic": recorded_traffic(dom_name)})
    outer = int(round(sum(s["outer_iters"] for s in stats) / len(stats)))
    worst = max(s["rel_residual"] for s in stats)
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
        "dtype": "f64",
        "data": "synthetic (step-domain flow generated by the library's own mesh/assembly; no dataset)",
        "config": {"workload": f"{args.config} Stokes Picard-step system, 64x192 grid (h=1/16), m=4, p=3 (n_xi=35), "
                               f"nt=128, tau=0.05, plain FP64, tol 1e-8, TT eps 1e-6",
                   "unknowns": int(128 * 35 * (S.nu + S.np)) if args.config == "C2" else None,
                   "solver": ("Alg. 4.2 (explicit residual each outer iteration)" if args.outer_explicit
                              else "Alg. 4.2 cycles stopped on the least-squares estimate"),
                   "restart": args.restart, "relaxed_truncation": bool(args.relax),
                   "preconditioner_velocity_block": ("time-stepped mean solve (full tensor)" if args.inner_mode == 1
                                                     else "inner low-rank GMRES with M")},
        "solve": {"outer_iters": outer, "cycles": stats[-1]["cycles"], "inner_iters": stats[-1]["inner_iters"],
                  "max_rel_residual": worst, "converged": worst <= 1e-8,
                  "max_krylov_rank_u": stats[-1]["max_rank_krylov_u"], "setup_s": setup_s},
        "roofline": roof,
        # per-class and per-phase event times of one profiled solve after the
        # warm-up (every class evented, so it runs slower than a timed step)
        "kernels": {k: {"ms": v["seconds"] * 1e3, "launches": v["launches"]} for k, v in breakdown.items()
                    if v["launches"]},
        "phases_ms": {r: {k: round(v * 1e3, 1) for k, v in row.items()} for r, row in phases.items()},
    }
    if not args.no_cpu_baseline:
        try:
            res["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds, outer)
        except Exception as e:  # the baseline is informative only
            res["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
