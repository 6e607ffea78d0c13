#!/usr/bin/env python3
"""Benchmark: SRJ with the data-driven scheme selector on one MI355X.

Workload: 2D Poisson, 5-point stencil, 2048 x 2048 interior grid, Dirichlet
zero, b = 8 random-amplitude low sine modes + U(-1e-3, 1e-3) noise (seed 0),
x0 = 0, relative residual target 1e-10, scheme chosen per cycle by
Algorithm 1.  Inputs are generated once and resident on the GPU before any
timing starts.

One step = one plain binary64 SRJ solve (capped at --max-cycles cycles: on
this grid binary64 round-off stops the relative residual near 1.4e-9, above
the target).  value = GLUPS = (sweeps x interior points) / step time.  The
same line reports the binary32-refined solve of the same problem (binary64
residual and update, binary32 inner cycles) with its time to the target, the
roofline of the dominant kernel measured with HIP events on the solver's
stream, and the CPU oracle timed on a bounded sample of the binary64 solve.
--copy-probe-mib runs one plain device copy of known size first (a reference
dispatch for hardware byte counters).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the binary64 tile kernel on the 2048 x 2048 grid,
# from rocprofv3 FETCH_SIZE and WRITE_SIZE runs scaled by a 1 GiB device copy
# (fetch x2.000, write x1.000).  Valid only for the kernel plan and source they
# were taken with; any other plan reports null.
MEASURED_TRAFFIC = {(1, 24, 4, 1): 144.8e6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2048, help="grid side (default 2048)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--max-cycles", type=int, default=50)
    ap.add_argument("--plan", type=str, default="", help="kind:rows:T:occ kernel plan override")
    ap.add_argument("--copy-probe-mib", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target length of the CPU oracle sample (0 = skip)")
    return ap.parse_args()


def cpu_baseline(prob, target_s):
    import oracle
    rate_probe = prob.zeros()
    rate_probe = oracle.sweep(prob, rate_probe, 0.6)
    t = time.perf_counter()
    for w in (0.6, 1.1, 0.9):
        rate_probe = oracle.sweep(prob, rate_probe, w)
    per_sweep = (time.perf_counter() - t) / 3.0
    # cycles of the heuristic climb 0, 1, 2, ... until the sample fills target_s
    budget = max(1, int(target_s / max(per_sweep, 1e-9)))
    cycles, sweeps = 0, 0
    while cycles < 25 and sweeps + oracle.level_M(cycles) <= budget:
        sweeps += oracle.level_M(cycles)
        cycles += 1
    cycles = max(cycles, 1)
    t = time.perf_counter()
    out = oracle.solve(prob, tol=1e-300, max_cycles=cycles)
    dt = time.perf_counter() - t
    return {
        "value": out["sweeps"] * prob.npoints / dt / 1e9, "unit": "GLUPS",
        "cores": oracle.num_threads(), "kind": "oracle",
        "sample": f"first {out['cycles']} cycles (levels {out['levels'][0]}..{out['levels'][-1]}, "
                  f"{out['sweeps']} sweeps, residual after each cycle) of the same solve, "
                  f"{dt:.1f} s",
    }


def run_leg(s, x, kw, steps, warmup, label):
    """warmup + timed solves; returns per-step times, results and the sweep profile."""
    import torch
    for i in range(warmup):
        x.zero_()
        out = s.solve(x, **kw)
        print(f"# {label} warmup {i}: {out['status']} cycles {out['cycles']} "
              f"sweeps {out['sweeps']}", file=sys.stderr, flush=True)
    s.set_profiling(True)
    torch.cuda.synchronize()
    times, results = [], []
    for i in range(steps):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = s.solve(x, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        results.append(out)
        print(f"# {label} step {i}: {dt * 1e3:.1f} ms {out['status']} cycles {out['cycles']} "
              f"sweeps {out['sweeps']}", file=sys.stderr, flush=True)
    prof = s.profile()
    s.set_profiling(False)
    return times, results, prof


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is design-only in this build)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads
    from paper_2011_06636_amd.solver import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe_mib > 0:
        n_el = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n_el, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    prob = workloads.c2(n=args.n)
    s = Solver(prob)
    if args.plan:
        assert s.set_plan(*(int(v) for v in args.plan.split(":"))) == 0, "plan not supported"
    plan = s.get_plan(0)
    plan_inner = s.get_plan(1)
    x = s.zeros()
    print(f"# workload c2 {args.n}x{args.n}, plans f64 {plan} inner {plan_inner}",
          file=sys.stderr, flush=True)

    # plain binary64 SRJ: the headline GLUPS
    kw64 = dict(tol=args.tol, max_cycles=args.max_cycles)
    times, results, (sweep_ms, launches, prof_sweeps) = run_leg(
        s, x, kw64, args.steps, args.warmup, "f64")
    total = sum(times)
    sweeps = sum(r["sweeps"] for r in results)
    glups = sweeps * prob.npoints / total / 1e9
    last = results[-1]
    rel = last["norms"] / last["r0"]
    best = int(np.argmin(rel))

    # binary32-refined SRJ: time to the same tolerance
    kw32 = dict(tol=args.tol, max_cycles=args.max_cycles, precision="f32")
    t32, r32, (ms32, la32, sw32) = run_leg(s, x, kw64 | kw32, args.steps, args.warmup, "f32")
    l32 = r32[-1]
    resid32 = s.residual_norm(x) / l32["r0"]

    # dominant kernel of the binary64 leg: the relaxation launches.  Algorithmic
    # bytes per launch: read x and b, write x' once (binary64): 24 B per point,
    # whatever the number of sweeps fused into the launch.
    avg_launch_s = sweep_ms / 1e3 / max(launches, 1)
    alg_bytes = 24.0 * prob.npoints
    achieved = alg_bytes / avg_launch_s / 1e9
    f64_time = total / args.steps
    f32_time = sum(t32) / args.steps
    rec = {
        "metric": "GLUPS + time-to-1e-10 residual: plain FP64 SRJ vs FP32-refined/batched, 1 GPU",
        "value": round(glups, 3), "unit": "GLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(f64_time * 1e3, 3),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D Poisson 5-point {args.n}x{args.n}, b = 8 sine modes + "
                               f"U(-1e-3,1e-3) noise (seed 0), x0 = 0, relative residual "
                               f"{args.tol:g}, Algorithm 1 level choice; plain FP64 SRJ "
                               f"(cap {args.max_cycles} cycles)",
                   "grid": [args.n, args.n], "tol": args.tol, "plan_f64": list(plan),
                   "plan_inner": list(plan_inner)},
        "f64": {"converged": bool(last["converged"]), "cycles": last["cycles"],
                "sweeps": last["sweeps"], "time_ms": round(f64_time * 1e3, 3),
                "best_rel_residual": float(rel[best]), "cycle_of_best": best,
                "final_rel_residual": float(rel[-1]),
                "levels": [int(v) for v in last["levels"]]},
        "f32_refined": {"converged": bool(l32["converged"]), "cycles": l32["cycles"],
                        "sweeps": l32["sweeps"], "time_to_tol_ms": round(f32_time * 1e3, 3),
                        "inner_GLUPS": round(sum(r["sweeps"] for r in r32) * prob.npoints
                                             / sum(t32) / 1e9, 3),
                        "final_rel_residual_f64": resid32,
                        "levels": [int(v) for v in l32["levels"]]},
        "time_to_tol_ms": {"f64": round(f64_time * 1e3, 3) if last["converged"] else None,
                           "f32_refined": round(f32_time * 1e3, 3) if l32["converged"] else None},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": MEASURED_TRAFFIC.get(tuple(plan)) if args.n == 2048 else None,
                     "kernel": "k_tile2d<StF64> (binary64 relaxation, fused sweeps)",
                     "sweeps_per_launch": round(prof_sweeps / max(launches, 1), 3),
                     "avg_launch_us": round(avg_launch_s * 1e6, 3),
                     "bytes_per_launch": alg_bytes,
                     "effective_GBps_per_sweep": round(24.0 * glups, 1)},
    }
    if args.cpu_seconds > 0:
        rec["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    s.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
