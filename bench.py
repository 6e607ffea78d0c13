#!/usr/bin/env python3
"""Benchmark: SRJ with the data-driven scheme selector on one MI355X.

Workload (one "step" = one whole solve to tolerance from x0 = 0): 2D Poisson,
5-point stencil, 2048 x 2048 interior grid, Dirichlet zero, binary64, b = 8
random-amplitude low sine modes + U(-1e-3, 1e-3) noise (seed 0), relative
residual target 1e-10, scheme chosen per cycle by Algorithm 1.  Inputs are
generated once and are resident on the GPU before timing starts.

value = GLUPS = (sweeps x interior points) / solve time, over the timed steps.
Also reported: time to tolerance, the roofline of the dominant kernel (the
relaxation sweep) measured with HIP events on the solver's stream, and the CPU
oracle timed on a bounded sample of the same solve.
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
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2048, help="grid side (default 2048)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--max-cycles", type=int, default=200)
    ap.add_argument("--plan", type=str, default="", help="kind:rows:T:occ kernel plan override")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the CPU oracle sample (0 = skip)")
    return ap.parse_args()


def cpu_baseline(prob, target_s):
    import oracle
    rate_probe = prob.zeros()
    t = time.perf_counter()
    for w in (0.6, 1.1):
        rate_probe = oracle.sweep(prob, rate_probe, w)
    per_sweep = (time.perf_counter() - t) / 2.0
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
    prob = workloads.c2(n=args.n)
    s = Solver(prob)
    if args.plan:
        assert s.set_plan(*(int(v) for v in args.plan.split(":"))) == 0, "plan not supported"
    plan = s.get_plan()
    x = s.zeros()
    kw = dict(tol=args.tol, max_cycles=args.max_cycles)
    print(f"# workload c2 {args.n}x{args.n} fp64, plan {plan}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        x.zero_()
        out = s.solve(x, **kw)
        print(f"# warmup {i}: {out['status']} cycles {out['cycles']} sweeps {out['sweeps']}",
              file=sys.stderr, flush=True)

    s.set_profiling(True)
    torch.cuda.synchronize()
    times, results = [], []
    for i in range(args.steps):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = s.solve(x, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        results.append(out)
        print(f"# step {i}: {dt * 1e3:.1f} ms {out['status']} cycles {out['cycles']} "
              f"sweeps {out['sweeps']}", file=sys.stderr, flush=True)
    sweep_ms, launches, prof_sweeps = s.profile()
    s.set_profiling(False)

    total = sum(times)
    sweeps = sum(r["sweeps"] for r in results)
    glups = sweeps * prob.npoints / total / 1e9
    last = results[-1]
    # dominant kernel: the relaxation launches.  Algorithmic bytes per launch:
    # read x and b, write x' once (binary64): 24 B per interior point.
    avg_launch_s = sweep_ms / 1e3 / max(launches, 1)
    alg_bytes = 24.0 * prob.npoints
    achieved = alg_bytes / avg_launch_s / 1e9
    rec = {
        "metric": "GLUPS + time-to-1e-10 residual: plain FP64 SRJ vs FP32-refined/batched, 1 GPU",
        "value": round(glups, 3), "unit": "GLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D Poisson 5-point {args.n}x{args.n} FP64, b = 8 sine modes + "
                               f"U(-1e-3,1e-3) noise (seed 0), x0 = 0, relative residual "
                               f"{args.tol:g}, Algorithm 1 level choice",
                   "grid": [args.n, args.n], "tol": args.tol, "plan": list(plan)},
        "time_to_tol_ms": round(total / args.steps * 1e3, 3),
        "converged": bool(last["converged"]), "cycles": last["cycles"], "sweeps": last["sweeps"],
        "final_rel_residual": last["r_final"] / last["r0"],
        "levels": [int(v) for v in last["levels"]],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "relaxation sweep launch", "sweeps_per_launch": prof_sweeps / max(launches, 1),
                     "avg_launch_us": round(avg_launch_s * 1e6, 3),
                     "bytes_per_launch": alg_bytes},
    }
    if args.cpu_seconds > 0:
        rec["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    s.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
