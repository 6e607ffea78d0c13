#!/usr/bin/env python3
"""Benchmark: SRJ with the data-driven scheme selector on one MI355X.

Workload: 2D Poisson, 5-point stencil, 2048 x 2048 interior grid, Dirichlet
zero, b = 8 random-amplitude low sine modes + U(-1e-3, 1e-3) noise (seed 0),
x0 = 0, scheme chosen per cycle by Algorithm 1.  Inputs are generated once
and resident on the GPU before any timing starts.

One step = one plain binary64 SRJ solve to the common relative residual
--common-tol (2e-9 by default): binary64 round-off stops this grid's
relative residual near 1.4e-9, above the 1e-10 target, so the plain and the
binary32-refined solves are compared at a tolerance both reach.  value =
GLUPS = (sweeps x interior points) / step time.  The same line reports the
binary32-refined solve (binary64 residual and update, binary32 inner cycles)
to the common tolerance and to the 1e-10 target, the binary64 solve capped
at --max-cycles cycles (best residual and the cycle of it), the roofline of
the dominant kernel measured with HIP events on the solver's stream, the
1D N = 255 solve (the whole solve in one workgroup) against the oracle's
time on the same input, a grid whose arrays do not fit the 256 MB Infinity
Cache (8192^2) timed against a streaming kernel of the library, and the CPU
oracle timed on bounded samples (all host threads and one thread).
Unless --no-extras is given, the line also carries the other workloads'
comparisons: the 256^3 variable-coefficient problem (binary64 vs
binary32-refined time to 1e-10) and the two batches (512 2D problems,
binary32-refined; 128 3D anisotropic boxes, bfloat16-stored correction),
each batched solve against a loop of single-problem binary64 solves, and the
selector's training data of section 3 collected on the GPU at the paper's
scale with the rule fitted to it, and the Neumann Laplace scaling study of
section 4.2.2 with the per-sweep update stopping test, and the general
sparse matrices of sections 4.2.1 and 4.2.4.
--copy-probe-mib runs one streaming copy of known size first (the reference
dispatch for hardware byte counters).
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2011_06636_amd", "csrc")


def source_sha(files):
    """sha256 (16 hex digits) of kernel source files: counter figures below
    hold only for the sources they were taken with."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# HBM bytes per launch on the 2048 x 2048 grid, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by a reference copy of known size (fetch x2.000,
# write x1.000): (bytes, source files, their sha at counter time).  A plan
# whose sources changed since reports null.
MEASURED_TRAFFIC = {
    (8, 8, 10, 8): (111.1e6, ("block2d.h", "tile2d.h"), "c7d76330bd34261a"),
    (0, 0, 1, 1): (104.4e6, ("sweep.hip",), "6bfcf0ef0b31c00a"),
    (5, 8, 1, 1): (101.1e6, ("wave2d.h", "tile2d.h"), "11a310246989742f"),
}
# the single-sweep plan timed beside the default one (wavefront strips, T = 1)
ONE_SWEEP_PLAN = (5, 8, 1, 1)
# VALU issue bound of the default block kernel (plan (8, 8, 10, 8)): its
# interior sweep loop issues 228 vector instructions for a wave's 16 point
# updates (read from the kernel's gfx950 assembly), each wave64 instruction
# occupies a SIMD for 4 cycles, 256 CUs x 4 SIMDs at 2.4 GHz; a block of
# 128 x 64 points writes 108 x 44 of them, so 1.724 updates per useful one
VALU_CEILING = {(8, 8, 10, 8): {"instr_per_update": 228 / 16,
                                "updates_per_written": (128 * 64) / (108 * 44),
                                "sources": ("block2d.h", "tile2d.h"),
                                "sha": "c7d76330bd34261a"}}


def measured_traffic(plan):
    e = MEASURED_TRAFFIC.get(tuple(plan))
    if e is None:
        return None
    val, files, sha = e
    if sha is not None and source_sha(files) != sha:
        return None
    return val


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2048, help="grid side (default 2048)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--max-cycles", type=int, default=50)
    ap.add_argument("--plan", type=str, default="", help="kind:rows:T:occ kernel plan override")
    ap.add_argument("--common-tol", type=float, default=2e-9,
                    help="relative residual both the plain binary64 and the refined solve reach")
    ap.add_argument("--copy-probe-mib", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 3D and batched comparison legs")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target length of each CPU oracle sample (0 = skip)")
    ap.add_argument("--ooc-n", type=int, default=8192,
                    help="side of the out-of-cache 2D grid (0 = skip)")
    ap.add_argument("--only", choices=["c1", "ooc", "mg", "c3", "c4", "c5", "c2vc", "training",
                                       "neumann", "general", "c4once", "c5once"],
                    default="", help="run one leg alone and print its record")
    ap.add_argument("--precision", default="bf16", choices=["f64", "f32", "bf16", "f16"],
                    help="precision of --only c5once")
    ap.add_argument("--c3-cycles", type=int, default=200,
                    help="cycle cap of each 3D variable-coefficient solve")
    return ap.parse_args()


def host_cpu():
    """Model name and usable threads of the host (for the CPU baseline)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_threads": usable}


def _oracle_sample(prob, target_s, levels, norms, threads):
    """The oracle on the first cycles of the same solve, about target_s seconds
    with `threads` threads; states whether its levels and norms agree with the
    GPU solve's."""
    import numpy as np

    import oracle
    oracle.set_num_threads(threads)
    rate_probe = prob.zeros()
    rate_probe = oracle.sweep(prob, rate_probe, 0.6)
    t = time.perf_counter()
    for w in (0.6, 1.1, 0.9):
        rate_probe = oracle.sweep(prob, rate_probe, w)
    per_sweep = (time.perf_counter() - t) / 3.0
    budget = max(1, int(target_s / max(per_sweep, 1e-9)))
    cycles, sweeps = 0, 0
    for lv in levels:
        if sweeps + oracle.level_M(int(lv)) > budget:
            break
        sweeps += oracle.level_M(int(lv))
        cycles += 1
    cycles = max(cycles, 1)
    t = time.perf_counter()
    out = oracle.solve(prob, tol=1e-300, max_cycles=cycles)
    dt = time.perf_counter() - t
    k = int(out["cycles"])
    gpu_n = np.asarray(norms[:k + 1], dtype=np.float64)
    agree = {"cycles": k,
             "same_levels": bool(np.array_equal(out["levels"], np.asarray(levels[:k]))),
             "max_rel_norm_diff": float(np.max(np.abs(out["norms"] - gpu_n) / out["norms"]))}
    return {"value": out["sweeps"] * prob.npoints / dt / 1e9, "unit": "GLUPS",
            "cores": oracle.num_threads(), "agrees_with_gpu": agree,
            "sample": f"first {out['cycles']} cycles (levels {out['levels'][0]}..{out['levels'][-1]}, "
                      f"{out['sweeps']} sweeps, residual after each cycle) of the same solve, "
                      f"{dt:.1f} s"}


def cpu_baseline(prob, target_s, levels, norms):
    """The oracle, as it stands, on bounded samples of the same binary64 solve:
    OpenMP's default thread count (the record's value), then one thread."""
    import oracle
    cpu = host_cpu()
    default = oracle.num_threads()  # OpenMP's default (OMP_NUM_THREADS where set)
    allcores = _oracle_sample(prob, target_s, levels, norms, default)
    one = _oracle_sample(prob, target_s * 0.75, levels, norms, 1)
    oracle.set_num_threads(default)
    rec = dict(allcores)
    rec["kind"] = "oracle"
    rec["host"] = cpu
    rec["single_thread"] = {k: one[k] for k in ("value", "unit", "cores", "sample", "agrees_with_gpu")}
    return rec


KERNEL_NAMES = {
    0: "k_sweep_generic<2> (one sweep per launch)",
    1: "k_tile2d<StF64> (register tiles, fused sweeps)",
    2: "k_tile2d<StF64> (register tiles, right-hand side in LDS)",
    5: "k_wave2d<StF64> (wavefront strips)",
    7: "k_block2d<StF64, C=1> (cooperative wave blocks, fused sweeps)",
    8: "k_block2d<StF64, C=2> (cooperative wave blocks, two columns per lane)",
}


def valu_issue(plan, npoints, sweeps, launches, avg_launch_s):
    """The block kernel's useful point updates per second (kernel time only)
    against its VALU issue ceiling (VALU_CEILING); None for other plans or
    once the kernel's sources have changed since the instruction count."""
    c = VALU_CEILING.get(tuple(plan))
    if c is None or launches == 0 or source_sha(c["sources"]) != c["sha"]:
        return None
    raw = 256 * 4 * 64 / (c["instr_per_update"] * 4) * 2.4e9  # updates per second
    ceiling = raw / c["updates_per_written"]
    achieved = npoints * sweeps / launches / avg_launch_s
    return {"ceiling_GLUPS": round(ceiling / 1e9, 1), "achieved_GLUPS": round(achieved / 1e9, 1),
            "frac": round(achieved / ceiling, 4),
            "basis": f"{c['instr_per_update'] * 16:.0f} VALU instructions per 16 updates of a wave "
                     "in the interior sweep loop, 4 cycles each, 256 CUs x 4 SIMDs at 2.4 GHz, "
                     f"{c['updates_per_written']:.3f} updates per written point"}


def plan_rate(s, x, prob, plan, level=12, ceiling=None):
    """One cycle of `level` with `plan` on the problem: kernel time per launch
    (HIP events on the solver's stream), GLUPS, algorithmic GB/s (24 B per
    point per launch, whatever the sweeps fused into it) and the fraction of
    8 TB/s and of the measured streaming ceiling."""
    keep = s.get_plan(0)
    assert s.set_plan(*plan) == 0
    s.run_cycle(x, level)
    s.set_profiling(True)
    s.run_cycle(x, level)
    ms, launches, sweeps = s.profile()
    s.set_profiling(False)
    assert s.set_plan(*keep) == 0
    t = ms / 1e3 / max(launches, 1)
    per_launch = sweeps / max(launches, 1)
    gbps = 24.0 * prob.npoints / t / 1e9
    rec = {"kernel": KERNEL_NAMES.get(plan[0], f"plan kind {plan[0]}"), "plan": list(plan),
           "sweeps_per_launch": round(per_launch, 3), "avg_launch_us": round(t * 1e6, 3),
           "GLUPS": round(prob.npoints * per_launch / t / 1e9, 3),
           "achieved_GBps": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBS, 4),
           "traffic": measured_traffic(plan) if tuple(prob.n[:2]) == (2048, 2048) else None}
    if ceiling:
        rec["frac_of_stream_ceiling"] = round(gbps / ceiling, 4)
    return rec


def stream_ceiling(n, reps=5):
    """Streaming kernels of the library (srj_stream_probe) over arrays of n
    binary64 values: copy (16 B per value) and a + b (24 B per value, the
    one-sweep mix), best of reps, in GB/s, timed with events on torch's
    current stream (the one the kernels are launched on)."""
    import torch

    from paper_2011_06636_amd import abi
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    o = torch.empty(n, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    out = {}
    for kind, name, per in ((0, "copy", 16.0), (1, "read2_write1", 24.0)):
        abi.srj_stream_probe(kind, a.data_ptr(), b.data_ptr(), o.data_ptr(), n, st)
        best = 0.0
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            abi.srj_stream_probe(kind, a.data_ptr(), b.data_ptr(), o.data_ptr(), n, st)
            e1.record()
            e1.synchronize()
            best = max(best, per * n / (e0.elapsed_time(e1) / 1e3) / 1e9)
        out[name + "_GBps"] = round(best, 1)
    del a, b, o
    torch.cuda.empty_cache()
    return out


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t


def extra_c3(max_cycles=200):
    """3D variable-coefficient 256^3: plain binary64 vs binary32-refined, to 1e-10
    (at most max_cycles cycles each)."""
    import workloads
    from paper_2011_06636_amd.solver import Solver
    prob = workloads.c3()
    s = Solver(prob)
    s.autotune(0)
    s.autotune(1)
    rec = {"workload": "3D -div(k grad u) = 1, 7-point, 256^3, k log-normal (sigma 1, "
                       "correlation 8 cells, seed 0), relative residual 1e-10",
           "plans": {"f64": list(s.get_plan(0)), "inner": list(s.get_plan(1))}}
    for prec in ("f64", "f32"):
        x = s.zeros()
        s.solve(x, tol=1e-10, precision=prec, max_cycles=max_cycles)
        x.zero_()
        out, dt = _timed(lambda: s.solve(x, tol=1e-10, precision=prec, max_cycles=max_cycles))
        rec[prec] = {"converged": out["converged"], "cycles": out["cycles"],
                     "sweeps": out["sweeps"], "time_ms": round(dt * 1e3, 3),
                     "GLUPS": round(out["sweeps"] * prob.npoints / dt / 1e9, 3),
                     "final_rel_residual_f64": s.residual_norm(x) / out["r0"]}
        print(f"# c3 {prec}: {dt * 1e3:.1f} ms {out['status']}", file=sys.stderr, flush=True)
    if rec["f64"]["converged"] and rec["f32"]["converged"]:
        rec["f32_refined_speedup_time_to_tol"] = round(rec["f64"]["time_ms"] / rec["f32"]["time_ms"], 3)
    s.close()
    return rec


def extra_c2_varcoef(n=2048, cycles=40, tol=1e-6, tol_cycles=100):
    """2D variable-coefficient n x n grid (per-face couplings and diagonal):
    the same capped solve with one sweep per launch and with the default
    fused per-face block plan (bit-identical iterates); then plain binary64
    and binary32-refined solves to a relative residual of tol with the
    default plans (at most tol_cycles cycles each)."""
    import numpy as np
    import workloads
    from paper_2011_06636_amd.solver import Solver
    prob = workloads.variable_coefficient_2d(n, n, seed=0)
    s = Solver(prob)
    default = tuple(s.get_plan(0))
    rec = {"workload": f"2D -div(k grad u) = 1, 5-point, {n}x{n}, k log-normal (sigma 1, "
                       f"correlation 8 cells, seed 0), x0 = 0, first {cycles} cycles of "
                       "Algorithm 1 (relative residual 1e-10 or the cap)",
           "plan_default": list(default)}
    runs = {}
    for name, plan in (("one_sweep", (0, 0, 1, 1)), ("default", default)):
        assert s.set_plan(*plan) == 0
        x = s.zeros()
        s.solve(x, tol=1e-10, max_cycles=2)
        x.zero_()
        out, dt = _timed(lambda: s.solve(x, tol=1e-10, max_cycles=cycles))
        runs[name] = (out, x.cpu().numpy())
        rec[name] = {"plan": list(plan), "cycles": out["cycles"], "sweeps": out["sweeps"],
                     "time_ms": round(dt * 1e3, 3),
                     "GLUPS": round(out["sweeps"] * prob.npoints / dt / 1e9, 3),
                     "final_rel_residual": float(out["norms"][-1] / out["r0"])}
        print(f"# c2 varcoef {name} {plan}: {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
    a, b = runs["one_sweep"], runs["default"]
    rec["bit_identical"] = bool(np.array_equal(a[0]["levels"], b[0]["levels"])
                                and np.array_equal(a[1], b[1]))
    rec["speedup"] = round(rec["one_sweep"]["time_ms"] / rec["default"]["time_ms"], 3)
    # to the tolerance with the default plans: plain binary64 and binary32-refined
    assert s.set_plan(*default) == 0
    rec["to_tol"] = {"tol": tol, "cap_cycles": tol_cycles, "plan_inner": list(s.get_plan(1))}
    for prec in ("f64", "f32"):
        x = s.zeros()
        s.solve(x, tol=tol, precision=prec, max_cycles=2)
        x.zero_()
        out, dt = _timed(lambda: s.solve(x, tol=tol, precision=prec, max_cycles=tol_cycles))
        rec["to_tol"][prec] = {"converged": out["converged"], "cycles": out["cycles"],
                               "sweeps": out["sweeps"], "time_ms": round(dt * 1e3, 3),
                               "GLUPS": round(out["sweeps"] * prob.npoints / dt / 1e9, 3),
                               "final_rel_residual_f64": s.residual_norm(x) / out["r0"]}
        print(f"# c2 varcoef to {tol:g} {prec}: {dt * 1e3:.1f} ms {out['status']}", file=sys.stderr,
              flush=True)
    s.close()
    return rec


def batch_once(which, prec):
    """One batched solve of workload 4 ("c4", binary32-refined) or 5 ("c5",
    `prec`) with a fixed plan, no autotuning and no loop of single solves:
    the run that the batched kernel traces are taken from."""
    import torch

    import workloads
    from paper_2011_06636_amd.solver import BatchSolver
    if which == "c4":
        bs = BatchSolver(workloads.c4())
        assert bs.set_plan(12, 8, 16, True, 8) == 0
        kw = dict(tol=1e-10, precision="f32", max_cycles=300)
    else:
        bs = BatchSolver(workloads.c5())
        bs.set_plan3d(8, 16, 2)
        kw = dict(tol=1e-8, precision=prec, max_cycles=300)
    out, dt = _timed(lambda: bs.solve(**kw))
    conv = sum(i["converged"] for i in out["instances"])
    plan = bs.get_plan() if which == "c4" else bs.get_plan3d()
    bs.close()
    torch.cuda.synchronize()
    return {"workload": which, "precision": kw["precision"], "plan": list(plan),
            "converged": conv, "instances": len(out["instances"]), "time_ms": round(dt * 1e3, 3)}


def extra_batch(which):
    """Batched solve vs a sequential loop of single-problem binary64 solves."""
    import numpy as np
    import torch

    import workloads
    from paper_2011_06636_amd.solver import BatchSolver, Solver
    if which == "c4":
        probs, precs, tol = workloads.c4(), ("f32",), 1e-10
        desc = ("512 2D Poisson squares, sides log-uniform in [64, 1024] (seed 1000+i), "
                "b ~ U(-1,1), relative residual 1e-10")
    else:
        probs, precs, tol = workloads.c5(), ("f64", "bf16"), 1e-8
        desc = ("128 3D anisotropic boxes, sides uniform in [32, 128], couplings (1, a, b), "
                "a, b log-uniform in [0.01, 1] (seed 2000+i), b ~ U(-1,1), relative residual "
                "1e-8")
    npts = sum(p.npoints for p in probs)
    bs = BatchSolver(probs)
    batched, best, xs_by_prec = [], None, {}
    for prec in precs:
        tune_us = bs.autotune(prec, sweeps=48)
        bs.solve(tol=tol, precision=prec, max_cycles=300)
        out, dt_b = _timed(lambda: bs.solve(tol=tol, precision=prec, max_cycles=300))
        conv_b = sum(i["converged"] for i in out["instances"])
        sweeps_b = sum(i["sweeps"] * p.npoints for i, p in zip(out["instances"], probs))
        rec = {"precision": prec, "time_ms": round(dt_b * 1e3, 3), "converged": conv_b,
               "GLUPS": round(sweeps_b / dt_b / 1e9, 3)}
        if which == "c4":
            rec |= {"plan": list(bs.get_plan()), "autotune_us_per_sweep": round(tune_us, 3)}
        else:
            rec |= {"plane_plan_rows_planes_sweeps": list(bs.get_plan3d()), "autotune_us_per_step": round(tune_us, 3)}
        batched.append(rec)
        xs_by_prec[prec] = [x.clone() for x in out["xs"]]
        if best is None or dt_b < best[0]:
            best = (dt_b, prec)
        print(f"# {which} batch {prec}: {dt_b * 1e3:.1f} ms, {conv_b}/{len(probs)}",
              file=sys.stderr, flush=True)
    bs.close()
    t_seq, conv_s, errs = 0.0, 0, {prec: [] for prec in precs}
    for k, p in enumerate(probs):
        s = Solver(p)
        x = s.zeros()
        if k == 0:
            s.solve(x, tol=tol, max_cycles=300)
            x.zero_()
        o, dt = _timed(lambda: s.solve(x, tol=tol, max_cycles=300))
        t_seq += dt
        conv_s += o["converged"]
        for prec in precs:
            errs[prec].append(float(torch.linalg.norm(xs_by_prec[prec][k] - x) / torch.linalg.norm(x)))
        s.close()
    print(f"# {which} sequential f64: {t_seq * 1e3:.1f} ms", file=sys.stderr, flush=True)
    # per-instance relative error of each batched form against the binary64
    # solves (which match the CPU oracle bit for bit)
    for rec in batched:
        e = errs[rec["precision"]]
        rec["rel_error_vs_sequential_f64"] = {"max": max(e), "median": float(np.median(e))}
        if which == "c5":
            rec["rel_error_vs_sequential_f64"]["per_instance"] = [float(f"{v:.3g}") for v in e]
    return {"workload": desc, "instances": len(probs), "points": npts, "batched": batched,
            "sequential_f64": {"time_ms": round(t_seq * 1e3, 3), "converged": conv_s},
            "fastest_batched": best[1],
            "batched_speedup_time_to_tol": round(t_seq / best[0], 3),
            "fastest_batched_rel_error_vs_sequential_f64": {
                "max": max(errs[best[1]]), "median": float(np.median(errs[best[1]]))}}


def extra_training(per_size=1_000_000, n_set=10000, z=1.96):
    """Section 3 on the GPU: selector training data at the paper's scale, the
    clusters, the rule fitted to them, and the CPU reference on a sample."""
    import numpy as np
    import torch

    import oracle
    import workloads
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import Solver
    sizes, flats, t_total, lups = [], [], 0.0, 0
    for N in workloads.TRAINING_SIZES:
        s = Solver(workloads.training_problem(N))
        # a pilot sizes the run: trials for about per_size tuples, step cap 2x the longest
        pilot = s.collect(torch.from_numpy(workloads.training_draws(256, 4000, seed=N)).cuda(),
                          compact=True)
        mean_steps = float(pilot["steps"].mean())
        max_steps = int(min(4000, 2 * int(pilot["steps"].max()) + 16))
        trials = int(np.ceil(per_size / (2.9 * mean_steps)))
        u = torch.from_numpy(workloads.training_draws(trials, max_steps, seed=1000 + N)).cuda()
        out, dt = _timed(lambda: s.collect(u, compact=True))
        s.close()
        flat = out["samples"][out["samples"]["M"] > 0]
        t_total += dt
        lups += (int(flat["M"].astype(np.int64).sum()) + trials) * N
        flats.append(flat)
        sizes.append({"N": N, "trials": trials, "tuples": int(len(flat)), "time_ms": round(dt * 1e3, 2),
                      "capped_trials": int((out["steps"] == max_steps).sum())})
        print(f"# training N={N}: {len(flat)} tuples, {dt * 1e3:.0f} ms", file=sys.stderr, flush=True)
    flat = np.concatenate(flats)
    clusters, t_cl = _timed(lambda: abi.srj_cluster_samples(flat, n_set=n_set, z=z))
    t_low, t_high, agree, decided = abi.srj_fit_rule(clusters)
    dec = clusters[clusters["best"] != abi.SRJ_ACTION_NONE]

    def agreement(lo, hi, cs=None):
        ok = 0
        for c in (dec if cs is None else cs):
            r = float(c["mean_ratio"])
            act = 1 if r > hi else (-1 if lo < r < hi else 0)
            ok += int(act == int(c["best"]))
        return ok
    # does the best action depend on the level?  one rule, scored level by level
    per_level = []
    for lv in range(25):
        cs = dec[dec["level"] == lv]
        if len(cs):
            per_level.append({"level": lv, "decided": int(len(cs)),
                              "agree_fitted": agreement(t_low, t_high, cs),
                              "agree_paper": agreement(0.2, 0.4, cs)})
    # CPU reference on a bounded sample: N = 100, 64 trials
    u = workloads.training_draws(64, 2000, seed=7)
    ref, t_ref = _timed(lambda: oracle.collect(workloads.training_problem(100), u))
    n_ref = int((ref["samples"]["M"] > 0).sum())
    gpu100 = next(r for r in sizes if r["N"] == 100)
    return {"workload": "section 3 data collection: 1D Poisson N in {2, 5, 10, 20, ..., 100, 200, "
                        "300, 400}, b = 1, x0 = 0, random branch per step (seeded draws), trials "
                        f"to about {per_size} tuples per size, stop at residual norm 1e-8; "
                        f"clusters of {n_set} tuples per level, {z} sigma intervals",
            "tuples": int(len(flat)), "time_ms": round(t_total * 1e3, 1),
            "tuples_per_s": round(len(flat) / t_total, 1), "GLUPS": round(lups / t_total / 1e9, 3),
            "sizes": sizes, "clusters": int(len(clusters)), "decided": int(decided),
            "cluster_time_ms": round(t_cl * 1e3, 1),
            "fitted_rule": {"t_low": t_low, "t_high": t_high, "agree": int(agree)},
            "paper_rule": {"t_low": 0.2, "t_high": 0.4, "agree": agreement(0.2, 0.4)},
            "per_level": per_level,
            "cpu_reference_sample": {"N": 100, "trials": 64, "tuples": n_ref,
                                     "time_ms": round(t_ref * 1e3, 1),
                                     "tuples_per_s": round(n_ref / t_ref, 1),
                                     "threads": oracle.num_threads(),
                                     "gpu_tuples_per_s_N100": round(gpu100["tuples"] * 1e3 /
                                                                    gpu100["time_ms"], 1)}}


def extra_neumann(sizes=(32, 64, 128, 256, 512, 1024), trials=10, tol=1e-10):
    """Section 4.2.2: 2D Laplace with Neumann boundaries from random starts,
    stopped by the largest update of a sweep; heuristic vs increasing rule."""
    import numpy as np
    import torch

    import oracle
    import workloads
    from paper_2011_06636_amd.solver import Solver
    rows = []
    for n in sizes:
        prob = workloads.neumann_laplace(n)
        s = Solver(prob)
        row = {"n": n, "unknowns": n * n}
        for rule in ("heuristic", "increasing"):
            sweeps, times = [], []
            for t in range(trials):
                x = s.to_device(workloads.random_start(prob, t))
                torch.cuda.synchronize()
                out, dt = _timed(lambda: s.solve(x, rule=rule, tol=tol, tol_mode="update_inf",
                                                 max_cycles=100000, max_sweeps=2_000_000))
                assert out["converged"], (n, rule, t)
                sweeps.append(out["sweeps"])
                times.append(dt)
            row[rule] = {"mean_sweeps": float(np.mean(sweeps)), "min_sweeps": int(min(sweeps)),
                         "max_sweeps": int(max(sweeps)), "mean_time_ms": round(1e3 * float(np.mean(times)), 3),
                         "GLUPS": round(sum(sweeps) * n * n / sum(times) / 1e9, 3)}
        s.close()
        rows.append(row)
        print(f"# neumann {n}: heuristic {row['heuristic']['mean_sweeps']:.0f} sweeps, increasing "
              f"{row['increasing']['mean_sweeps']:.0f}", file=sys.stderr, flush=True)
    prob = workloads.neumann_laplace(256)
    ref, t_ref = _timed(lambda: oracle.solve(prob, workloads.random_start(prob, 0), rule="heuristic",
                                             tol=tol, tol_mode="update_inf", max_cycles=100000))
    return {"workload": "2D Laplace, homogeneous Neumann (ghost-node central differences, rows "
                        "symmetrised), n x n nodes, b = 0, x0 ~ U(-1, 1) (seeds 0..9), stop when "
                        f"max |x' - x| of a sweep < {tol:g}", "trials": trials, "sizes": rows,
            "cpu_reference_sample": {"n": 256, "rule": "heuristic", "sweeps": ref["sweeps"],
                                     "time_ms": round(t_ref * 1e3, 1),
                                     "GLUPS": round(ref["sweeps"] * 256 * 256 / t_ref / 1e9, 3),
                                     "threads": oracle.num_threads()}}


def extra_general(big_h=0.003125):
    """Sections 4.2.1 and 4.2.4: random tridiagonal systems and finite element
    systems on unstructured meshes (heuristic vs increasing rule), and the
    sparse-matrix sweep's throughput on a large mesh."""
    import numpy as np

    import oracle
    import workloads
    from paper_2011_06636_amd.solver import Solver

    def run(prob, rule, tol):
        s = Solver(prob)
        x = s.zeros()
        s.solve(x, rule=rule, tol=tol, tol_mode="absolute", max_cycles=100000)
        x.zero_()
        out, dt = _timed(lambda: s.solve(x, rule=rule, tol=tol, tol_mode="absolute",
                                         max_cycles=100000))
        s.close()
        assert out["converged"], (prob.name, rule)
        return out["sweeps"], dt

    tri = []
    for N in (2, 5, 10, 20, 30, 40, 50, 60, 70, 80, 90, 100, 200, 300, 400, 500, 600, 700,
              800, 900, 1000):
        row = {"N": N}
        for rule in ("heuristic", "increasing"):
            sw = [run(workloads.random_tridiagonal(N, seed=k), rule, 1e-7)[0] for k in range(20)]
            row[rule] = float(np.mean(sw))
        tri.append(row)
    print("# tridiagonal: " + ", ".join(f"{r['N']}: {r['heuristic']:.0f}/{r['increasing']:.0f}"
                                        for r in tri), file=sys.stderr, flush=True)
    fem = []
    for geometry in ("disk", "plate_hole"):
        for h in (0.1, 0.05, 0.025):
            prob = workloads.fem_poisson(geometry, h, seed=0)
            row = {"geometry": geometry, "h": h, "unknowns": prob.npoints,
                   "nnz": int(len(prob.csr[2]))}
            for rule in ("heuristic", "increasing"):
                sw, dt = run(prob, rule, 1e-9)
                row[rule] = {"sweeps": sw, "time_ms": round(dt * 1e3, 3)}
            fem.append(row)
            print(f"# fem {geometry} h={h}: {prob.npoints} unknowns, heuristic "
                  f"{row['heuristic']['sweeps']} / increasing {row['increasing']['sweeps']} sweeps",
                  file=sys.stderr, flush=True)
    # throughput of the sparse sweep on a large mesh (one sweep per launch)
    big = workloads.fem_poisson("plate_hole", big_h, seed=0)
    n, nnz = big.npoints, int(len(big.csr[2]))
    s = Solver(big)
    x = s.zeros()
    s.run_cycle(x, 12)
    s.set_profiling(True)
    s.run_cycle(x, 12)
    ms, launches, sweeps = s.profile()
    s.set_profiling(False)
    kw = dict(tol=1e-9, tol_mode="absolute", max_cycles=100000)
    x.zero_()
    out, dt = _timed(lambda: s.solve(x, **kw))
    s.close()
    per_launch = ms / 1e3 / max(launches, 1)
    # compulsory bytes per row: x, b, D, 1/D, the row length, x' (8+8+8+8+4+8) and
    # 4 + 8 bytes per off-diagonal entry
    alg = 44.0 * n + 12.0 * (nnz - n)
    small = workloads.fem_poisson("plate_hole", 0.025, seed=0)
    ref, t_ref = _timed(lambda: oracle.solve(small, **kw))
    return {"workload": "random symmetric diagonally dominant tridiagonal systems (section "
                        "4.2.1, 20 per size, b ~ U(-1, 1), residual norm 1e-7) and -laplace(u) = 1 "
                        "with P1 finite elements on seeded Delaunay meshes of a disk and a plate "
                        "with a hole (section 4.2.4, residual norm 1e-9); sweeps counted at cycle "
                        "ends",
            "tridiagonal_mean_sweeps": tri, "fem": fem,
            "sparse_sweep": {"mesh": f"plate_hole h={big_h}", "rows": n, "nnz": nnz,
                             "avg_launch_us": round(per_launch * 1e6, 3),
                             "GLUPS": round(n / per_launch / 1e9, 3),
                             "alg_bytes_per_launch": alg,
                             "achieved_GBps": round(alg / per_launch / 1e9, 1),
                             "frac_of_8TBps": round(alg / per_launch / 1e9 / HBM_PEAK_GBS, 4),
                             "solve_sweeps": out["sweeps"], "solve_time_ms": round(dt * 1e3, 2)},
            "cpu_reference_sample": {"mesh": "plate_hole h=0.025", "rows": small.npoints,
                                     "sweeps": ref["sweeps"], "time_ms": round(t_ref * 1e3, 1),
                                     "GLUPS": round(ref["sweeps"] * small.npoints / t_ref / 1e9, 3),
                                     "threads": oracle.num_threads()}}


def leg_c1(runs=7, warmup=2):
    """1D Poisson N = 255 (h = 1/256), b ~ U(-1, 1) (seed 0), x0 = 0, relative
    residual 1e-10, Algorithm 1: the whole solve in one workgroup.  Median of
    `runs` timed solves after `warmup`, the oracle's time on the same input,
    and whether the levels and iterates agree."""
    import numpy as np

    import oracle
    import workloads
    from paper_2011_06636_amd.solver import Solver
    prob = workloads.c1()
    s = Solver(prob)
    x = s.zeros()
    for _ in range(warmup):
        x.zero_()
        s.solve(x, tol=1e-10)
    times = []
    for _ in range(runs):
        x.zero_()
        out, dt = _timed(lambda: s.solve(x, tol=1e-10))
        times.append(dt)
    xg = x.cpu().numpy()
    s.close()
    ref_t = []
    for _ in range(3):
        t0 = time.perf_counter()
        ref = oracle.solve(prob, tol=1e-10)
        ref_t.append(time.perf_counter() - t0)
    med = statistics.median(times)
    rec = {"workload": "1D Poisson, 3-point, N = 255, h = 1/256, b ~ U(-1, 1) (seed 0), x0 = 0, "
                       "relative residual 1e-10, Algorithm 1",
           "converged": bool(out["converged"]), "cycles": int(out["cycles"]),
           "sweeps": int(out["sweeps"]), "levels": [int(v) for v in out["levels"]],
           "time_to_tol_ms": {"median": round(med * 1e3, 4), "min": round(min(times) * 1e3, 4),
                              "max": round(max(times) * 1e3, 4), "runs": runs},
           "GLUPS": round(out["sweeps"] * prob.npoints / med / 1e9, 4),
           "oracle": {"time_to_tol_ms": round(statistics.median(ref_t) * 1e3, 4),
                      "threads": oracle.num_threads(), "cycles": int(ref["cycles"]),
                      "sweeps": int(ref["sweeps"])},
           "same_levels_as_oracle": bool(np.array_equal(out["levels"], ref["levels"])),
           "max_abs_diff_vs_oracle": float(np.max(np.abs(xg.ravel() - ref["x"].ravel())))}
    rec["speedup_vs_oracle"] = round(rec["oracle"]["time_to_tol_ms"] / rec["time_to_tol_ms"]["median"], 2)
    return rec


def leg_out_of_cache(n=8192, level=12):
    """The 2D binary64 sweep on an n x n grid (C2's recipe, seed 0) whose x, x'
    and b (3 x 8 n^2 bytes) do not fit the 256 MB Infinity Cache: one cycle of
    `level` with the default block plan, the single-sweep plan and the generic
    one-sweep kernel, against the library's streaming kernels on arrays of
    the same size."""
    import torch

    import workloads
    from paper_2011_06636_amd.solver import Solver
    ceil = stream_ceiling(n * n)
    prob = workloads.c2(n=n)
    s = Solver(prob)
    x = s.zeros()
    plan = tuple(s.get_plan(0))
    ref = ceil["read2_write1_GBps"]
    rec = {"workload": f"2D Poisson 5-point {n}x{n} (b = 8 sine modes + noise, seed 0), one "
                       f"cycle of level {level} per plan from x0 = 0",
           "working_set_MB": round(3 * 8 * n * n / 1e6, 1), "stream_ceiling": ceil,
           "default": plan_rate(s, x, prob, plan, level, ref),
           "single_sweep": plan_rate(s, x, prob, ONE_SWEEP_PLAN, level, ref),
           "unfused_one_sweep": plan_rate(s, x, prob, (0, 0, 1, 1), level, ref)}
    s.close()
    del x
    torch.cuda.empty_cache()
    return rec


def leg_multigrid(runs=5):
    """SRJ as the smoother of a multigrid V-cycle (section 5 names the use):
    2D Poisson 2047^2 (the C2 recipe on an odd grid, seed 0) and 3D Poisson
    255^3 (b ~ U(-1, 1), seed 0), V-cycles with Algorithm 1 choosing the
    smoothing scheme, to relative 1e-10, against plain binary64 SRJ on the
    same problem (2D to the tolerance both reach, 2e-9; 3D to 1e-10).  The
    CPU oracle's multigrid on 255^2 sits beside it with its time and the GPU's
    agreement on that grid."""
    import numpy as np
    import torch

    import oracle
    import workloads
    from paper_2011_06636_amd.solver import MgSolver, Solver

    def med(fn):
        fn()
        ts, out = [], None
        for _ in range(runs):
            out, dt = _timed(fn)
            ts.append(dt)
        return out, statistics.median(ts)

    recs = {}
    rng = np.random.default_rng(0)
    cases = [("2d_2047", workloads.c2(n=2047), 2e-9),
             ("3d_255", workloads.poisson([255, 255, 255], b=rng.uniform(-1, 1, (255, 255, 255))), 1e-10)]
    for name, prob, srj_tol in cases:
        m = MgSolver(prob)
        x = m.zeros()

        def mg_run(tol):
            x.zero_()
            return m.solve(x, tol=tol)
        out, t_mg = med(lambda: mg_run(1e-10))
        outc, t_mgc = med(lambda: mg_run(srj_tol))
        m.close()
        del x
        s = Solver(prob)
        y = s.zeros()

        def srj_run():
            y.zero_()
            return s.solve(y, tol=srj_tol, max_cycles=300)
        ref, t_srj = med(srj_run)
        s.close()
        del y
        torch.cuda.empty_cache()
        recs[name] = {
            "grid": list(prob.n[:prob.ndim]), "grid_levels": out["levels_grid"],
            "mg_to_1e-10": {"converged": out["converged"], "vcycles": out["vcycles"],
                            "smoothing_levels": [int(v) for v in out["levels"]],
                            "fine_sweeps": out["sweeps"], "coarse_sweeps": out["coarse_sweeps"],
                            "work_fine_sweep_equivalents": round(out["work"], 2),
                            "time_ms": round(t_mg * 1e3, 3),
                            "final_rel_residual": float(out["r_final"] / out["r0"])},
            "common_tol": srj_tol,
            "mg_to_common_tol": {"vcycles": outc["vcycles"], "time_ms": round(t_mgc * 1e3, 3),
                                 "work_fine_sweep_equivalents": round(outc["work"], 2)},
            "srj_f64_to_common_tol": {"converged": ref["converged"], "cycles": ref["cycles"],
                                      "sweeps": ref["sweeps"], "time_ms": round(t_srj * 1e3, 3)},
            "mg_speedup_at_common_tol": round(t_srj / t_mgc, 2)}
        print(f"# multigrid {name}: {t_mgc * 1e3:.2f} ms vs SRJ {t_srj * 1e3:.1f} ms",
              file=sys.stderr, flush=True)
    # the oracle's multigrid on a smaller grid, and the GPU's agreement there
    small = workloads.c2(n=255)
    t0 = time.perf_counter()
    ro = oracle.mg_solve(small, rule="heuristic", start_level=0, tol=1e-10)
    t_or = time.perf_counter() - t0
    m = MgSolver(small)
    go = m.solve(tol=1e-10)
    xg = go["x"].cpu().numpy()
    m.close()
    recs["cpu_reference_sample"] = {
        "grid": [255, 255], "vcycles": ro["vcycles"], "time_ms": round(t_or * 1e3, 1),
        "threads": oracle.num_threads(),
        "gpu_same_levels": bool(np.array_equal(go["levels"], ro["levels"])),
        "gpu_bit_identical": bool(np.array_equal(xg, ro["x"]))}
    return {"workload": "multigrid V-cycles with SRJ smoothing: full weighting, multilinear "
                        "interpolation, coarse couplings / 4, one pre- and one post-cycle, "
                        "coarsest grid by SRJ to 1e-8", "cases": recs}


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


def summary(times, results, prob, x=None, s=None):
    """Per-solve record of a timed leg: status, counters, median and mean time."""
    last = results[-1]
    rec = {"converged": bool(last["converged"]), "cycles": int(last["cycles"]),
           "sweeps": int(last["sweeps"]),
           "time_ms": round(sum(times) / len(times) * 1e3, 3),
           "median_ms": round(statistics.median(times) * 1e3, 3),
           "GLUPS": round(sum(r["sweeps"] for r in results) * prob.npoints / sum(times) / 1e9, 3),
           "final_rel_residual": float(last["norms"][-1] / last["r0"])}
    if s is not None and x is not None:
        rec["final_rel_residual_f64_recomputed"] = s.residual_norm(x) / last["r0"]
    return rec


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the library runs on one GPU; sharding over several is designed, not built)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe_mib > 0:
        # one streaming copy of exactly copy_probe_mib MiB each way: the
        # reference dispatch that scales FETCH_SIZE and WRITE_SIZE
        n_el = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n_el, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        abi.srj_stream_probe(0, src.data_ptr(), src.data_ptr(), dst.data_ptr(), n_el,
                             torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        del src, dst
    if args.only:
        legs = {"c1": leg_c1, "ooc": lambda: leg_out_of_cache(args.ooc_n), "mg": leg_multigrid,
                "c3": lambda: extra_c3(args.c3_cycles), "c4": lambda: extra_batch("c4"),
                "c5": lambda: extra_batch("c5"), "c2vc": extra_c2_varcoef,
                "training": extra_training,
                "neumann": extra_neumann, "general": extra_general,
                "c4once": lambda: batch_once("c4", "f32"),
                "c5once": lambda: batch_once("c5", args.precision)}
        print(json.dumps({"only": args.only, "record": legs[args.only]()}), flush=True)
        return
    prob = workloads.c2(n=args.n)
    s = Solver(prob)
    if args.plan:
        assert s.set_plan(*(int(v) for v in args.plan.split(":"))) == 0, "plan not supported"
    plan = s.get_plan(0)
    plan_inner = s.get_plan(1)
    x = s.zeros()
    print(f"# workload c2 {args.n}x{args.n}, plans f64 {plan} inner {plan_inner}",
          file=sys.stderr, flush=True)
    tol, ctol = args.tol, args.common_tol

    # plain binary64 SRJ to the common tolerance: the timed steps and the headline GLUPS
    kw64 = dict(tol=ctol, max_cycles=args.max_cycles)
    times, results, (sweep_ms, launches, prof_sweeps) = run_leg(
        s, x, kw64, args.steps, args.warmup, "f64")
    total = sum(times)
    sweeps = sum(r["sweeps"] for r in results)
    glups = sweeps * prob.npoints / total / 1e9
    f64c = summary(times, results, prob, x, s)
    last = results[-1]
    f64_time = total / args.steps

    # binary32-refined SRJ: to the common tolerance and to the target
    steps_b = max(3, args.steps // 2)
    t32c, r32c, _ = run_leg(s, x, dict(tol=ctol, max_cycles=args.max_cycles, precision="f32"),
                            steps_b, 1, "f32 common")
    f32c = summary(t32c, r32c, prob, x, s)
    t32, r32, _ = run_leg(s, x, dict(tol=tol, max_cycles=args.max_cycles, precision="f32"),
                          steps_b, 1, "f32")
    f32t = summary(t32, r32, prob, x, s)
    f32t["levels"] = [int(v) for v in r32[-1]["levels"]]

    # plain binary64 to the target, capped: where binary64 round-off stops it
    tcap, rcap, _ = run_leg(s, x, dict(tol=tol, max_cycles=args.max_cycles), 1, 0, "f64 capped")
    capped = summary(tcap, rcap, prob, x, s)
    rel = rcap[-1]["norms"] / rcap[-1]["r0"]
    best = int(np.argmin(rel))
    capped.update({"cap_cycles": args.max_cycles, "best_rel_residual": float(rel[best]),
                   "cycle_of_best": best, "levels": [int(v) for v in rcap[-1]["levels"]]})

    # dominant kernel of the timed binary64 steps: the relaxation launches.
    # Algorithmic bytes per launch: read x and b, write x' once (binary64):
    # 24 B per point, whatever the number of sweeps fused into the launch.
    avg_launch_s = sweep_ms / 1e3 / max(launches, 1)
    alg_bytes = 24.0 * prob.npoints
    achieved = alg_bytes / avg_launch_s / 1e9
    ceil = stream_ceiling(prob.npoints)
    ref = ceil["read2_write1_GBps"]
    unfused = plan_rate(s, x, prob, (0, 0, 1, 1), ceiling=ref)
    single = plan_rate(s, x, prob, ONE_SWEEP_PLAN, ceiling=ref)
    s.close()
    del x
    torch.cuda.empty_cache()
    c1 = leg_c1()
    print(f"# c1: {c1['time_to_tol_ms']['median']} ms median", file=sys.stderr, flush=True)
    ooc = leg_out_of_cache(args.ooc_n) if args.ooc_n > 0 else None
    if ooc:
        print(f"# out of cache {args.ooc_n}: default {ooc['default']['frac']} single "
              f"{ooc['single_sweep']['frac']} of 8 TB/s", file=sys.stderr, flush=True)
    rec = {
        "metric": "GLUPS + time-to-1e-10 residual: plain FP64 SRJ vs FP32-refined/batched, 1 GPU",
        "value": round(glups, 3), "unit": "GLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(f64_time * 1e3, 3),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D Poisson 5-point {args.n}x{args.n}, b = 8 sine modes + "
                               f"U(-1e-3,1e-3) noise (seed 0), x0 = 0, Algorithm 1 level choice; "
                               f"one step = plain FP64 SRJ solve to relative residual {ctol:g} "
                               f"(FP64 round-off floor ~1.4e-9 on this grid, above {tol:g})",
                   "grid": [args.n, args.n], "tol": tol, "common_tol": ctol,
                   "plan_f64": list(plan), "plan_inner": list(plan_inner)},
        "f64_to_common_tol": f64c | {"levels": [int(v) for v in last["levels"]]},
        "f32_refined_to_common_tol": f32c,
        "f32_refined_to_tol": f32t,
        "f64_capped_to_tol": capped,
        "time_to_tol_ms": {"common_tol": ctol, "f64_at_common_tol": f64c["time_ms"],
                           "f32_refined_at_common_tol": f32c["time_ms"],
                           "f32_refined_speedup_at_common_tol":
                               round(f64c["time_ms"] / f32c["time_ms"], 3),
                           "tol": tol, "f64": None if not capped["converged"] else capped["time_ms"],
                           "f64_note": f"FP64 does not reach {tol:g}: best relative residual "
                                       f"{rel[best]:.3g} at cycle {best} of {args.max_cycles}",
                           "f32_refined": f32t["time_ms"] if f32t["converged"] else None},
        "c1_1d": c1,
        "out_of_cache_2d": ooc,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(plan) if args.n == 2048 else None,
                     "kernel": KERNEL_NAMES.get(plan[0], f"plan kind {plan[0]}"),
                     "sweeps_per_launch": round(prof_sweeps / max(launches, 1), 3),
                     "avg_launch_us": round(avg_launch_s * 1e6, 3),
                     "bytes_per_launch": alg_bytes,
                     "kernel_GLUPS": round(prof_sweeps * prob.npoints / (sweep_ms / 1e3) / 1e9, 1),
                     "effective_GBps_per_sweep": round(24.0 * glups, 1),
                     "stream_ceiling_same_arrays": ceil,
                     "frac_of_stream_ceiling": round(achieved / ref, 4),
                     "in_cache": "x, x' and b of 2048^2 (101 MB) fit the 256 MB Infinity Cache; "
                                 "out_of_cache_2d holds the same kernels on 8192^2",
                     "unfused_one_sweep": unfused,
                     "single_sweep_best": single,
                     "valu_issue": valu_issue(plan, prob.npoints, prof_sweeps, launches,
                                              avg_launch_s)},
    }
    if not args.no_extras:
        rec["extras"] = {"c3_3d_varcoef": extra_c3(args.c3_cycles), "c4_batch_2d": extra_batch("c4"),
                         "c5_batch_3d": extra_batch("c5"), "c2_2d_varcoef": extra_c2_varcoef(),
                         "selector_training": extra_training(),
                         "neumann_update_test": extra_neumann(),
                         "general_matrices": extra_general(),
                         "multigrid_srj_smoother": leg_multigrid()}
    if args.cpu_seconds > 0:
        rec["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds, last["levels"], last["norms"])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
