"""ctypes binding of libsrj.so (the C ABI declared in include/srj.h).

Argument marshalling only: every step of the solver runs in the HIP library.
The functions keep the C names (srj_setup, srj_run_cycle, srj_solve, ...).
If libsrj.so has not been built, load() raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# SRJ_LIB_PATH selects another build of the same library (the host-sanitizer
# build of sanitize_build.py); by default the in-tree libsrj.so
LIB_PATH = os.environ.get("SRJ_LIB_PATH") or os.path.join(HERE, "libsrj.so")

SRJ_OK = 0
SRJ_ERR_INVALID = 1
SRJ_ERR_NOMEM = 2
SRJ_ERR_HIP = 3
SRJ_ERR_NOT_CONVERGED = 4
SRJ_ERR_NONFINITE = 5
SRJ_ERR_UNSUPPORTED = 6
STATUS_NAMES = {0: "ok", 1: "invalid", 2: "nomem", 3: "hip", 4: "not_converged",
                5: "nonfinite", 6: "unsupported"}

PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
RULE = {"heuristic": 0, "increasing": 1, "fixed": 2}
TOL_MODE = {"relative": 0, "absolute": 1, "update_inf": 2}
NUM_LEVELS = 25
MAX_M = 2362

# Public entry points of include/srj.h (checked by the tests).
EXPORTS = [
    "srj_default_opts", "srj_scheme", "srj_setup", "srj_setup_csr", "srj_run_cycle",
    "srj_residual_norm", "srj_residual_norm_noalloc",
    "srj_solve", "srj_destroy", "srj_set_plan", "srj_get_plan", "srj_plan_variants",
    "srj_autotune", "srj_set_resident",
    "srj_set_profiling",
    "srj_get_profile", "srj_batch_setup", "srj_batch_set_plan", "srj_batch_get_plan",
    "srj_batch_set_plan3d", "srj_batch_get_plan3d",
    "srj_batch_autotune",
    "srj_batch_solve", "srj_batch_destroy", "srj_collect", "srj_cluster_samples",
    "srj_fit_rule", "srj_set_scheme_family", "srj_last_error", "srj_stream_probe",
    "srj_mg_default_opts", "srj_mg_setup", "srj_mg_solve", "srj_mg_destroy",
]

SRJ_ACTION_NONE = 2


class SrjProblem(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
                ("cconst", ctypes.c_double * 3), ("face", ctypes.c_void_p * 3),
                ("dconst", ctypes.c_double), ("diag", ctypes.c_void_p), ("b", ctypes.c_void_p)]


class SrjCsrProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("b", ctypes.c_void_p)]


class SrjSolveOpts(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("fixed_level", ctypes.c_int32),
                ("tol_mode", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_cycles", ctypes.c_int32), ("max_sweeps", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("start_level", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("scale_target", ctypes.c_double),
                ("r0", ctypes.c_double)]


class SrjSolveResult(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("final_level", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sweeps", ctypes.c_int64), ("r0", ctypes.c_double),
                ("r_final", ctypes.c_double), ("min_margin", ctypes.c_double)]


class SrjMgOpts(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("start_level", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("pre", ctypes.c_int32), ("post", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("coarse_tol", ctypes.c_double),
                ("coarse_max_cycles", ctypes.c_int32), ("tol_mode", ctypes.c_int32),
                ("tol", ctypes.c_double), ("max_vcycles", ctypes.c_int32)]


class SrjMgResult(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("vcycles", ctypes.c_int32),
                ("final_level", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("sweeps", ctypes.c_int64), ("coarse_sweeps", ctypes.c_int64),
                ("work", ctypes.c_double), ("r0", ctypes.c_double), ("r_final", ctypes.c_double)]


class SrjSample(ctypes.Structure):
    _fields_ = [("trial", ctypes.c_int32), ("step", ctypes.c_int32), ("level", ctypes.c_int32),
                ("action", ctypes.c_int32), ("M", ctypes.c_int32), ("chosen", ctypes.c_int32),
                ("prev_ratio", ctypes.c_double), ("r_before", ctypes.c_double),
                ("r_after", ctypes.c_double)]


class SrjCluster(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("count", ctypes.c_int32),
                ("mean_ratio", ctypes.c_double), ("best", ctypes.c_int32),
                ("n", ctypes.c_int32 * 3), ("mean_rate", ctypes.c_double * 3),
                ("half_width", ctypes.c_double * 3)]


# numpy views of the same layouts (for device buffers copied to the host)
SAMPLE_DTYPE = [("trial", "<i4"), ("step", "<i4"), ("level", "<i4"), ("action", "<i4"),
                ("M", "<i4"), ("chosen", "<i4"), ("prev_ratio", "<f8"), ("r_before", "<f8"),
                ("r_after", "<f8")]
CLUSTER_DTYPE = [("level", "<i4"), ("count", "<i4"), ("mean_ratio", "<f8"), ("best", "<i4"),
                 ("n", "<i4", (3,)), ("mean_rate", "<f8", (3,)), ("half_width", "<f8", (3,))]


_lib = None


def load() -> ctypes.CDLL:
    """Load libsrj.so; raises if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__; __graft_entry__.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "srj_default_opts": (None, [P(SrjSolveOpts)]),
        "srj_scheme": (i32, [i32, P(f64), i32, P(i32)]),
        "srj_setup": (i32, [P(SrjProblem), vp, P(vp)]),
        "srj_run_cycle": (i32, [vp, vp, i32, P(f64)]),
        "srj_residual_norm": (i32, [vp, vp, P(f64)]),
        "srj_residual_norm_noalloc": (i32, [P(SrjProblem), vp, vp, vp]),
        "srj_solve": (i32, [vp, vp, P(SrjSolveOpts), P(SrjSolveResult), P(i32), P(f64)]),
        "srj_destroy": (i32, [vp]),
        "srj_set_plan": (i32, [vp, i32, i32, i32, i32, i32]),
        "srj_get_plan": (i32, [vp, i32, P(i32), P(i32), P(i32), P(i32)]),
        "srj_plan_variants": (i32, [i32, P(i32), i32, P(i32)]),
        "srj_autotune": (i32, [vp, i32, i32, i32, P(f64)]),
        "srj_set_resident": (i32, [vp, i32]),
        "srj_set_profiling": (i32, [vp, i32]),
        "srj_get_profile": (i32, [vp, P(f64), P(i64), P(i64)]),
        "srj_batch_setup": (i32, [i32, P(SrjProblem), vp, P(vp)]),
        "srj_batch_set_plan": (i32, [vp, i32, i32, i32, i32, i32]),
        "srj_batch_get_plan": (i32, [vp, P(i32), P(i32), P(i32), P(i32), P(i32)]),
        "srj_batch_set_plan3d": (i32, [vp, i32, i32, i32]),
        "srj_batch_get_plan3d": (i32, [vp, P(i32), P(i32), P(i32)]),
        "srj_batch_autotune": (i32, [vp, i32, i32, P(f64)]),
        "srj_batch_solve": (i32, [vp, P(vp), P(SrjSolveOpts), P(SrjSolveResult), P(i32)]),
        "srj_batch_destroy": (i32, [vp]),
        "srj_setup_csr": (i32, [P(SrjCsrProblem), vp, P(vp)]),
        "srj_set_scheme_family": (i32, [vp, i32, P(i32), P(f64)]),
        "srj_collect": (i32, [vp, i32, i32, vp, f64, i32, vp, vp]),
        "srj_cluster_samples": (i32, [vp, ctypes.c_int64, i32, f64, vp, i32, P(i32)]),
        "srj_fit_rule": (i32, [vp, i32, P(f64), P(f64), P(i32), P(i32)]),
        "srj_last_error": (ctypes.c_char_p, []),
        "srj_stream_probe": (i32, [i32, vp, vp, vp, i64, vp]),
        "srj_mg_default_opts": (None, [P(SrjMgOpts)]),
        "srj_mg_setup": (i32, [P(SrjProblem), vp, P(vp)]),
        "srj_mg_solve": (i32, [vp, vp, P(SrjMgOpts), P(SrjMgResult), P(i32), P(f64)]),
        "srj_mg_destroy": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().srj_last_error().decode()


class SrjError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {last_error()}")


def check(status: int, where: str, ok=(SRJ_OK,)) -> int:
    if status not in ok:
        raise SrjError(status, where)
    return status


# Thin wrappers with the C names ------------------------------------------------

def srj_default_opts() -> SrjSolveOpts:
    o = SrjSolveOpts()
    load().srj_default_opts(ctypes.byref(o))
    return o


def srj_scheme(level: int):
    buf = (ctypes.c_double * MAX_M)()
    M = ctypes.c_int32()
    check(load().srj_scheme(level, buf, MAX_M, ctypes.byref(M)), "srj_scheme")
    return [buf[i] for i in range(M.value)]


def srj_setup(prob: SrjProblem, stream: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(load().srj_setup(ctypes.byref(prob), ctypes.c_void_p(stream), ctypes.byref(h)),
          "srj_setup")
    return h


def srj_setup_csr(prob: SrjCsrProblem, stream: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(load().srj_setup_csr(ctypes.byref(prob), ctypes.c_void_p(stream), ctypes.byref(h)),
          "srj_setup_csr")
    return h


def srj_run_cycle(ctx, x_ptr: int, level: int) -> float:
    nrm = ctypes.c_double()
    check(load().srj_run_cycle(ctx, ctypes.c_void_p(x_ptr), level, ctypes.byref(nrm)),
          "srj_run_cycle")
    return nrm.value


def srj_residual_norm(ctx, x_ptr: int) -> float:
    nrm = ctypes.c_double()
    check(load().srj_residual_norm(ctx, ctypes.c_void_p(x_ptr), ctypes.byref(nrm)),
          "srj_residual_norm")
    return nrm.value


def srj_residual_norm_noalloc(prob: SrjProblem, x_ptr: int, stream: int, norm_ptr: int) -> None:
    """Enqueues ||b - A x|| into the device double at norm_ptr (no allocation, no sync)."""
    check(load().srj_residual_norm_noalloc(ctypes.byref(prob), ctypes.c_void_p(x_ptr),
                                           ctypes.c_void_p(stream), ctypes.c_void_p(norm_ptr)),
          "srj_residual_norm_noalloc")


def srj_stream_probe(kind: int, a_ptr: int, b_ptr, out_ptr: int, n: int, stream: int) -> None:
    """One streaming launch (0: copy, 1: a + b) of n binary64 values on `stream`."""
    check(load().srj_stream_probe(kind, ctypes.c_void_p(a_ptr), ctypes.c_void_p(b_ptr),
                                  ctypes.c_void_p(out_ptr), n, ctypes.c_void_p(stream)),
          "srj_stream_probe")


def srj_mg_default_opts() -> SrjMgOpts:
    o = SrjMgOpts()
    load().srj_mg_default_opts(ctypes.byref(o))
    return o


def srj_mg_setup(prob: SrjProblem, stream: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(load().srj_mg_setup(ctypes.byref(prob), ctypes.c_void_p(stream), ctypes.byref(h)),
          "srj_mg_setup")
    return h


def srj_mg_solve(mg, x_ptr: int, opts: SrjMgOpts, levels=None, norms=None):
    res = SrjMgResult()
    st = load().srj_mg_solve(mg, ctypes.c_void_p(x_ptr), ctypes.byref(opts), ctypes.byref(res),
                             levels, norms)
    return st, res


def srj_mg_destroy(mg) -> None:
    if mg:
        load().srj_mg_destroy(mg)


def srj_solve(ctx, x_ptr: int, opts: SrjSolveOpts, levels=None, norms=None):
    res = SrjSolveResult()
    st = load().srj_solve(ctx, ctypes.c_void_p(x_ptr), ctypes.byref(opts), ctypes.byref(res),
                          levels, norms)
    return st, res


def srj_set_plan(ctx, kind: int, tile_rows: int = 0, sweeps: int = 1, occ: int = 1,
                 which: int = 0) -> int:
    return load().srj_set_plan(ctx, which, kind, tile_rows, sweeps, occ)


def srj_get_plan(ctx, which: int = 0):
    k, r, t, o = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(load().srj_get_plan(ctx, which, ctypes.byref(k), ctypes.byref(r), ctypes.byref(t),
                              ctypes.byref(o)), "srj_get_plan")
    return k.value, r.value, t.value, o.value


def srj_plan_variants(which: int = 0):
    """Fused kernel variants as (kind, tile_rows, max sweeps per launch, waves_per_simd)."""
    buf = (ctypes.c_int32 * 512)()
    n = ctypes.c_int32()
    check(load().srj_plan_variants(which, buf, 128, ctypes.byref(n)), "srj_plan_variants")
    return [tuple(buf[4 * i:4 * i + 4]) for i in range(min(n.value, 128))]


def srj_autotune(ctx, which: int = 0, sweeps: int = 48, use_cache: bool = True) -> float:
    us = ctypes.c_double()
    check(load().srj_autotune(ctx, which, sweeps, 1 if use_cache else 0, ctypes.byref(us)),
          "srj_autotune")
    return us.value


def srj_set_resident(ctx, enable: bool) -> int:
    return load().srj_set_resident(ctx, 1 if enable else 0)


def srj_set_profiling(ctx, enable: bool) -> None:
    check(load().srj_set_profiling(ctx, 1 if enable else 0), "srj_set_profiling")


def srj_get_profile(ctx):
    ms, la, sw = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
    check(load().srj_get_profile(ctx, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(sw)),
          "srj_get_profile")
    return ms.value, la.value, sw.value


def srj_destroy(ctx) -> None:
    if ctx:
        load().srj_destroy(ctx)


def srj_batch_setup(probs, stream: int = 0):
    arr = (SrjProblem * len(probs))(*probs)
    h = ctypes.c_void_p()
    st = load().srj_batch_setup(len(probs), arr, ctypes.c_void_p(stream), ctypes.byref(h))
    return st, h


def srj_batch_set_plan(batch, tile_rows: int, sweeps: int, waves_per_block: int = 1,
                       steps_per_graph: int = 16, use_graph: bool = True) -> int:
    return load().srj_batch_set_plan(batch, tile_rows, sweeps, waves_per_block, steps_per_graph,
                                     1 if use_graph else 0)


def srj_batch_get_plan(batch):
    v = [ctypes.c_int32() for _ in range(5)]
    check(load().srj_batch_get_plan(batch, *[ctypes.byref(a) for a in v]), "srj_batch_get_plan")
    return tuple(a.value for a in v)


def srj_batch_set_plan3d(batch, tile_rows: int, planes: int, sweeps: int = 2) -> None:
    check(load().srj_batch_set_plan3d(batch, tile_rows, planes, sweeps), "srj_batch_set_plan3d")


def srj_batch_get_plan3d(batch):
    v = [ctypes.c_int32() for _ in range(3)]
    check(load().srj_batch_get_plan3d(batch, *[ctypes.byref(a) for a in v]), "srj_batch_get_plan3d")
    return tuple(a.value for a in v)


def srj_batch_autotune(batch, precision: str = "f32", sweeps: int = 48) -> float:
    us = ctypes.c_double()
    check(load().srj_batch_autotune(batch, PREC[precision], sweeps, ctypes.byref(us)),
          "srj_batch_autotune")
    return us.value


def srj_batch_solve(batch, x_ptrs, opts: SrjSolveOpts, levels=None):
    n = len(x_ptrs)
    xs = (ctypes.c_void_p * n)(*[ctypes.c_void_p(p) for p in x_ptrs])
    res = (SrjSolveResult * n)()
    st = load().srj_batch_solve(batch, xs, ctypes.byref(opts), res, levels)
    return st, res


def srj_batch_destroy(batch) -> None:
    if batch:
        load().srj_batch_destroy(batch)


def srj_collect(ctx, trials: int, max_steps: int, u_ptr: int, tol: float, max_level: int,
                samples_ptr: int, steps_ptr: int) -> None:
    """Device pointers: u (trials * max_steps), samples (trials * max_steps * 3), steps."""
    check(load().srj_collect(ctx, trials, max_steps, u_ptr, tol, max_level, samples_ptr,
                             steps_ptr), "srj_collect")


def srj_cluster_samples(samples, n_set: int = 10000, z: float = 1.96):
    """samples: numpy array of SAMPLE_DTYPE (host); returns a CLUSTER_DTYPE array."""
    import numpy as np
    samples = np.ascontiguousarray(samples, dtype=SAMPLE_DTYPE)
    n = ctypes.c_int32()
    cap = len(samples) // max(n_set, 1) + 1  # bound on the number of whole clusters
    out = np.zeros(cap, dtype=CLUSTER_DTYPE)
    check(load().srj_cluster_samples(samples.ctypes.data if len(samples) else None, len(samples),
                                     n_set, z, out.ctypes.data, cap, ctypes.byref(n)),
          "srj_cluster_samples")
    return out[:n.value]


def srj_fit_rule(clusters):
    """clusters: CLUSTER_DTYPE array; returns (t_low, t_high, agree, decided)."""
    import numpy as np
    clusters = np.ascontiguousarray(clusters, dtype=CLUSTER_DTYPE)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    ag, de = ctypes.c_int32(), ctypes.c_int32()
    check(load().srj_fit_rule(clusters.ctypes.data if len(clusters) else None, len(clusters),
                              ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(ag),
                              ctypes.byref(de)), "srj_fit_rule")
    return lo.value, hi.value, ag.value, de.value


def srj_set_scheme_family(ctx, levels=None) -> None:
    """levels: list of factor sequences (one per level, in application order);
    None or [] restores the paper's family."""
    if not levels:
        check(load().srj_set_scheme_family(ctx, 0, None, None), "srj_set_scheme_family")
        return
    M = (ctypes.c_int32 * len(levels))(*[len(w) for w in levels])
    flat = [float(v) for w in levels for v in w]
    om = (ctypes.c_double * len(flat))(*flat)
    check(load().srj_set_scheme_family(ctx, len(levels), M, om), "srj_set_scheme_family")
