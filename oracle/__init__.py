"""CPU reference (the oracle) of the SRJ method with the data-driven selector.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark import this package.  It wraps ``srj_oracle.c``
(plain binary64 loops, written from the paper's equations) through ctypes and
shares no code with the GPU library in ``paper_2011_06636_amd``.

Paper references (Islam & Wang, arXiv 2011.06636):
  * scheme factors: section 2, Eq. (17); levels: Appendix B;
  * order of the factors in a cycle: section 2, last paragraph (Leja order);
  * sweep: section 2, Eq. 3; cycle: Eq. 7;
  * residual after each cycle: section 3; relative residual: Eq. (27);
  * selector: section 3, Algorithm 1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "srj_oracle.c")
_SRC_MG = os.path.join(_HERE, "srj_mg.c")
# SRJ_ORACLE_LIB selects another build of the same source (the sanitizer
# build); by default the in-tree liboracle.so
_LIB = os.environ.get("SRJ_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

RULES = {"heuristic": 0, "increasing": 1, "fixed": 2, "jacobi": 3}
TOL_MODES = {"relative": 0, "absolute": 1, "update_inf": 2}
PRECISIONS = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
STATUS = {0: "ok", 1: "invalid", 4: "not_converged", 5: "nonfinite"}


def build(force: bool = True) -> str:
    """Compile srj_oracle.c into oracle/liboracle.so (gcc, -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, _SRC_MG, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("c", ctypes.c_double * 3),
                ("face", ctypes.c_void_p * 3), ("dconst", ctypes.c_double),
                ("diag", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("fixed_level", ctypes.c_int32),
                ("tol_mode", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_cycles", ctypes.c_int32), ("max_sweeps", ctypes.c_int64),
                ("stop_per_sweep", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("start_level", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("scale_target", ctypes.c_double)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("cycles", ctypes.c_int32), ("final_level", ctypes.c_int32),
                ("sweeps", ctypes.c_int64), ("r0", ctypes.c_double),
                ("r_final", ctypes.c_double), ("min_margin", ctypes.c_double)]


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.srjo_level_M.restype = ctypes.c_int32
        lib.srjo_level_M.argtypes = [ctypes.c_int32]
        lib.srjo_omega_natural.argtypes = [ctypes.c_int32, P(ctypes.c_double)]
        lib.srjo_leja_order.argtypes = [ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_int32)]
        lib.srjo_scheme.restype = ctypes.c_int32
        lib.srjo_scheme.argtypes = [ctypes.c_int32, P(ctypes.c_double)]
        lib.srjo_sweep.argtypes = [P(_Problem), P(ctypes.c_double), ctypes.c_double,
                                   P(ctypes.c_double)]
        lib.srjo_residual_norm.restype = ctypes.c_double
        lib.srjo_residual_norm.argtypes = [P(_Problem), P(ctypes.c_double)]
        lib.srjo_apply.argtypes = [P(_Problem), P(ctypes.c_double), P(ctypes.c_double)]
        lib.srjo_solve.restype = ctypes.c_int32
        lib.srjo_solve.argtypes = [P(_Problem), P(ctypes.c_double), P(_Opts), P(_Result),
                                   P(ctypes.c_int32), P(ctypes.c_double)]
        lib.srjo_round_f16.restype = ctypes.c_float
        lib.srjo_round_f16.argtypes = [ctypes.c_float]
        lib.srjo_round_bf16.restype = ctypes.c_float
        lib.srjo_round_bf16.argtypes = [ctypes.c_float]
        lib.srjo_num_threads.restype = ctypes.c_int32
        lib.srjo_set_num_threads.argtypes = [ctypes.c_int32]
        lib.srjo_set_num_threads.restype = None
        lib.srjo_mg_hierarchy.restype = ctypes.c_int32
        lib.srjo_mg_hierarchy.argtypes = [P(_Problem), ctypes.c_int32, P(ctypes.c_int64)]
        lib.srjo_restrict_residual.argtypes = [P(_Problem), P(ctypes.c_double), P(ctypes.c_double)]
        lib.srjo_prolong_add.argtypes = [P(_Problem), P(ctypes.c_double), P(ctypes.c_double)]
        lib.srjo_mg_solve.restype = ctypes.c_int32
        lib.srjo_mg_solve.argtypes = [P(_Problem), P(ctypes.c_double), P(_MgOpts), P(_MgResult),
                                      P(ctypes.c_int32), P(ctypes.c_double)]
        lib.srjo_collect.argtypes = [P(_Problem), ctypes.c_int32, ctypes.c_int32,
                                     P(ctypes.c_double), ctypes.c_double, ctypes.c_int32,
                                     ctypes.c_void_p, P(ctypes.c_int32)]
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _cproblem(prob) -> tuple:
    """Build the C struct; returns (struct, keepalive list)."""
    keep = []
    cp = _Problem()
    cp.ndim = prob.ndim
    for d in range(3):
        cp.n[d] = int(prob.n[d])
        cp.c[d] = float(prob.c[d])
        f = prob.faces[d] if prob.faces is not None else None
        if f is not None:
            f = np.ascontiguousarray(f, dtype=np.float64)
            keep.append(f)
            cp.face[d] = f.ctypes.data
        else:
            cp.face[d] = None
    cp.dconst = float(prob.dconst)
    if prob.diag is not None:
        dg = np.ascontiguousarray(prob.diag, dtype=np.float64)
        keep.append(dg)
        cp.diag = dg.ctypes.data
    else:
        cp.diag = None
    b = np.ascontiguousarray(prob.b, dtype=np.float64)
    keep.append(b)
    cp.b = b.ctypes.data
    cp.rowptr = cp.col = cp.val = None
    if getattr(prob, "csr", None) is not None:
        rp, col, val = prob.csr
        rp = np.ascontiguousarray(rp, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        keep += [rp, col, val]
        cp.rowptr, cp.col, cp.val = rp.ctypes.data, col.ctypes.data, val.ctypes.data
    return cp, keep


def level_M(level: int) -> int:
    return int(load().srjo_level_M(level))


def omega_natural(M: int) -> np.ndarray:
    w = np.zeros(M, dtype=np.float64)
    load().srjo_omega_natural(M, _dptr(w))
    return w


def leja_order(M: int, w: Optional[np.ndarray] = None) -> np.ndarray:
    if w is None:
        w = omega_natural(M)
    w = np.ascontiguousarray(w, dtype=np.float64)
    order = np.zeros(M, dtype=np.int32)
    load().srjo_leja_order(M, _dptr(w), order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return order


def scheme(level: int) -> np.ndarray:
    """Relaxation factors of a scheme level in execution order."""
    w = np.zeros(2362, dtype=np.float64)
    M = load().srjo_scheme(level, _dptr(w))
    if M < 0:
        raise ValueError(f"level {level} outside 0..24")
    return w[:M].copy()


def sweep(prob, x: np.ndarray, w: float) -> np.ndarray:
    cp, keep = _cproblem(prob)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(prob.shape)
    out = np.empty_like(x)
    load().srjo_sweep(ctypes.byref(cp), _dptr(x), float(w), _dptr(out))
    return out


def residual_norm(prob, x: np.ndarray) -> float:
    cp, keep = _cproblem(prob)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(prob.shape)
    return float(load().srjo_residual_norm(ctypes.byref(cp), _dptr(x)))


def apply(prob, x: np.ndarray) -> np.ndarray:
    cp, keep = _cproblem(prob)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(prob.shape)
    y = np.empty_like(x)
    load().srjo_apply(ctypes.byref(cp), _dptr(x), _dptr(y))
    return y


def solve(prob, x0: Optional[np.ndarray] = None, *, rule: str = "heuristic",
          fixed_level: int = 0, tol: float = 1e-10, tol_mode: str = "relative",
          max_cycles: int = 10000, max_sweeps: int = 50_000_000, stop_per_sweep: bool = False,
          precision: str = "f64", start_level: int = 0, max_level: int = 24,
          scale_target: float = 0.0) -> Dict:
    """Run the solver; returns x, per-cycle levels and norms and the counters."""
    cp, keep = _cproblem(prob)
    x = (np.zeros(prob.shape) if x0 is None else np.array(x0, dtype=np.float64)
         .reshape(prob.shape)).copy()
    o = _Opts(RULES[rule], fixed_level, TOL_MODES[tol_mode], tol, max_cycles, max_sweeps,
              1 if stop_per_sweep else 0, PRECISIONS[precision], start_level, max_level,
              scale_target)
    r = _Result()
    levels = np.full(max_cycles, -2, dtype=np.int32)
    norms = np.full(max_cycles + 1, np.nan, dtype=np.float64)
    st = load().srjo_solve(ctypes.byref(cp), _dptr(x), ctypes.byref(o), ctypes.byref(r),
                           levels.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(norms))
    return {
        "status": STATUS.get(int(st), str(st)), "x": x, "converged": bool(r.converged),
        "cycles": int(r.cycles), "sweeps": int(r.sweeps), "final_level": int(r.final_level),
        "r0": float(r.r0), "r_final": float(r.r_final), "min_margin": float(r.min_margin),
        "levels": levels[:r.cycles].copy(), "norms": norms[:r.cycles + 1].copy(),
    }


class _MgOpts(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("start_level", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("pre", ctypes.c_int32), ("post", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("coarse_tol", ctypes.c_double),
                ("coarse_max_cycles", ctypes.c_int32), ("tol_mode", ctypes.c_int32),
                ("tol", ctypes.c_double), ("max_vcycles", ctypes.c_int32)]


class _MgResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("vcycles", ctypes.c_int32), ("final_level", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("sweeps", ctypes.c_int64),
                ("coarse_sweeps", ctypes.c_int64), ("work", ctypes.c_double),
                ("r0", ctypes.c_double), ("r_final", ctypes.c_double)]


def mg_hierarchy(prob, max_levels: int = 32) -> list:
    """Grid sizes of the multigrid levels (finest first)."""
    cp, keep = _cproblem(prob)
    dims = np.zeros(3 * 32, dtype=np.int64)
    L = load().srjo_mg_hierarchy(ctypes.byref(cp), min(max_levels, 32),
                                 dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return [tuple(int(v) for v in dims[3 * l:3 * l + 3]) for l in range(L)]


def coarse_shape(prob) -> tuple:
    """NumPy shape (n2, n1, n0) of the next coarser grid."""
    m = [(int(prob.n[d]) - 1) // 2 if d < prob.ndim else 1 for d in range(3)]
    return (m[2], m[1], m[0])


def restrict_residual(prob, x: np.ndarray) -> np.ndarray:
    """R (b - A x) on the next coarser grid (full weighting)."""
    cp, keep = _cproblem(prob)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(prob.shape)
    out = np.zeros(coarse_shape(prob))
    load().srjo_restrict_residual(ctypes.byref(cp), _dptr(x), _dptr(out))
    return out


def prolong_add(prob, ec: np.ndarray, x: np.ndarray) -> np.ndarray:
    """x + P ec (multilinear interpolation from the next coarser grid)."""
    cp, keep = _cproblem(prob)
    ec = np.ascontiguousarray(ec, dtype=np.float64).reshape(coarse_shape(prob))
    out = np.array(x, dtype=np.float64).reshape(prob.shape).copy()
    load().srjo_prolong_add(ctypes.byref(cp), _dptr(ec), _dptr(out))
    return out


def mg_solve(prob, x0: Optional[np.ndarray] = None, *, rule: str = "heuristic",
             start_level: int = 0, max_level: int = 24, pre: int = 1, post: int = 1,
             max_levels: int = 32, coarse_tol: float = 1e-8, coarse_max_cycles: int = 1000,
             tol: float = 1e-10, tol_mode: str = "relative", max_vcycles: int = 200) -> Dict:
    """V-cycles with SRJ smoothing to tolerance; per-V-cycle levels and norms."""
    cp, keep = _cproblem(prob)
    x = (np.zeros(prob.shape) if x0 is None else np.array(x0, dtype=np.float64)
         .reshape(prob.shape)).copy()
    o = _MgOpts(RULES[rule], start_level, max_level, pre, post, max_levels, coarse_tol,
                coarse_max_cycles, TOL_MODES[tol_mode], tol, max_vcycles)
    r = _MgResult()
    levels = np.full(max_vcycles, -2, dtype=np.int32)
    norms = np.full(max_vcycles + 1, np.nan, dtype=np.float64)
    st = load().srjo_mg_solve(ctypes.byref(cp), _dptr(x), ctypes.byref(o), ctypes.byref(r),
                              levels.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(norms))
    return {"status": STATUS.get(int(st), str(st)), "x": x, "converged": bool(r.converged),
            "vcycles": int(r.vcycles), "final_level": int(r.final_level), "levels_grid": int(r.levels),
            "sweeps": int(r.sweeps), "coarse_sweeps": int(r.coarse_sweeps), "work": float(r.work),
            "r0": float(r.r0), "r_final": float(r.r_final),
            "levels": levels[:r.vcycles].copy(), "norms": norms[:r.vcycles + 1].copy()}


def round_f16(v: np.ndarray) -> np.ndarray:
    f = load().srjo_round_f16
    return np.array([f(float(a)) for a in np.asarray(v, dtype=np.float32).ravel()],
                    dtype=np.float32).reshape(np.shape(v))


def round_bf16(v: np.ndarray) -> np.ndarray:
    f = load().srjo_round_bf16
    return np.array([f(float(a)) for a in np.asarray(v, dtype=np.float32).ravel()],
                    dtype=np.float32).reshape(np.shape(v))


def num_threads() -> int:
    return int(load().srjo_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of later oracle calls (timing only; results do not depend on it)."""
    load().srjo_set_num_threads(int(n))


# Record layout of srjo_sample (section 3 tuples, one per branch).
SAMPLE_DTYPE = np.dtype([("trial", "<i4"), ("step", "<i4"), ("level", "<i4"),
                         ("action", "<i4"), ("M", "<i4"), ("chosen", "<i4"),
                         ("prev_ratio", "<f8"), ("r_before", "<f8"), ("r_after", "<f8")])


def collect(prob, u: np.ndarray, tol: float = 1e-8, max_level: int = 24) -> dict:
    """Section 3 data collection: one trial per row of u (draws in [0, 1)).

    Returns samples (SAMPLE_DTYPE, shape (trials, max_steps, 3); slots of
    steps a trial did not take are zero) and steps (int32 per trial)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    trials, max_steps = u.shape
    cp, keep = _cproblem(prob)
    out = np.zeros((trials, max_steps, 3), dtype=SAMPLE_DTYPE)
    steps = np.zeros(trials, dtype=np.int32)
    load().srjo_collect(ctypes.byref(cp), trials, max_steps, _dptr(u), float(tol), int(max_level),
                        out.ctypes.data, steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return {"samples": out, "steps": steps}
