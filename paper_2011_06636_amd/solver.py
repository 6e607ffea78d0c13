"""PyTorch-facing wrapper of the C ABI: device memory and streams only.

torch supplies device buffers (``data_ptr()``) and the current HIP stream;
every arithmetic step runs in libsrj.so.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import abi


def _dev(a, device) -> torch.Tensor:
    t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64))
    return t.to(device=device, non_blocking=False).contiguous()


class _Ordered:
    """Orders the library's stream after the caller's current stream on entry
    (the tensors it reads were produced there) and the caller's stream after
    the library's on exit."""

    def __init__(self, device, stream):
        self.device, self.stream = device, stream

    def __enter__(self):
        self.cur = torch.cuda.current_stream(self.device)
        if self.cur != self.stream:
            self.stream.wait_stream(self.cur)

    def __exit__(self, *exc):
        if self.cur != self.stream:
            self.cur.wait_stream(self.stream)
        return False


def check_iterate(x, device, npoints: int, what: str = "x") -> None:
    """x must be a contiguous float64 tensor of npoints values on `device`:
    the library reads and writes it in place through its address."""
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    dev = torch.device(device)
    if x.device.type != dev.type:
        raise ValueError(f"{what} is on {x.device}, the solver on {dev}")
    if dev.type == "cuda":
        want = dev.index if dev.index is not None else torch.cuda.current_device()
        if x.device.index != want:
            raise ValueError(f"{what} is on {x.device}, the solver on cuda:{want}")
    if x.dtype != torch.float64:
        raise ValueError(f"{what} must be float64, not {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if x.numel() != npoints:
        raise ValueError(f"{what} holds {x.numel()} values, the problem {npoints}")


def make_problem(ndim: int, n: Sequence[int], c: Sequence[float], dconst: float,
                 b: torch.Tensor, faces: Optional[Sequence[Optional[torch.Tensor]]] = None,
                 diag: Optional[torch.Tensor] = None) -> abi.SrjProblem:
    """srj_problem from device tensors (the tensors must outlive the context)."""
    p = abi.SrjProblem()
    p.ndim = ndim
    for d in range(3):
        p.n[d] = int(n[d])
        p.cconst[d] = float(c[d])
        f = faces[d] if faces is not None else None
        p.face[d] = f.data_ptr() if f is not None else None
    p.dconst = float(dconst)
    p.diag = diag.data_ptr() if diag is not None else None
    p.b = b.data_ptr()
    return p


class Solver:
    """One problem on one GPU: wraps srj_setup / srj_solve / srj_run_cycle.

    ``problem`` has the attributes ndim, n, c, dconst, b and optionally faces
    and diag as host NumPy arrays of shape (n2, n1, n0) (axis 0 contiguous).
    """

    def __init__(self, problem, device: str = "cuda", stream: Optional[torch.cuda.Stream] = None):
        abi.load()
        self.device = torch.device(device)
        self.shape = tuple(problem.b.shape)
        self.npoints = int(np.prod(self.shape))
        self.ndim = int(problem.ndim)
        self.b = _dev(problem.b, self.device)
        faces = getattr(problem, "faces", None)
        self.faces = [(_dev(f, self.device) if f is not None else None) for f in faces] \
            if faces is not None else None
        diag = getattr(problem, "diag", None)
        self.diag = _dev(diag, self.device) if diag is not None else None
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        csr = getattr(problem, "csr", None)
        if csr is not None:  # general sparse matrix: the library copies it at setup
            rp = torch.as_tensor(np.ascontiguousarray(csr[0], dtype=np.int64)).to(self.device)
            col = torch.as_tensor(np.ascontiguousarray(csr[1], dtype=np.int32)).to(self.device)
            val = torch.as_tensor(np.ascontiguousarray(csr[2], dtype=np.float64)).to(self.device)
            self._prob = abi.SrjCsrProblem(self.npoints, rp.data_ptr(), col.data_ptr(),
                                           val.data_ptr(), self.b.data_ptr())
            torch.cuda.synchronize(self.device)
            self.ctx = abi.srj_setup_csr(self._prob, self.stream.cuda_stream)
            return
        self._prob = make_problem(self.ndim, problem.n, problem.c, problem.dconst, self.b,
                                  self.faces, self.diag)
        torch.cuda.synchronize(self.device)
        self.ctx = abi.srj_setup(self._prob, self.stream.cuda_stream)

    def close(self) -> None:
        if getattr(self, "ctx", None):
            abi.srj_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def zeros(self) -> torch.Tensor:
        return torch.zeros(self.shape, dtype=torch.float64, device=self.device)

    def to_device(self, a) -> torch.Tensor:
        return _dev(np.asarray(a).reshape(self.shape), self.device)

    def set_plan(self, kind: int, tile_rows: int = 0, sweeps: int = 1, occ: int = 1,
                 which: int = 0) -> int:
        """which = 0: binary64 sweeps; which = 1: inner sweeps of the refinement modes."""
        return abi.srj_set_plan(self.ctx, kind, tile_rows, sweeps, occ, which)

    def get_plan(self, which: int = 0):
        return abi.srj_get_plan(self.ctx, which)

    def set_resident(self, enable: bool) -> int:
        """Whole binary64 solve of a small grid in one workgroup (default when it fits)."""
        return abi.srj_set_resident(self.ctx, enable)

    def autotune(self, which: int = 0, sweeps: int = 48, use_cache: bool = True) -> float:
        """Pick the fastest plan for `which` by timing; returns its us per sweep."""
        return abi.srj_autotune(self.ctx, which, sweeps, use_cache)

    def set_profiling(self, enable: bool = True) -> None:
        abi.srj_set_profiling(self.ctx, enable)

    def profile(self):
        """(sweep-launch milliseconds, launches, sweeps) since profiling was enabled."""
        return abi.srj_get_profile(self.ctx)

    def residual_norm(self, x: torch.Tensor) -> float:
        check_iterate(x, self.device, self.npoints)
        with _Ordered(self.device, self.stream):
            return abi.srj_residual_norm(self.ctx, x.data_ptr())

    def run_cycle(self, x: torch.Tensor, level: int) -> float:
        check_iterate(x, self.device, self.npoints)
        with _Ordered(self.device, self.stream):
            return abi.srj_run_cycle(self.ctx, x.data_ptr(), level)

    @staticmethod
    def opts(rule: str = "heuristic", fixed_level: int = 0, tol: float = 1e-10,
             tol_mode: str = "relative", max_cycles: int = 10000, max_sweeps: int = 50_000_000,
             precision: str = "f64", start_level: int = 0, max_level: int = 24,
             scale_target: float = 0.0, r0: float = 0.0) -> abi.SrjSolveOpts:
        o = abi.srj_default_opts()
        o.rule = abi.RULE[rule]
        o.fixed_level = fixed_level
        o.tol = tol
        o.tol_mode = abi.TOL_MODE[tol_mode]
        o.max_cycles = max_cycles
        o.max_sweeps = max_sweeps
        o.precision = abi.PREC[precision]
        o.start_level = start_level
        o.max_level = max_level
        o.scale_target = scale_target
        o.r0 = r0
        return o

    def solve(self, x: Optional[torch.Tensor] = None, **kw) -> Dict:
        """Solve in place on x (zeros if None); returns counters, levels and norms."""
        if x is None:
            x = self.zeros()
        o = self.opts(**kw)
        levels = (ctypes.c_int32 * o.max_cycles)()
        norms = (ctypes.c_double * (o.max_cycles + 1))()
        check_iterate(x, self.device, self.npoints)
        with _Ordered(self.device, self.stream):
            st, res = abi.srj_solve(self.ctx, x.data_ptr(), o, levels, norms)
        if st not in (abi.SRJ_OK, abi.SRJ_ERR_NOT_CONVERGED, abi.SRJ_ERR_NONFINITE):
            raise abi.SrjError(st, "srj_solve")
        nc = res.cycles
        return {
            "status": abi.STATUS_NAMES[st], "x": x, "converged": bool(res.converged),
            "cycles": nc, "sweeps": int(res.sweeps), "final_level": res.final_level,
            "r0": res.r0, "r_final": res.r_final, "min_margin": res.min_margin,
            "levels": np.array(levels[:nc], dtype=np.int32),
            "norms": np.array(norms[:nc + 1], dtype=np.float64),
        }

    def set_scheme_family(self, levels=None) -> None:
        """Replace the scheme family (list of per-level factor lists, applied
        in the given order); None restores the paper's family."""
        torch.cuda.synchronize(self.device)
        abi.srj_set_scheme_family(self.ctx, levels)

    def collect(self, u: torch.Tensor, tol: float = 1e-8, max_level: int = 24,
                compact: bool = False) -> Dict:
        """Selector training data (srj_collect): one trial per row of u.

        u: float64 tensor (trials, max_steps) of draws in [0, 1) on this device.
        Returns samples (SAMPLE_DTYPE, shape (trials, max_steps, 3); slots of
        steps a trial did not take are zeroed) and steps (int32, trials).
        With compact, samples is the flat array of the steps taken only
        (trial, step, slot order), gathered on the device before the copy."""
        trials, max_steps = u.shape
        u = u.to(device=self.device, dtype=torch.float64).contiguous()
        nbytes = np.dtype(abi.SAMPLE_DTYPE).itemsize
        raw = torch.zeros(trials * max_steps * 3 * nbytes, dtype=torch.uint8, device=self.device)
        steps = torch.zeros(trials, dtype=torch.int32, device=self.device)
        torch.cuda.synchronize(self.device)
        abi.srj_collect(self.ctx, trials, max_steps, u.data_ptr(), tol, max_level,
                        raw.data_ptr(), steps.data_ptr())
        if compact:
            rows = raw.view(trials, max_steps, 3 * nbytes)
            taken = torch.arange(max_steps, device=self.device)[None, :] < steps[:, None]
            flat = rows[taken].cpu().numpy().reshape(-1).view(abi.SAMPLE_DTYPE)
            return {"samples": flat, "steps": steps.cpu().numpy()}
        samples = raw.cpu().numpy().view(abi.SAMPLE_DTYPE).reshape(trials, max_steps, 3)
        return {"samples": samples, "steps": steps.cpu().numpy()}


class MgSolver:
    """SRJ-smoothed multigrid V-cycles on one problem: wraps srj_mg_setup /
    srj_mg_solve (constant-coefficient stencils with odd active sizes)."""

    def __init__(self, problem, device: str = "cuda", stream: Optional[torch.cuda.Stream] = None):
        abi.load()
        self.device = torch.device(device)
        self.shape = tuple(problem.b.shape)
        self.npoints = int(np.prod(self.shape))
        self.b = _dev(problem.b, self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # per-face couplings or a diagonal array are passed on (the library
        # refuses them for multigrid)
        faces = getattr(problem, "faces", None)
        self.faces = [(_dev(f, self.device) if f is not None else None) for f in faces] \
            if faces is not None else None
        diag = getattr(problem, "diag", None)
        self.diag = _dev(diag, self.device) if diag is not None else None
        self._prob = make_problem(int(problem.ndim), problem.n, problem.c, problem.dconst, self.b,
                                  self.faces, self.diag)
        torch.cuda.synchronize(self.device)
        self.handle = abi.srj_mg_setup(self._prob, self.stream.cuda_stream)

    def close(self) -> None:
        if getattr(self, "handle", None):
            abi.srj_mg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def zeros(self) -> torch.Tensor:
        return torch.zeros(self.shape, dtype=torch.float64, device=self.device)

    def to_device(self, a) -> torch.Tensor:
        return _dev(np.asarray(a).reshape(self.shape), self.device)

    @staticmethod
    def opts(rule: str = "heuristic", start_level: int = 0, max_level: int = 24, pre: int = 1,
             post: int = 1, max_levels: int = 32, coarse_tol: float = 1e-8,
             coarse_max_cycles: int = 1000, tol: float = 1e-10, tol_mode: str = "relative",
             max_vcycles: int = 200) -> abi.SrjMgOpts:
        o = abi.srj_mg_default_opts()
        o.rule = abi.RULE[rule]
        o.start_level, o.max_level, o.pre, o.post = start_level, max_level, pre, post
        o.max_levels, o.coarse_tol, o.coarse_max_cycles = max_levels, coarse_tol, coarse_max_cycles
        o.tol, o.tol_mode, o.max_vcycles = tol, abi.TOL_MODE[tol_mode], max_vcycles
        return o

    def solve(self, x: Optional[torch.Tensor] = None, **kw) -> Dict:
        """V-cycles in place on x (zeros if None); returns counters, levels and norms."""
        if x is None:
            x = self.zeros()
        o = self.opts(**kw)
        levels = (ctypes.c_int32 * o.max_vcycles)()
        norms = (ctypes.c_double * (o.max_vcycles + 1))()
        check_iterate(x, self.device, self.npoints)
        with _Ordered(self.device, self.stream):
            st, res = abi.srj_mg_solve(self.handle, x.data_ptr(), o, levels, norms)
        if st not in (abi.SRJ_OK, abi.SRJ_ERR_NOT_CONVERGED, abi.SRJ_ERR_NONFINITE):
            raise abi.SrjError(st, "srj_mg_solve")
        nv = res.vcycles
        return {"status": abi.STATUS_NAMES[st], "x": x, "converged": bool(res.converged),
                "vcycles": nv, "final_level": res.final_level, "levels_grid": res.levels,
                "sweeps": int(res.sweeps), "coarse_sweeps": int(res.coarse_sweeps),
                "work": res.work, "r0": res.r0, "r_final": res.r_final,
                "levels": np.array(levels[:nv], dtype=np.int32),
                "norms": np.array(norms[:nv + 1], dtype=np.float64)}


class BatchSolver:
    """Many problems solved together: wraps srj_batch_setup / srj_batch_solve.

    ``problems`` is a sequence of objects with the attributes of ``Solver``'s
    problem (constant couplings and diagonal only).
    """

    def __init__(self, problems, device: str = "cuda",
                 stream: Optional[torch.cuda.Stream] = None):
        abi.load()
        self.device = torch.device(device)
        self.shapes = [tuple(p.b.shape) for p in problems]
        self.count = len(problems)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        bs = [_dev(p.b, self.device) for p in problems]
        probs = [make_problem(int(p.ndim), p.n, p.c, p.dconst, b) for p, b in zip(problems, bs)]
        torch.cuda.synchronize(self.device)
        st, h = abi.srj_batch_setup(probs, self.stream.cuda_stream)
        if st != abi.SRJ_OK:
            raise abi.SrjError(st, "srj_batch_setup")
        self.handle = h
        del bs  # packed into the batch at setup

    def close(self) -> None:
        if getattr(self, "handle", None):
            abi.srj_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_plan(self, tile_rows: int, sweeps: int, steps_per_graph: int = 16,
                 use_graph: bool = True, waves_per_block: int = 1) -> int:
        """waves_per_block 1: single-wave tiles; > 1: cooperative blocks."""
        return abi.srj_batch_set_plan(self.handle, tile_rows, sweeps, waves_per_block,
                                      steps_per_graph, use_graph)

    def autotune(self, precision: str = "f32", sweeps: int = 48) -> float:
        """Pick the fastest batch plan by timing; returns its us per sweep."""
        return abi.srj_batch_autotune(self.handle, precision, sweeps)

    def get_plan(self):
        """(tile_rows, sweeps per step, waves per block, steps per graph, use_graph)."""
        return abi.srj_batch_get_plan(self.handle)

    def set_plan3d(self, tile_rows: int, planes: int, sweeps: int = 2) -> None:
        """Plane tile of the 3D instances: rows per tile, planes per work item,
        most sweeps per step (1 or 2)."""
        abi.srj_batch_set_plan3d(self.handle, tile_rows, planes, sweeps)

    def get_plan3d(self):
        return abi.srj_batch_get_plan3d(self.handle)

    def zeros(self):
        return [torch.zeros(sh, dtype=torch.float64, device=self.device) for sh in self.shapes]

    def solve(self, xs=None, **kw) -> Dict:
        """Solve every instance in place on xs (zeros if None)."""
        if xs is None:
            xs = self.zeros()
        o = Solver.opts(**kw)
        levels = (ctypes.c_int32 * (self.count * o.max_cycles))()
        if len(xs) != self.count:
            raise ValueError(f"{len(xs)} iterates for {self.count} instances")
        for k, (x, sh) in enumerate(zip(xs, self.shapes)):
            check_iterate(x, self.device, int(np.prod(sh)), f"xs[{k}]")
        with _Ordered(self.device, self.stream):
            st, res = abi.srj_batch_solve(self.handle, [x.data_ptr() for x in xs], o, levels)
        if st not in (abi.SRJ_OK, abi.SRJ_ERR_NOT_CONVERGED, abi.SRJ_ERR_NONFINITE):
            raise abi.SrjError(st, "srj_batch_solve")
        lv = np.array(levels, dtype=np.int32).reshape(self.count, o.max_cycles)
        out = []
        for i in range(self.count):
            r = res[i]
            out.append({"converged": bool(r.converged), "cycles": r.cycles,
                        "sweeps": int(r.sweeps), "final_level": r.final_level, "r0": r.r0,
                        "r_final": r.r_final, "min_margin": r.min_margin,
                        "levels": lv[i, :r.cycles].copy()})
        return {"status": abi.STATUS_NAMES[st], "xs": xs, "instances": out}
