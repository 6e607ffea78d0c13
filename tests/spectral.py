"""Independent models used to pin the CPU oracle (test code only).

None of this imports the oracle or the GPU library.  It rests on textbook
facts, not on the oracle's code path:

* dense matrices built entry by entry from the definition A = D + L + U
  (section 2, Eq. 1) and solved with ``numpy.linalg``;
* the eigen-decomposition of constant-coefficient Dirichlet stencils: the
  orthonormal DST-I (``scipy.fft.dstn``) diagonalises them, and D^-1 A has
  eigenvalues mu_k = sum_d (c_d / D) * 2 (1 - cos(k_d pi / (n_d + 1)));
* the closed form of the amplification polynomial from Appendix A,
  G_M(l) = T_M(f(l)) / 3 with f(l) = ((l* + 1) l + l* - 1) / 2 and
  T_M(l*) = 3 (Eq. (13)), evaluated with the Chebyshev identities
  T_M(cos t) = cos(M t) and T_M(cosh t) = cosh(M t).

Because every cycle multiplies the residual's mode k by G_M(1 - mu_k) (Eq.
(12) applied to r = -A e), the cycle-end residual norms of a solve follow
from the right-hand side's DST coefficients alone, without running any sweep
and independently of the order of the factors inside a cycle.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np
import scipy.fft

from golden_io import rows


def appendix_b_M() -> List[int]:
    return [int(r[1]) for r in rows("appendixB_levels.txt")]


# --------------------------------------------------------------------------
# Dense matrices from the definition
# --------------------------------------------------------------------------

def dense_matrix(prob) -> np.ndarray:
    """A as a dense matrix, entry by entry (tiny grids only)."""
    n0, n1, n2 = prob.n
    N = n0 * n1 * n2
    A = np.zeros((N, N))
    strides = (1, n0, n0 * n1)
    for i2 in range(n2):
        for i1 in range(n1):
            for i0 in range(n0):
                ii = (i0, i1, i2)
                p = i0 + n0 * (i1 + n1 * i2)
                A[p, p] = prob.diag.reshape(-1)[p] if prob.diag is not None else prob.dconst
                for d in range(prob.ndim):
                    if ii[d] < prob.n[d] - 1:
                        q = p + strides[d]
                        if prob.faces is not None and prob.faces[d] is not None:
                            c = prob.faces[d].reshape(-1)[p]
                        else:
                            c = prob.c[d]
                        A[p, q] = -c
                        A[q, p] = -c
    return A


# --------------------------------------------------------------------------
# Chebyshev closed forms (Appendix A)
# --------------------------------------------------------------------------

def chebyshev_T(M: int, x: np.ndarray) -> np.ndarray:
    """T_M(x) from T_M(cos t) = cos(M t), T_M(+-cosh t) = (+-1)^M cosh(M t)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(M * np.arccos(x[inside]))
    hi = x > 1.0
    out[hi] = np.cosh(M * np.arccosh(x[hi]))
    lo = x < -1.0
    out[lo] = (-1.0) ** M * np.cosh(M * np.arccosh(-x[lo]))
    return out


def lstar(M: int) -> float:
    """The real root > 1 of T_M(l) = 3."""
    return math.cosh(math.acosh(3.0) / M)


def G_closed(M: int, lam: np.ndarray) -> np.ndarray:
    """G_M(l) = T_M(f(l)) / 3 (Eq. (13))."""
    ls = lstar(M)
    f = ((ls + 1.0) * np.asarray(lam, dtype=np.float64) + (ls - 1.0)) / 2.0
    return chebyshev_T(M, f) / 3.0


# --------------------------------------------------------------------------
# Spectral model of constant-coefficient Dirichlet problems
# --------------------------------------------------------------------------

def mu_grid(prob) -> np.ndarray:
    """Eigenvalues of D^-1 A on the grid of mode numbers, shape (n2, n1, n0)."""
    assert prob.faces is None and prob.diag is None
    out = np.zeros(prob.shape)
    for d in range(prob.ndim):
        n = prob.n[d]
        k = np.arange(1, n + 1, dtype=np.float64)
        v = (prob.c[d] / prob.dconst) * 2.0 * (1.0 - np.cos(k * np.pi / (n + 1)))
        shp = [1, 1, 1]
        shp[2 - d] = n
        out = out + v.reshape(shp)
    return out


def dst(v: np.ndarray, ndim: int) -> np.ndarray:
    axes = [2 - d for d in range(ndim)]
    return scipy.fft.dstn(v, type=1, norm="ortho", axes=axes)


def heuristic_next(level: int, ratio: float, max_level: int = 24) -> int:
    if ratio > 0.4:
        level += 1
    elif 0.2 < ratio < 0.4:
        level -= 1
    return min(max(level, 0), max_level)


def spectral_solve(prob, *, rule: str = "heuristic", fixed_level: int = 0, tol: float = 1e-10,
                   tol_mode: str = "relative", max_cycles: int = 1000) -> Dict:
    """Cycle-end residual norms and levels of an SRJ solve from x0 = 0."""
    Ms = appendix_b_M()
    lamJ = 1.0 - mu_grid(prob)
    rhat = dst(prob.b, prob.ndim)
    r0 = float(np.sqrt(np.sum(rhat * rhat)))
    target = tol * r0 if tol_mode == "relative" else tol
    level = 0
    prev = r0
    levels, norms = [], [r0]
    sweeps = 0
    converged = False
    for _ in range(max_cycles):
        lv = fixed_level if rule == "fixed" else level
        M = Ms[lv]
        rhat = rhat * G_closed(M, lamJ)
        sweeps += M
        nrm = float(np.sqrt(np.sum(rhat * rhat)))
        levels.append(lv)
        norms.append(nrm)
        if nrm < target:
            converged = True
            break
        ratio = nrm / prev
        prev = nrm
        if rule == "heuristic":
            level = heuristic_next(level, ratio)
        elif rule == "increasing":
            level = min(level + 1, 24)
    return {"levels": np.array(levels), "norms": np.array(norms), "sweeps": sweeps,
            "cycles": len(levels), "converged": converged, "r0": r0}


def jacobi_sweeps_to_tol(prob, tol: float, max_sweeps: int = 10_000_000) -> int:
    """First n with ||B_J^n r0|| < tol ||r0|| for unweighted Jacobi (Eq. 2).

    Mode k of the residual is multiplied by l_k = 1 - mu_k every sweep, so the
    norm after n sweeps is sqrt(sum_k rhat_k^2 l_k^(2n)); it decreases
    monotonically in n, so a bisection finds the first crossing.
    """
    lam = (1.0 - mu_grid(prob)).ravel()
    r2 = dst(prob.b, prob.ndim).ravel() ** 2
    keep = r2 > 0
    lam, r2 = np.abs(lam[keep]), r2[keep]
    r0sq = r2.sum()

    def ratio2(n):
        return float(np.sum(r2 * lam ** (2 * n)) / r0sq)

    lo, hi = 0, 1
    while ratio2(hi) >= tol * tol:
        lo, hi = hi, hi * 2
        assert hi < max_sweeps
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if ratio2(mid) >= tol * tol:
            lo = mid
        else:
            hi = mid
    return hi
