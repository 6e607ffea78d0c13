"""Seeded synthetic inputs for the SRJ solver and for its CPU reference.

This module builds problems only: grid sizes, stencil couplings, diagonals and
right-hand sides, drawn from ``numpy.random.default_rng(seed)`` in a fixed
order.  It contains none of the solver's arithmetic (no relaxation factors, no
sweeps, no residuals, no scheme selection), so both the GPU library's tests and
the CPU reference can take their inputs from here without sharing any of the
method's code.

Array convention (used by every consumer): a problem on an ``n0 x n1 x n2``
interior grid stores each field as a float64 NumPy array of C-order shape
``(n2, n1, n0)``, i.e. axis 0 is the contiguous one and the flat index of
point ``(i0, i1, i2)`` is ``i0 + n0 * (i1 + n1 * i2)``.  Unused axes have
size 1.  Boundary conditions are homogeneous Dirichlet: the ghost layer around
the grid is zero and is not stored.

The matrix is ``A = D + L + U`` (section 2, Eq. 1) with

* ``A[p, p] = D_p`` (``dconst`` or ``diag[p]``);
* ``A[p, p + e_d] = A[p + e_d, p] = -coupling_d(p)``, where
  ``coupling_d(p) = c[d]`` for a constant stencil or ``face[d][p]`` (the
  coupling between point ``p`` and ``p + e_d``) for a variable one.

Recipes (the paper's own problems, section 3 and section 4, plus the
benchmark workloads built in their image):

* ``poisson``: finite-difference Poisson on the unit interval / square / cube
  with ``h_d = 1/(n_d + 1)``, coupling ``1/h_d^2`` and diagonal
  ``sum_d 2/h_d^2`` (the 1D matrix of section 3, the 3D problem of
  section 4.2.3).
* ``c1``: 1D, N = 255, b ~ U(-1, 1) (seed 0).
* ``c2``: 2D 2048 x 2048, b = sum of 8 random-amplitude low sine modes plus
  U(-1e-3, 1e-3) noise (seed 0).
* ``c3``: 3D 256^3 variable coefficient -div(k grad u) = 1, with k
  log-normal (sigma = 1, Gaussian correlation length 8 cells), harmonic-mean
  faces and ``D_p`` equal to the sum of the six face couplings (seed 0).
* ``c4``: 512 2D Poisson squares with log-uniform sides in [64, 1024] and
  b ~ U(-1, 1) (instance i uses seed 1000 + i).
* ``c5``: 128 3D anisotropic boxes, sides uniform in [32, 128], couplings
  (1, a, b) with a, b log-uniform in [0.01, 1], unit spacing, b ~ U(-1, 1)
  (instance i uses seed 2000 + i).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Problem", "poisson", "poisson_1d", "sine_mode", "c1", "c2", "c3",
    "c4_instance", "c4", "c5_instance", "c5", "lognormal_field",
    "variable_coefficient", "anisotropic",
]


@dataclasses.dataclass
class Problem:
    """A symmetric stencil matrix A = D + L + U and a right-hand side b."""

    ndim: int
    n: Tuple[int, int, int]
    c: Tuple[float, float, float]
    dconst: float
    b: np.ndarray
    faces: Optional[List[Optional[np.ndarray]]] = None
    diag: Optional[np.ndarray] = None
    # general sparse matrix instead of a stencil: (rowptr int64, col int32,
    # val float64) in CSR form, ndim = 1, n = (rows, 1, 1)
    csr: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = None
    name: str = ""

    @property
    def npoints(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def shape(self) -> Tuple[int, int, int]:
        """NumPy shape of every field: (n2, n1, n0)."""
        return (int(self.n[2]), int(self.n[1]), int(self.n[0]))

    def zeros(self) -> np.ndarray:
        return np.zeros(self.shape, dtype=np.float64)

    def check(self) -> None:
        assert self.ndim in (1, 2, 3)
        for d in range(3):
            assert self.n[d] >= 1
            if d >= self.ndim:
                assert self.n[d] == 1
        assert self.b.shape == self.shape and self.b.dtype == np.float64
        if self.faces is not None:
            assert len(self.faces) == 3
            for f in self.faces:
                if f is not None:
                    assert f.shape == self.shape and f.dtype == np.float64
        if self.diag is not None:
            assert self.diag.shape == self.shape and self.diag.dtype == np.float64


def _dims(n: Sequence[int]) -> Tuple[int, Tuple[int, int, int]]:
    n = [int(v) for v in n]
    ndim = len(n)
    assert 1 <= ndim <= 3
    return ndim, tuple(n + [1] * (3 - ndim))  # type: ignore[return-value]


def poisson(n: Sequence[int], b: Optional[np.ndarray] = None, name: str = "") -> Problem:
    """Finite-difference Poisson -Laplace(u) = f on the unit box, Dirichlet zero.

    Spacing ``h_d = 1/(n_d + 1)`` on every axis; coupling ``1/h_d^2``; diagonal
    ``sum_d 2/h_d^2`` (the tridiagonal matrix (1/dx^2) tridiag(-1, 2, -1) of
    section 3 in 1D).  ``b`` defaults to all ones (f = 1).
    """
    ndim, n3 = _dims(n)
    c = [0.0, 0.0, 0.0]
    for d in range(ndim):
        c[d] = float((n3[d] + 1) ** 2)
    dconst = 2.0 * sum(c)
    shape = (n3[2], n3[1], n3[0])
    if b is None:
        b = np.ones(shape, dtype=np.float64)
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(shape))
    return Problem(ndim, n3, tuple(c), dconst, b, name=name or f"poisson{ndim}d")


def poisson_1d(N: int, b: Optional[np.ndarray] = None) -> Problem:
    return poisson([N], b=b, name=f"poisson1d_N{N}")


def anisotropic(n: Sequence[int], coup: Sequence[float], b: np.ndarray, name: str = "") -> Problem:
    """-(u_xx + a u_yy + b u_zz) = f on unit spacing: couplings ``coup``, D = 2 sum(coup)."""
    ndim, n3 = _dims(n)
    c = [0.0, 0.0, 0.0]
    for d in range(ndim):
        c[d] = float(coup[d])
    shape = (n3[2], n3[1], n3[0])
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(shape))
    return Problem(ndim, n3, tuple(c), 2.0 * sum(c), b, name=name or "anisotropic")


def sine_mode(n: Sequence[int], k: Sequence[int]) -> np.ndarray:
    """Discrete Dirichlet sine mode prod_d sin(k_d pi i_d / (n_d + 1)), i_d = 1..n_d."""
    ndim, n3 = _dims(n)
    k3 = list(k) + [1] * (3 - len(k))
    out = np.ones((n3[2], n3[1], n3[0]), dtype=np.float64)
    for d in range(ndim):
        i = np.arange(1, n3[d] + 1, dtype=np.float64)
        v = np.sin(k3[d] * np.pi * i / (n3[d] + 1))
        shp = [1, 1, 1]
        shp[2 - d] = n3[d]
        out = out * v.reshape(shp)
    return out


# --------------------------------------------------------------------------
# Benchmark workloads
# --------------------------------------------------------------------------

def c1(seed: int = 0, N: int = 255) -> Problem:
    """1D Poisson, N = 255, b ~ U(-1, 1).  h = 1/256 so 1/h^2 = 2^16 exactly."""
    rng = np.random.default_rng(seed)
    b = rng.uniform(-1.0, 1.0, size=(1, 1, N))
    return poisson([N], b=b, name=f"c1_poisson1d_N{N}")


def c2(seed: int = 0, n: int = 2048) -> Problem:
    """2D Poisson on an n x n grid; b = 8 low sine modes + U(-1e-3, 1e-3) noise.

    Draw order: 8 amplitudes a_m ~ U(-1, 1), then 8 wavenumbers k_m, then 8
    wavenumbers l_m (each uniform on {1..8}), then the noise field in storage
    order.  Mode m is a_m sin(k_m pi x) sin(l_m pi y) with x along axis 0.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=8)
    kx = rng.integers(1, 9, size=8)
    ly = rng.integers(1, 9, size=8)
    noise = rng.uniform(-1e-3, 1e-3, size=(n, n))
    h = 1.0 / (n + 1)
    xs = np.arange(1, n + 1, dtype=np.float64) * h
    b = np.zeros((n, n), dtype=np.float64)
    for m in range(8):
        b += a[m] * np.outer(np.sin(ly[m] * np.pi * xs), np.sin(kx[m] * np.pi * xs))
    b += noise
    return poisson([n, n], b=b.reshape(1, n, n), name=f"c2_poisson2d_{n}")


def lognormal_field(shape: Tuple[int, int, int], rng: np.random.Generator,
                    corr_len: float = 8.0, sigma: float = 1.0) -> np.ndarray:
    """k = exp(sigma g) with g a zero-mean, unit-variance Gaussian field.

    g is white noise filtered on the periodic box by exp(-l^2 |kappa|^2 / 4),
    the square root of the spectrum of the covariance exp(-d^2 / (2 l^2)).
    """
    noise = rng.standard_normal(size=shape)
    spec = np.fft.rfftn(noise)
    kz = 2.0 * np.pi * np.fft.fftfreq(shape[0])
    ky = 2.0 * np.pi * np.fft.fftfreq(shape[1])
    kx = 2.0 * np.pi * np.fft.rfftfreq(shape[2])
    k2 = (kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    spec *= np.exp(-(corr_len ** 2) * k2 / 4.0)
    del k2
    g = np.fft.irfftn(spec, s=shape, axes=(0, 1, 2))
    del spec
    g -= g.mean()
    g /= g.std()
    return np.exp(sigma * g)


def variable_coefficient(n: int, seed: int, corr_len: float = 8.0, sigma: float = 1.0,
                         name: str = "") -> Problem:
    """-div(k grad u) = 1 on the unit cube, n^3 interior nodes, Dirichlet zero.

    k lives on all (n+2)^3 nodes (boundary nodes included).  The coupling
    across the face between nodes p and q is the harmonic mean
    2 k_p k_q / (k_p + k_q) divided by h^2; D_p is the sum of the couplings of
    its six faces, boundary faces included.
    """
    rng = np.random.default_rng(seed)
    m = n + 2
    k = lognormal_field((m, m, m), rng, corr_len=corr_len, sigma=sigma)
    inv_h2 = float((n + 1) ** 2)
    inner = k[1:-1, 1:-1, 1:-1]

    def hmean(a, b):
        return 2.0 * a * b / (a + b)

    # upper faces along each axis (axis 0 = last numpy axis)
    up0 = hmean(inner, k[1:-1, 1:-1, 2:]) * inv_h2
    up1 = hmean(inner, k[1:-1, 2:, 1:-1]) * inv_h2
    up2 = hmean(inner, k[2:, 1:-1, 1:-1]) * inv_h2
    lo0 = hmean(inner, k[1:-1, 1:-1, :-2]) * inv_h2
    lo1 = hmean(inner, k[1:-1, :-2, 1:-1]) * inv_h2
    lo2 = hmean(inner, k[:-2, 1:-1, 1:-1]) * inv_h2
    diag = up0 + lo0
    diag += up1
    diag += lo1
    diag += up2
    diag += lo2
    del lo0, lo1, lo2
    b = np.ones((n, n, n), dtype=np.float64)
    faces = [np.ascontiguousarray(up0), np.ascontiguousarray(up1), np.ascontiguousarray(up2)]
    return Problem(3, (n, n, n), (0.0, 0.0, 0.0), 0.0, b, faces=faces,
                   diag=np.ascontiguousarray(diag), name=name or f"varcoef3d_{n}")


def variable_coefficient_2d(n0: int, n1: int, seed: int, corr_len: float = 8.0,
                            sigma: float = 1.0, name: str = "") -> Problem:
    """-div(k grad u) = 1 on the unit square, n0 x n1 interior nodes, Dirichlet
    zero: the 2D counterpart of variable_coefficient (k on all nodes,
    boundary nodes included; harmonic-mean face couplings divided by h_d^2;
    D_p the sum of its four face couplings)."""
    rng = np.random.default_rng(seed)
    k = lognormal_field((1, n1 + 2, n0 + 2), rng, corr_len=corr_len, sigma=sigma)[0]
    inv0, inv1 = float((n0 + 1) ** 2), float((n1 + 1) ** 2)
    inner = k[1:-1, 1:-1]

    def hmean(a, b):
        return 2.0 * a * b / (a + b)

    up0 = hmean(inner, k[1:-1, 2:]) * inv0
    lo0 = hmean(inner, k[1:-1, :-2]) * inv0
    up1 = hmean(inner, k[2:, 1:-1]) * inv1
    lo1 = hmean(inner, k[:-2, 1:-1]) * inv1
    diag = up0 + lo0
    diag += up1
    diag += lo1
    b = np.ones((1, n1, n0), dtype=np.float64)
    faces = [np.ascontiguousarray(up0).reshape(1, n1, n0), np.ascontiguousarray(up1).reshape(1, n1, n0),
             None]
    return Problem(2, (n0, n1, 1), (0.0, 0.0, 0.0), 0.0, b, faces=faces,
                   diag=np.ascontiguousarray(diag).reshape(1, n1, n0),
                   name=name or f"varcoef2d_{n0}x{n1}")


def random_faces(n: Sequence[int], seed: int, name: str = "") -> Problem:
    """A symmetric stencil with per-face couplings on any box (2D or 3D):
    every stored coupling (the ones towards the outside included) U(0.5, 1.5),
    a coupling to the ghost below the first layer U(0.5, 1.5) per axis, D_p
    the sum of the 2 ndim couplings of p (strictly diagonally dominant only
    through the ghost couplings, as a Dirichlet problem), b ~ U(-1, 1).  Drawn
    in that order: faces, then the low ghost couplings, then b."""
    ndim, n3 = _dims(n)
    shape = (n3[2], n3[1], n3[0])
    rng = np.random.default_rng(seed)
    faces = [rng.uniform(0.5, 1.5, shape) for _ in range(ndim)]
    diag = np.zeros(shape)
    for d in range(ndim):
        ax = 2 - d  # axis d is numpy axis 2 - d
        lo = np.empty(shape)
        idx_first = [slice(None)] * 3
        idx_first[ax] = slice(0, 1)
        idx_rest = [slice(None)] * 3
        idx_rest[ax] = slice(1, None)
        idx_prev = [slice(None)] * 3
        idx_prev[ax] = slice(0, -1)
        lo[tuple(idx_rest)] = faces[d][tuple(idx_prev)]
        ghost_shape = list(shape)
        ghost_shape[ax] = 1
        lo[tuple(idx_first)] = rng.uniform(0.5, 1.5, ghost_shape)
        diag += faces[d] + lo
    b = rng.uniform(-1, 1, shape)
    return Problem(ndim, n3, (0.0, 0.0, 0.0), 0.0, b, faces=faces + [None] * (3 - ndim),
                   diag=diag, name=name or f"randfaces{ndim}d")


def c3(seed: int = 0, n: int = 256) -> Problem:
    return variable_coefficient(n, seed, name=f"c3_varcoef3d_{n}")


def c4_instance(i: int, lo: int = 64, hi: int = 1024) -> Problem:
    """Instance i of the 2D batch: side n = round(exp(U(ln lo, ln hi))), b ~ U(-1, 1)."""
    rng = np.random.default_rng(1000 + i)
    n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    b = rng.uniform(-1.0, 1.0, size=(1, n, n))
    return poisson([n, n], b=b, name=f"c4_{i}_poisson2d_{n}")


def c4(count: int = 512, lo: int = 64, hi: int = 1024) -> List[Problem]:
    return [c4_instance(i, lo, hi) for i in range(count)]


def c5_instance(i: int, lo: int = 32, hi: int = 128) -> Problem:
    """Instance i of the 3D anisotropic batch.

    Draw order: the three sides (uniform on {lo..hi}), then a and b
    (log-uniform on [0.01, 1]), then the right-hand side U(-1, 1).
    """
    rng = np.random.default_rng(2000 + i)
    n = [int(v) for v in rng.integers(lo, hi + 1, size=3)]
    ab = np.exp(rng.uniform(math.log(0.01), math.log(1.0), size=2))
    rhs = rng.uniform(-1.0, 1.0, size=(n[2], n[1], n[0]))
    return anisotropic(n, (1.0, float(ab[0]), float(ab[1])), rhs,
                       name=f"c5_{i}_aniso3d_{n[0]}x{n[1]}x{n[2]}")


def c5(count: int = 128, lo: int = 32, hi: int = 128) -> List[Problem]:
    return [c5_instance(i, lo, hi) for i in range(count)]


# Section 3 data collection: the 1D Poisson training sizes and the random
# draws that pick a branch at every step (the draws are inputs, so the GPU
# collection and its CPU reference take the same walk).
TRAINING_SIZES = (2, 5, 10, 20, 30, 40, 50, 60, 70, 80, 90, 100, 200, 300, 400)


def training_problem(N: int) -> Problem:
    """1D Poisson, N unknowns, h = 1/(N+1), b = 1 (section 3)."""
    return poisson_1d(N, b=np.ones(N))


def training_draws(trials: int, max_steps: int, seed: int) -> np.ndarray:
    """Uniform draws in [0, 1), one per (trial, step)."""
    return np.random.default_rng(seed).random((trials, max_steps))


def neumann_laplace(n: int) -> Problem:
    """2D Laplace on the unit square with homogeneous Neumann boundaries
    (section 4.2.2): n x n grid nodes, boundary nodes included, h = 1/(n-1).

    Central differences with ghost nodes give the row 4 u_p - sum of the four
    neighbours (times 1/h^2), where a boundary node's inward neighbour stands
    in for the ghost and counts twice.  Halving every edge row and quartering
    the corner rows (exact in binary arithmetic, and without effect on Jacobi
    iterates, which are invariant under row scaling) makes the matrix
    symmetric: couplings 1/h^2 between interior faces, 1/(2 h^2) along the
    boundary, and D = the sum of a node's couplings, so A 1 = 0 (singular,
    constant null space).  b = 0."""
    assert n >= 2
    c = float((n - 1) ** 2)
    f0 = np.full((n, n), c)
    f1 = np.full((n, n), c)
    f0[0, :] *= 0.5       # faces along x on the rows y = 0 and y = 1
    f0[-1, :] *= 0.5
    f1[:, 0] *= 0.5       # faces along y on the columns x = 0 and x = 1
    f1[:, -1] *= 0.5
    f0[:, -1] = 0.0       # no neighbour beyond the last column / row
    f1[-1, :] = 0.0
    diag = np.zeros((n, n))
    diag[:, :-1] += f0[:, :-1]
    diag[:, 1:] += f0[:, :-1]
    diag[:-1, :] += f1[:-1, :]
    diag[1:, :] += f1[:-1, :]
    faces = [f0.reshape(1, n, n), f1.reshape(1, n, n), None]
    return Problem(2, (n, n, 1), (0.0, 0.0, 0.0), 0.0, np.zeros((1, n, n)), faces=faces,
                   diag=diag.reshape(1, n, n), name=f"neumann_laplace_{n}")


def random_start(prob: Problem, seed: int) -> np.ndarray:
    """Random initial guess U(-1, 1) (section 4.2.2 starts from a random vector)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, prob.shape)


# ---------------------------------------------------------------------------
# General matrices (section 4.2.1 random tridiagonal systems, section 4.2.4
# finite elements on unstructured meshes)
# ---------------------------------------------------------------------------

def csr_problem(rowptr: np.ndarray, col: np.ndarray, val: np.ndarray, b: np.ndarray,
                name: str = "") -> Problem:
    n = len(rowptr) - 1
    return Problem(1, (n, 1, 1), (0.0, 0.0, 0.0), 0.0,
                   np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(1, 1, n)),
                   csr=(np.asarray(rowptr, dtype=np.int64), np.asarray(col, dtype=np.int32),
                        np.asarray(val, dtype=np.float64)), name=name or "csr")


def to_csr(prob: Problem) -> Problem:
    """A stencil problem written as a sparse matrix: per row the diagonal, then
    the neighbours in the stencil's order (axis 0 lower, upper, axis 1 lower,
    upper, ...), entries -coupling."""
    n0, n1, n2 = prob.n
    N = n0 * n1 * n2
    strides = (1, n0, n0 * n1)
    diag = prob.diag.reshape(-1) if prob.diag is not None else np.full(N, prob.dconst)
    faces = [prob.faces[d].reshape(-1) if prob.faces is not None and prob.faces[d] is not None
             else None for d in range(3)] if prob.faces is not None else [None, None, None]
    rowptr, col, val = [0], [], []
    for i2 in range(n2):
        for i1 in range(n1):
            for i0 in range(n0):
                ii = (i0, i1, i2)
                p = i0 + n0 * (i1 + n1 * i2)
                col.append(p)
                val.append(diag[p])
                for d in range(prob.ndim):
                    if ii[d] > 0:
                        q = p - strides[d]
                        col.append(q)
                        val.append(-(faces[d][q] if faces[d] is not None else prob.c[d]))
                    if ii[d] < prob.n[d] - 1:
                        q = p + strides[d]
                        col.append(q)
                        val.append(-(faces[d][p] if faces[d] is not None else prob.c[d]))
                rowptr.append(len(col))
    return csr_problem(np.array(rowptr), np.array(col), np.array(val), prob.b.reshape(-1),
                       name=(prob.name or "stencil") + "_csr")


def random_tridiagonal(N: int, seed: int) -> Problem:
    """Random symmetric diagonally dominant tridiagonal matrix (section 4.2.1).

    Draw order: the diagonal d ~ U(0, 1) (N values), then the off-diagonal e ~
    U(0, 1) (N - 1 values, used above and below the diagonal), then b ~
    U(-1, 1).  A row that is not diagonally dominant gets |d_i| = the sum of
    its off-diagonal |e|; then d_0 = 2 e_0 and d_{N-1} = 2 e_{N-2}.  (The paper
    does not state b; with b = 1 the smallest systems are solved by a single
    weighted-Jacobi sweep, and a random b reproduces all of its comparisons.)
    Returned as a 1D problem with per-face couplings (face = -e) and a
    per-point diagonal."""
    assert N >= 2
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.0, 1.0, N)
    e = rng.uniform(0.0, 1.0, N - 1)
    off = np.zeros(N)
    off[:-1] += np.abs(e)
    off[1:] += np.abs(e)
    d = np.where(np.abs(d) < off, off, d)
    d[0] = 2.0 * e[0]
    d[-1] = 2.0 * e[-1]
    b = rng.uniform(-1.0, 1.0, N)
    face = np.zeros(N)
    face[:-1] = -e
    return Problem(1, (N, 1, 1), (0.0, 0.0, 0.0), 0.0, b.reshape(1, 1, N),
                   faces=[face.reshape(1, 1, N), None, None], diag=d.reshape(1, 1, N),
                   name=f"tridiag_{N}_{seed}")


def _fem_mesh(geometry: str, h: float, seed: int):
    """Seeded point set and Delaunay triangles of a disk (radius 1) or a plate
    with a hole ([-1, 1]^2 minus the disk of radius 0.5, points twice as dense
    near the hole).  Returns (points, triangles, boundary mask)."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)

    def jittered(lo, hi, step):
        g = np.arange(lo, hi + 1e-12, step)
        X, Y = np.meshgrid(g, g)
        pts = np.stack([X.ravel(), Y.ravel()], axis=1)
        return pts + rng.uniform(-0.25 * step, 0.25 * step, pts.shape)

    def circle(r, step, c=(0.0, 0.0)):
        m = max(8, int(math.ceil(2 * math.pi * r / step)))
        t = 2 * math.pi * np.arange(m) / m
        return np.stack([c[0] + r * np.cos(t), c[1] + r * np.sin(t)], axis=1)

    if geometry == "disk":
        bnd = circle(1.0, h)
        inner = jittered(-1.0, 1.0, h)
        inner = inner[np.hypot(inner[:, 0], inner[:, 1]) < 1.0 - 0.5 * h]
    elif geometry == "plate_hole":
        m = int(round(2.0 / h))
        s = np.linspace(-1.0, 1.0, m + 1)
        edges = np.concatenate([np.stack([s, -np.ones_like(s)], 1), np.stack([s, np.ones_like(s)], 1),
                                np.stack([-np.ones_like(s[1:-1]), s[1:-1]], 1),
                                np.stack([np.ones_like(s[1:-1]), s[1:-1]], 1)])
        hole = circle(0.5, 0.5 * h)
        bnd = np.concatenate([edges, hole])
        coarse = jittered(-1.0, 1.0, h)
        fine = jittered(-1.0, 1.0, 0.5 * h)
        rc, rf = np.hypot(coarse[:, 0], coarse[:, 1]), np.hypot(fine[:, 0], fine[:, 1])
        coarse = coarse[(rc > 0.5 + 0.5 * h) & (rc >= 0.8) & (np.max(np.abs(coarse), 1) < 1.0 - 0.5 * h)]
        fine = fine[(rf > 0.5 + 0.25 * h) & (rf < 0.8) & (np.max(np.abs(fine), 1) < 1.0 - 0.25 * h)]
        inner = np.concatenate([coarse, fine])
    else:
        raise ValueError(geometry)
    pts = np.concatenate([bnd, inner])
    is_bnd = np.zeros(len(pts), dtype=bool)
    is_bnd[:len(bnd)] = True
    tri = Delaunay(pts).simplices
    if geometry == "plate_hole":
        cen = pts[tri].mean(axis=1)
        tri = tri[np.hypot(cen[:, 0], cen[:, 1]) > 0.5]
    return pts, tri, is_bnd


def fem_stiffness(pts: np.ndarray, tri: np.ndarray):
    """P1 stiffness matrix (dense-free, COO) and lumped load for f = 1:
    K_e[i][j] = area * grad(phi_i) . grad(phi_j), b_i += area / 3."""
    P = pts[tri]                                   # (T, 3, 2)
    d1 = P[:, 1] - P[:, 0]
    d2 = P[:, 2] - P[:, 0]
    area = 0.5 * np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    # gradients of the barycentric functions: rotate the opposite edge
    g = np.empty_like(P)
    for i in range(3):
        a, b = P[:, (i + 1) % 3], P[:, (i + 2) % 3]
        edge = b - a
        g[:, i, 0] = edge[:, 1]
        g[:, i, 1] = -edge[:, 0]
    sign = np.sign((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                   - (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0]))
    g = g * (sign / (2.0 * area))[:, None, None]
    rows, cols, vals = [], [], []
    for i in range(3):
        for j in range(3):
            rows.append(tri[:, i])
            cols.append(tri[:, j])
            vals.append(area * np.sum(g[:, i] * g[:, j], axis=1))
    load = np.zeros(len(pts))
    for i in range(3):
        np.add.at(load, tri[:, i], area / 3.0)
    return (np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)), load, area


def fem_poisson(geometry: str, h: float, seed: int = 0) -> Problem:
    """-laplace(u) = 1 with u = 0 on the boundary, P1 finite elements on a
    seeded Delaunay mesh (a stand-in for the paper's distmesh meshes, which
    are not available); unknowns are the interior nodes."""
    import scipy.sparse as sp
    pts, tri, is_bnd = _fem_mesh(geometry, h, seed)
    (r, c, v), load, _ = fem_stiffness(pts, tri)
    K = sp.coo_matrix((v, (r, c)), shape=(len(pts), len(pts))).tocsr()
    inner = np.nonzero(~is_bnd)[0]
    A = K[inner][:, inner].tocsr()
    A.sort_indices()
    A.eliminate_zeros()
    return csr_problem(A.indptr, A.indices, A.data, load[inner],
                       name=f"fem_{geometry}_h{h:g}_s{seed}")
