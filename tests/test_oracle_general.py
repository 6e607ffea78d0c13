"""Pins of the CPU reference on general matrices (sections 4.2.1 and 4.2.4).

* A stencil written as a sparse matrix (entries -c in the stencil's order)
  gives the stencil's sweeps bit for bit; both solve to numpy's dense answer.
* The random tridiagonal systems follow the paper's construction (symmetric,
  diagonally dominant, end rows 2 e), D^-1 A has its spectrum in (0, 2), and
  the paper's comparisons hold on 20 matrices per size: the heuristic needs
  fewer sweeps than the increasing rule, about half at the larger sizes, and
  unweighted Jacobi beats the increasing rule only for the smallest systems.
* The finite element systems: the stiffness matrix is symmetric with zero row
  sums, reproduces the energy of linear functions exactly, the load sums to
  the area, Delaunay meshes give non-positive couplings; SRJ reaches the
  sparse direct solution; sweeps to 1e-9 grow about like sqrt(N) under
  refinement (the paper's scaling), far slower than Jacobi's N.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import workloads
from spectral import dense_matrix

STENCILS = [
    ("1d_faces", lambda: workloads.random_tridiagonal(30, 1)),
    ("2d_const", lambda: workloads.poisson([9, 7], b=np.random.default_rng(1).uniform(-1, 1, (1, 7, 9)))),
    ("3d_aniso", lambda: workloads.anisotropic([5, 4, 6], (1.0, 0.3, 0.05),
                                               np.random.default_rng(2).uniform(-1, 1, (6, 4, 5)))),
    ("3d_varcoef", lambda: workloads.variable_coefficient(5, seed=3, corr_len=2.0)),
]


def _dense_csr(prob):
    rp, col, val = prob.csr
    return sp.csr_matrix((val, col, rp), shape=(len(rp) - 1, len(rp) - 1)).toarray()


@pytest.mark.parametrize("name,make", STENCILS, ids=[s[0] for s in STENCILS])
def test_stencil_as_sparse_matrix_is_bit_identical(name, make):
    prob = make()
    csr = workloads.to_csr(prob)
    assert np.array_equal(_dense_csr(csr), dense_matrix(prob))
    x = np.random.default_rng(4).uniform(-1, 1, prob.shape)
    for w in (0.7, 1.9, 13.0):
        a = oracle.sweep(prob, x, w).reshape(-1)
        b = oracle.sweep(csr, x.reshape(csr.shape), w).reshape(-1)
        assert np.array_equal(a, b)
    ra = oracle.solve(prob, tol=1e-11, max_cycles=400)
    rb = oracle.solve(csr, tol=1e-11, max_cycles=400)
    assert np.array_equal(ra["levels"], rb["levels"]) and np.array_equal(ra["norms"], rb["norms"])
    exact = np.linalg.solve(dense_matrix(prob), prob.b.reshape(-1))
    assert np.max(np.abs(rb["x"].reshape(-1) - exact)) <= 1e-8 * np.max(np.abs(exact))


@pytest.mark.parametrize("N", [2, 3, 10, 57])
def test_random_tridiagonal_construction(N):
    prob = workloads.random_tridiagonal(N, seed=N)
    A = dense_matrix(prob)
    assert np.array_equal(A, A.T)
    off = np.sum(np.abs(A), axis=1) - np.abs(np.diag(A))
    assert np.all(np.diag(A) >= off * (1 - 1e-15))
    assert A[0, 0] == 2 * abs(A[0, 1]) and A[-1, -1] == 2 * abs(A[-1, -2])
    lam = np.linalg.eigvals(np.diag(1 / np.diag(A)) @ A).real
    assert np.all(lam > 0) and np.all(lam < 2)
    ref = oracle.solve(prob, tol=1e-12, tol_mode="absolute", max_cycles=5000)
    assert ref["converged"]
    exact = np.linalg.solve(A, prob.b.reshape(-1))
    assert np.max(np.abs(ref["x"].reshape(-1) - exact)) <= 1e-9 * max(1.0, np.max(np.abs(exact)))


def _mean_sweeps(N, rule):
    out = []
    for s in range(20):
        o = oracle.solve(workloads.random_tridiagonal(N, seed=s), rule=rule, tol=1e-7,
                         tol_mode="absolute", stop_per_sweep=True, max_cycles=2_000_000,
                         max_sweeps=5_000_000)
        assert o["converged"]
        out.append(o["sweeps"])
    return float(np.mean(out))


def test_tridiagonal_comparisons_of_the_paper():
    # heuristic below increasing everywhere, about half at the larger sizes
    for N in (5, 20, 100, 400):
        h, i = _mean_sweeps(N, "heuristic"), _mean_sweeps(N, "increasing")
        assert h < i, N
        if N >= 100:
            assert h < 0.6 * i, N
    # unweighted Jacobi beats the increasing rule only for the smallest systems
    assert _mean_sweeps(2, "jacobi") < _mean_sweeps(2, "increasing")
    assert _mean_sweeps(20, "jacobi") > _mean_sweeps(20, "increasing")


@pytest.mark.parametrize("geometry", ["disk", "plate_hole"])
def test_fem_assembly(geometry):
    pts, tri, is_bnd = workloads._fem_mesh(geometry, 0.1, seed=3)
    (r, c, v), load, area = workloads.fem_stiffness(pts, tri)
    K = sp.coo_matrix((v, (r, c)), shape=(len(pts), len(pts))).toarray()
    assert np.allclose(K, K.T, atol=1e-13)
    assert np.max(np.abs(K.sum(axis=1))) < 1e-12
    total = float(np.sum(area))
    assert np.sum(load) == pytest.approx(total, rel=1e-13)
    u = 2.0 * pts[:, 0] - 3.0 * pts[:, 1]  # energy of a linear function: |grad u|^2 * area
    assert u @ K @ u == pytest.approx(13.0 * total, rel=1e-12)
    offd = K[~np.eye(len(pts), dtype=bool)]
    assert np.max(offd) <= 1e-12  # Delaunay: no positive coupling
    # the mesh covers the domain: area of the disk / plate minus hole polygon
    want = np.pi if geometry == "disk" else 4.0 - np.pi * 0.25
    assert total == pytest.approx(want, rel=0.02)


@pytest.mark.parametrize("geometry", ["disk", "plate_hole"])
def test_fem_solve_reaches_the_direct_solution(geometry):
    prob = workloads.fem_poisson(geometry, 0.1, seed=1)
    rp, col, val = prob.csr
    A = sp.csr_matrix((val, col, rp))
    exact = spla.spsolve(A.tocsc(), prob.b.reshape(-1))
    out = oracle.solve(prob, tol=1e-12, tol_mode="absolute", max_cycles=5000)
    assert out["converged"]
    assert np.max(np.abs(out["x"].reshape(-1) - exact)) <= 1e-9 * np.max(np.abs(exact))


def test_fem_sweeps_grow_like_sqrt_n():
    sweeps, ns = [], []
    for h in (0.1, 0.05, 0.025):
        prob = workloads.fem_poisson("disk", h, seed=0)
        o = oracle.solve(prob, tol=1e-9, tol_mode="absolute", stop_per_sweep=True, max_cycles=10000)
        assert o["converged"]
        sweeps.append(o["sweeps"])
        ns.append(prob.npoints)
    for k in (1, 2):
        growth = sweeps[k] / sweeps[k - 1]
        n_ratio = ns[k] / ns[k - 1]  # about 4 per halving of h
        assert 0.5 * np.sqrt(n_ratio) < growth < 1.6 * np.sqrt(n_ratio), (sweeps, ns)
