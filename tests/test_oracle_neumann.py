"""Pins of the CPU reference for the Neumann Laplace problem and the update
stopping test (section 4.2.2, Eq. (25)).

* The operator: built entry by entry from the ghost-node central differences
  the paper describes, then row-scaled by 1/2 on edges and 1/4 at corners, it
  equals the symmetric face form the solver takes, exactly; it is symmetric
  with A 1 = 0, and one Jacobi step is the same in both forms.
* The iteration: D^-1 A of this stencil is diagonalised by products of
  DCT-I cosines with eigenvalues (2 - cos(k pi/(n-1)) - cos(l pi/(n-1))) / 2,
  so every sweep multiplies mode (k, l) by 1 - w mu.  That model, with no
  stencil code, fixes every sweep's largest update, the sweep at which the
  test first holds, and (through the residual norms) the levels Algorithm 1
  picks.
* The paper's comparison: the heuristic needs fewer sweeps than the
  increasing rule.
"""
import numpy as np
import pytest
import scipy.fft

import oracle
import workloads
from spectral import dense_matrix

TOL = 1e-10


def ghost_node_matrix(n):
    """Rows 4 u_p - sum of neighbours / h^2, a ghost replaced by its mirror."""
    c = float((n - 1) ** 2)
    A = np.zeros((n * n, n * n))
    for j in range(n):
        for i in range(n):
            p = i + n * j
            A[p, p] += 4 * c
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ii, jj = i + di, j + dj
                if ii < 0 or ii >= n:
                    ii = i - di  # mirror node of the ghost
                if jj < 0 or jj >= n:
                    jj = j - dj
                A[p, ii + n * jj] -= c
    return A


@pytest.mark.parametrize("n", [2, 3, 6])
def test_operator_is_the_scaled_ghost_node_stencil(n):
    prob = workloads.neumann_laplace(n)
    A = dense_matrix(prob)
    G = ghost_node_matrix(n)
    scale = np.ones(n * n)
    for j in range(n):
        for i in range(n):
            k = (i in (0, n - 1)) + (j in (0, n - 1))
            scale[i + n * j] = 0.5 ** k
    assert np.array_equal(scale[:, None] * G, A)
    assert np.array_equal(A, A.T)
    assert np.array_equal(A @ np.ones(n * n), np.zeros(n * n))


def test_one_sweep_equals_the_ghost_node_jacobi_step():
    n = 7
    prob = workloads.neumann_laplace(n)
    x = workloads.random_start(prob, seed=1)
    G = ghost_node_matrix(n)
    w = 1.7
    want = x.reshape(-1) + w * (-(G @ x.reshape(-1)) / np.diag(G))
    got = oracle.sweep(prob, x, w).reshape(-1)
    assert np.max(np.abs(got - want)) <= 1e-13


def modal_model(prob, x0, rule, tol, max_cycles=100000):
    """Sweep-by-sweep model in the DCT-I eigenbasis of D^-1 A."""
    n = prob.n[0]
    th = np.arange(n) * np.pi / (n - 1)
    mu = (2.0 - np.cos(th)[None, :] - np.cos(th)[:, None]) / 2.0  # [j (y), i (x)]
    diag = prob.diag.reshape(n, n)
    C = scipy.fft.dctn(x0.reshape(n, n), type=1)

    def res_norm(C):
        r = -diag * scipy.fft.idctn(mu * C, type=1)
        return float(np.sqrt(np.sum(r * r)))

    r0 = res_norm(C)
    prev, level, sweeps, levels, maxes = r0, 0, 0, [], []
    for _ in range(max_cycles):
        lv = level
        levels.append(lv)
        for w in oracle.scheme(lv):
            upd = scipy.fft.idctn(-w * mu * C, type=1)
            C = C * (1.0 - w * mu)
            sweeps += 1
            m = float(np.max(np.abs(upd)))
            maxes.append(m)
            if m < tol:
                return {"sweeps": sweeps, "levels": levels, "maxes": maxes}
        nrm = res_norm(C)
        ratio = nrm / prev
        prev = nrm
        if rule == "heuristic":
            level = level + 1 if ratio > 0.4 else (level - 1 if 0.2 < ratio < 0.4 else level)
        else:
            level = level + 1
        level = min(max(level, 0), 24)
    return {"sweeps": sweeps, "levels": levels, "maxes": maxes}


@pytest.mark.parametrize("n,rule,seed", [(16, "heuristic", 0), (16, "increasing", 1),
                                         (33, "heuristic", 2), (24, "increasing", 3)])
def test_stop_sweep_and_levels_follow_the_modal_model(n, rule, seed):
    prob = workloads.neumann_laplace(n)
    x0 = workloads.random_start(prob, seed)
    model = modal_model(prob, x0, rule, TOL)
    got = oracle.solve(prob, x0, rule=rule, tol=TOL, tol_mode="update_inf", max_cycles=100000)
    assert got["converged"]
    # a stop decided by less than 1e-4 relative is left to rounding
    m = model["maxes"]
    if abs(m[-1] - TOL) > 1e-4 * TOL and (len(m) < 2 or abs(m[-2] - TOL) > 1e-4 * TOL):
        assert got["sweeps"] == model["sweeps"]
    assert list(got["levels"]) == model["levels"][:len(got["levels"])]
    assert len(got["levels"]) == len(model["levels"])


def test_heuristic_beats_the_increasing_rule():
    n = 32
    prob = workloads.neumann_laplace(n)
    for seed in range(3):
        x0 = workloads.random_start(prob, seed)
        h = oracle.solve(prob, x0, rule="heuristic", tol=TOL, tol_mode="update_inf", max_cycles=100000)
        i = oracle.solve(prob, x0, rule="increasing", tol=TOL, tol_mode="update_inf", max_cycles=100000)
        assert h["converged"] and i["converged"]
        assert h["sweeps"] < i["sweeps"]


def test_limit_is_a_constant():
    # the iterates converge to the constant mode of x0 (A is singular)
    n = 12
    prob = workloads.neumann_laplace(n)
    x0 = workloads.random_start(prob, 5)
    out = oracle.solve(prob, x0, rule="heuristic", tol=1e-12, tol_mode="update_inf", max_cycles=100000)
    x = out["x"].reshape(-1)
    assert np.max(x) - np.min(x) < 1e-9
    # the DCT-I mode (0, 0) is untouched by every sweep: it is the limit
    c00 = scipy.fft.dctn(x0.reshape(n, n), type=1)[0, 0] / (2 * (n - 1)) ** 2
    assert abs(np.mean(x) - c00) < 1e-9


def test_update_test_is_binary64_only():
    prob = workloads.neumann_laplace(8)
    x0 = workloads.random_start(prob, 0)
    out = oracle.solve(prob, x0, tol=TOL, tol_mode="update_inf", precision="f32")
    assert out["status"] == "invalid"
