"""Pins of the oracle's sweep, residual and cycle (no GPU).

* A x of the matrix-free stencil equals a dense matrix built entry by entry
  from A = D + L + U (section 2, Eq. 1), for constant, anisotropic and
  variable-coefficient stencils; the variable-coefficient A is symmetric.
* One sweep equals weighted Jacobi written as Eq. 3 with dense matrices:
  w (B_J x + D^-1 b) + (1 - w) x, B_J = -D^-1 (L + U).
* Level 0 (P = 1) is weighted Jacobi with w = 2/3 (section 2, discussion
  of Fig. 1).
* A sine-mode error shrinks in one cycle by exactly G_M(1 - mu_k) (Eq. (12)),
  with G_M from the closed form T_M(f(l)) / 3 (Eq. (13)).
* The residual norm equals numpy's norm of b - A x with the dense matrix.
"""
import functools

import numpy as np
import pytest

import workloads
from spectral import G_closed, dense_matrix


@functools.lru_cache(maxsize=1)
def small_problems():
    rng = np.random.default_rng(7)
    out = []
    out.append(workloads.poisson([9], b=rng.uniform(-1, 1, (1, 1, 9))))
    out.append(workloads.poisson([5, 4], b=rng.uniform(-1, 1, (1, 4, 5))))
    out.append(workloads.poisson([3, 4, 2], b=rng.uniform(-1, 1, (2, 4, 3))))
    out.append(workloads.anisotropic([4, 3, 3], (1.0, 0.05, 0.3), rng.uniform(-1, 1, (3, 3, 4))))
    out.append(workloads.variable_coefficient(4, seed=3, corr_len=2.0))
    vc = workloads.variable_coefficient(3, seed=4, corr_len=1.5)
    vc.b = rng.uniform(-1, 1, vc.shape)
    out.append(vc)
    vc2 = workloads.variable_coefficient_2d(5, 4, seed=5, corr_len=1.5)
    vc2.b = rng.uniform(-1, 1, vc2.shape)
    out.append(vc2)
    out.append(workloads.random_faces([4, 3, 2], seed=6))
    out.append(workloads.random_faces([3, 5], seed=7))
    return out


@pytest.mark.parametrize("k", range(9))
def test_apply_matches_dense(orc, k):
    prob = small_problems()[k]
    A = dense_matrix(prob)
    assert np.array_equal(A, A.T)
    x = np.random.default_rng(k).uniform(-1, 1, prob.shape)
    y = orc.apply(prob, x).ravel()
    np.testing.assert_allclose(y, A @ x.ravel(), rtol=1e-13, atol=1e-13 * np.abs(A).max())


@pytest.mark.parametrize("k", range(9))
def test_sweep_is_weighted_jacobi_eq3(orc, k):
    prob = small_problems()[k]
    A = dense_matrix(prob)
    D = np.diag(np.diag(A))
    LU = A - D
    Dinv = np.diag(1.0 / np.diag(A))
    BJ = -Dinv @ LU
    x = np.random.default_rng(10 + k).uniform(-1, 1, prob.shape)
    b = prob.b.ravel()
    for w in (2.0 / 3.0, 0.51, 1.7, 17.84):
        ref = w * (BJ @ x.ravel() + Dinv @ b) + (1.0 - w) * x.ravel()
        got = orc.sweep(prob, x, w).ravel()
        scale = np.abs(x).max() + w * np.abs(Dinv @ b).max() + w * np.abs(BJ @ x.ravel()).max()
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14 * scale)


@pytest.mark.parametrize("k", range(9))
def test_residual_norm_matches_dense(orc, k):
    prob = small_problems()[k]
    A = dense_matrix(prob)
    x = np.random.default_rng(20 + k).uniform(-1, 1, prob.shape)
    ref = np.linalg.norm(prob.b.ravel() - A @ x.ravel())
    assert abs(orc.residual_norm(prob, x) - ref) <= 1e-13 * (ref + np.abs(A).max())


def test_level0_is_weighted_jacobi_two_thirds(orc):
    prob = small_problems()[1]
    A = dense_matrix(prob)
    x0 = np.random.default_rng(1).uniform(-1, 1, prob.shape)
    out = orc.solve(prob, x0, rule="fixed", fixed_level=0, tol=1e-300, max_cycles=1)
    assert out["cycles"] == 1 and out["sweeps"] == 1
    Dinv = 1.0 / np.diag(A)
    ref = x0.ravel() + (2.0 / 3.0) * Dinv * (prob.b.ravel() - A @ x0.ravel())
    np.testing.assert_allclose(out["x"].ravel(), ref, rtol=1e-15, atol=1e-15)


def test_face_form_equals_constant_form(orc):
    # a variable-coefficient description with constant faces is the same operator
    rng = np.random.default_rng(5)
    prob = workloads.poisson([6, 5, 4], b=rng.uniform(-1, 1, (4, 5, 6)))
    faces = [np.full(prob.shape, prob.c[d]) for d in range(3)]
    vprob = workloads.Problem(3, prob.n, (0.0, 0.0, 0.0), 0.0, prob.b, faces=faces,
                              diag=np.full(prob.shape, prob.dconst))
    x = rng.uniform(-1, 1, prob.shape)
    assert np.array_equal(orc.sweep(prob, x, 1.3), orc.sweep(vprob, x, 1.3))
    assert orc.residual_norm(prob, x) == orc.residual_norm(vprob, x)


def _mu(prob, k):
    mu = 0.0
    for d in range(prob.ndim):
        mu += prob.c[d] / prob.dconst * 2.0 * (1.0 - np.cos(k[d] * np.pi / (prob.n[d] + 1)))
    return mu


@pytest.mark.parametrize("case", [
    ([100], [1]), ([100], [37]), ([100], [99]), ([255], [3]),
    ([24, 17], [2, 5]), ([12, 9, 7], [1, 4, 6])])
@pytest.mark.parametrize("level", [0, 2, 5, 9, 11, 14])
def test_sine_mode_decay(orc, case, level):
    n, k = case
    prob = workloads.poisson(n, b=np.zeros(tuple(reversed(list(n) + [1] * (3 - len(n))))))
    x0 = workloads.sine_mode(n, k)
    out = orc.solve(prob, x0, rule="fixed", fixed_level=level, tol=1e-300, max_cycles=1)
    M = orc.level_M(level)
    lam_j = 1.0 - _mu(prob, k)
    # closed form (Appendix A) and the factor product of Eq. (12) with the oracle's factors
    g = G_closed(M, np.array([lam_j]))[0]
    gp = np.prod([(1.0 - w * _mu(prob, k)) for w in orc.scheme(level)])
    assert abs(g - gp) <= 1e-12 * max(1.0, M / 10.0)
    err = np.max(np.abs(out["x"] - g * x0))
    # round-off injected mid-cycle can be amplified by the later factors
    assert err <= 1e-13 * max(1.0, M) * 50
