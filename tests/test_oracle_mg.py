"""Pins of the oracle's multigrid with SRJ smoothing (oracle/srj_mg.c).

The paper only names SRJ as a multigrid smoother (section 5); the design is
the library's reading (vertex-centred coarsening, full weighting, multilinear
interpolation, coarse couplings and diagonal / 4).  The oracle is pinned
against facts that do not come from its own code:

* transfer operators: full weighting is 2^-d times the transpose of the
  interpolation (an identity of the two definitions, checked on random
  vectors); interpolation reproduces a product of tent functions whose kinks
  lie on coarse points, and full weighting reproduces a multilinear
  function, both exactly (dyadic grid values);
* the Galerkin product R A P of the 1D Poisson matrix equals the
  rediscretised coarse matrix (couplings and diagonal / 4), exactly;
* the two-grid operator on a 1D sine mode: with one weighted-Jacobi
  (level 0, w = 2/3) pre-sweep and an exact coarse solve, the mode k maps to
  (1 - 2 w s) s (w_k + w_k'), s = sin^2(k pi h / 2), k' = n + 1 - k (the
  closed form follows from the mode algebra of the two transfer operators;
  derivation in the design notes), and with a post-sweep as well to
  (1 - 2 w s) s ((1 - 2 w s) w_k + (1 - 2 w c) w_k'), c = 1 - s;
* converged V-cycles reach the dense solution of A x = b (LAPACK through
  numpy) on small 2D and 3D grids;
* the smoothing level of each V-cycle follows Algorithm 1 from the V-cycle
  norms the oracle reports.
"""
import numpy as np
import pytest

import workloads


def _rand_problem(n, seed):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(list(n) + [1] * (3 - len(n))))
    return workloads.poisson(n, b=rng.uniform(-1, 1, shape))


def test_hierarchy_sizes(orc):
    assert orc.mg_hierarchy(workloads.poisson([95, 47])) == [
        (95, 47, 1), (47, 23, 1), (23, 11, 1), (11, 5, 1), (5, 2, 1)]
    assert orc.mg_hierarchy(workloads.poisson([31, 31, 31])) == [
        (31, 31, 31), (15, 15, 15), (7, 7, 7), (3, 3, 3), (1, 1, 1)]
    assert orc.mg_hierarchy(workloads.poisson([64, 63])) == [(64, 63, 1)]
    assert orc.mg_hierarchy(workloads.poisson([127]), max_levels=3) == [
        (127, 1, 1), (63, 1, 1), (31, 1, 1)]


@pytest.mark.parametrize("n", [[15], [15, 7], [7, 15, 5], [31, 9]])
def test_restriction_is_scaled_transpose_of_interpolation(orc, n):
    prob = _rand_problem(n, 1)
    d = len(n)
    rng = np.random.default_rng(2)
    r = rng.uniform(-1, 1, prob.shape)
    ec = rng.uniform(-1, 1, orc.coarse_shape(prob))
    # R r: the restricted residual of x = 0 for right-hand side r
    pr = workloads.poisson(n, b=r)
    Rr = orc.restrict_residual(pr, np.zeros(prob.shape))
    Pe = orc.prolong_add(prob, ec, np.zeros(prob.shape))
    lhs = 2.0 ** d * float(np.sum(Rr * ec))
    rhs = float(np.sum(r * Pe))
    assert abs(lhs - rhs) <= 1e-13 * (abs(rhs) + np.sum(np.abs(r)))


def _tent(m_plus_1, count):
    # tent(x) = min(x, 1 - x) at x = (j + 1) / (count + 1)
    x = (np.arange(count) + 1.0) / (count + 1.0)
    return np.minimum(x, 1.0 - x)


@pytest.mark.parametrize("n", [[15], [15, 31], [15, 7, 31]])
def test_interpolation_reproduces_tent_products(orc, n):
    # kinks at x = 1/2, a coarse point when (n - 1)/2 is odd; all values dyadic
    prob = workloads.poisson(n)
    d = len(n)
    fine = [_tent(None, n[a]) for a in range(d)] + [np.ones(1)] * (3 - d)
    coarse = [_tent(None, (n[a] - 1) // 2) for a in range(d)] + [np.ones(1)] * (3 - d)
    f_fine = np.einsum("k,j,i->kji", fine[2], fine[1], fine[0])
    f_coarse = np.einsum("k,j,i->kji", coarse[2], coarse[1], coarse[0])
    got = orc.prolong_add(prob, f_coarse, np.zeros(prob.shape))
    assert np.array_equal(got, f_fine)


@pytest.mark.parametrize("n", [[15], [15, 31], [7, 15, 31]])
def test_full_weighting_reproduces_multilinear(orc, n):
    d = len(n)
    axes = [(np.arange(n[a]) + 1.0) / (n[a] + 1.0) for a in range(d)] + [np.ones(1)] * (3 - d)
    cax = [(np.arange((n[a] - 1) // 2) + 1.0) / ((n[a] - 1) // 2 + 1.0) for a in range(d)] + \
        [np.ones(1)] * (3 - d)
    f = np.einsum("k,j,i->kji", axes[2], axes[1], axes[0])
    fc = np.einsum("k,j,i->kji", cax[2], cax[1], cax[0])
    prob = workloads.poisson(n, b=f)
    got = orc.restrict_residual(prob, np.zeros(prob.shape))
    assert np.array_equal(got, fc)


@pytest.mark.parametrize("n", [7, 15, 31])
def test_galerkin_product_equals_rediscretised_1d(orc, n):
    prob = workloads.poisson([n])
    m = (n - 1) // 2
    c = float((n + 1) ** 2)
    G = np.zeros((m, m))
    for J in range(m):
        v = np.zeros((1, 1, m))
        v[0, 0, J] = 1.0
        Pv = orc.prolong_add(prob, v, np.zeros(prob.shape))
        APv = orc.apply(prob, Pv)
        G[:, J] = orc.restrict_residual(workloads.poisson([n], b=APv), np.zeros(prob.shape)).ravel()
    want = np.diag(np.full(m, 2.0 * c / 4.0)) - np.diag(np.full(m - 1, c / 4.0), 1) - \
        np.diag(np.full(m - 1, c / 4.0), -1)
    assert np.array_equal(G, want)


@pytest.mark.parametrize("n,k,post", [(31, 3, 0), (31, 11, 0), (63, 5, 1), (63, 20, 1), (15, 2, 1)])
def test_two_grid_closed_form_1d(orc, n, k, post):
    h = 1.0 / (n + 1)
    j = np.arange(n) + 1.0
    wk = np.sin(k * np.pi * j * h)
    wk2 = np.sin((n + 1 - k) * np.pi * j * h)
    s = np.sin(k * np.pi * h / 2) ** 2
    c = 1.0 - s
    om = 2.0 / 3.0
    if post == 0:
        want = (1 - 2 * om * s) * s * (wk + wk2)
    else:
        want = (1 - 2 * om * s) * s * ((1 - 2 * om * s) * wk + (1 - 2 * om * c) * wk2)
    prob = workloads.poisson([n], b=np.zeros((1, 1, n)))
    out = orc.mg_solve(prob, wk.reshape(1, 1, n), rule="fixed", start_level=0, pre=1,
                       post=post, max_levels=2, coarse_tol=1e-14, coarse_max_cycles=5000,
                       tol=1e-300, max_vcycles=1)
    got = out["x"].ravel()
    assert out["vcycles"] == 1
    assert np.max(np.abs(got - want)) <= 1e-11 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("n", [[15, 7], [31, 15], [7, 7, 7], [15, 7, 3]])
def test_vcycles_reach_dense_solution(orc, n):
    prob = _rand_problem(n, 3)
    N = prob.npoints
    A = np.zeros((N, N))
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1.0
        A[:, i] = orc.apply(prob, e.reshape(prob.shape)).ravel()
    xd = np.linalg.solve(A, prob.b.ravel())
    out = orc.mg_solve(prob, rule="heuristic", start_level=0, tol=1e-13, coarse_tol=1e-12)
    assert out["status"] == "ok"
    assert np.max(np.abs(out["x"].ravel() - xd)) <= 1e-10 * np.max(np.abs(xd))


def test_smoothing_levels_follow_algorithm_1(orc):
    prob = workloads.c2(n=127)
    out = orc.mg_solve(prob, rule="heuristic", start_level=0, max_level=6, tol=1e-10)
    assert out["status"] == "ok"
    lv, nr = out["levels"], out["norms"]
    assert lv[0] == 0
    for v in range(1, len(lv)):
        ratio = nr[v] / nr[v - 1]
        want = lv[v - 1] + (1 if ratio > 0.4 else (-1 if 0.2 < ratio < 0.4 else 0))
        assert lv[v] == min(max(want, 0), 6)
    # and it does much less work than single-grid SRJ on the same problem
    ref = orc.solve(prob, tol=1e-10)
    assert out["work"] < ref["sweeps"] / 5


def test_invalid_options(orc):
    prob = workloads.poisson([64, 63])  # cannot be coarsened
    assert orc.mg_solve(prob)["status"] == "invalid"
    prob = workloads.poisson([15, 15])
    assert orc.mg_solve(prob, pre=-1)["status"] == "invalid"
    assert orc.mg_solve(prob, rule="increasing")["status"] == "invalid"
