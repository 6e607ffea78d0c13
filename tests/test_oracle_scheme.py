"""Pins of the oracle's scheme family against the paper (no GPU).

* Table 2: factor values (8 significant figures) and their printed order.
* Table 1: c1 and l_max of the amplification polynomials.
* Appendix B: level -> M.
* Appendix A / Eq. (13): prod_j (1 - w_j + w_j l) equals T_M(f(l)) / 3 at
  every level, with T_M from numpy's Chebyshev series (a library routine).
* Eq. (15): every factor is 1 / (1 - root of G_M).
"""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from golden_io import rows
from spectral import G_closed, chebyshev_T, lstar

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def G_product(w, lam):
    out = np.ones_like(lam)
    for wi in w:
        out = out * ((1.0 - wi) + wi * lam)
    return out


def test_appendix_b_levels(orc):
    for level, M in rows("appendixB_levels.txt"):
        assert orc.level_M(int(level)) == int(M)
    assert orc.level_M(25) == -1 and orc.level_M(-1) == -1


def test_table2_values_and_order(orc):
    for r in rows("table2_scheme_factors.txt"):
        level, M = int(r[0]), int(r[1])
        printed = np.array([float(v) for v in r[2:]])
        w = orc.scheme(level)
        assert len(w) == M == len(printed)
        # values printed to 8 significant figures; order is the printed order
        np.testing.assert_allclose(w, printed, rtol=1.2e-8, atol=0)


def test_table2_natural_roots_give_same_set(orc):
    for r in rows("table2_scheme_factors.txt"):
        M = int(r[1])
        printed = sorted(float(v) for v in r[2:])
        nat = sorted(orc.omega_natural(M))
        np.testing.assert_allclose(nat, printed, rtol=1.2e-8)


def test_lstar_solves_T_equals_3():
    # T_M(l*) = 3, checked with numpy's Chebyshev evaluation
    for M in (1, 2, 3, 5, 7, 10, 47, 63):
        coef = np.zeros(M + 1)
        coef[M] = 1.0
        assert abs(C.chebval(lstar(M), coef) - 3.0) < 1e-11 * M * M


def test_closed_form_T_matches_numpy():
    x = np.linspace(-1.3, 1.3, 53)
    for M in (1, 2, 3, 5, 7, 14, 35):
        coef = np.zeros(M + 1)
        coef[M] = 1.0
        np.testing.assert_allclose(chebyshev_T(M, x), C.chebval(x, coef), rtol=1e-9, atol=1e-9)


def test_table1_coefficients(orc):
    # leading coefficient of G_M is prod(w) = 2^(M-1) c1^M / 3  =>  c1
    for M_s, c1_s, c0_s, lmax_s in rows("table1_amplification.txt"):
        M = int(M_s)
        level = [int(r[0]) for r in rows("appendixB_levels.txt") if int(r[1]) == M][0]
        w = orc.scheme(level)
        c1 = (3.0 * np.prod(w) / 2.0 ** (M - 1)) ** (1.0 / M)
        assert abs(c1 - float(c1_s)) < 6e-5
        # c0 = c1 - 1 (f(-1) = -1 in Appendix A)
        assert abs((c1 - 1.0) - float(c0_s)) < 6e-5
        # l_max: largest l in (-1, 1) with G(l) <= 1/3, found by bisection on the product
        lo, hi = float(lmax_s) - 0.01, min(float(lmax_s) + 0.01, 0.999999)
        if M == 1:
            lo, hi = -0.5, 0.5
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if G_product(w, np.array([mid]))[0] <= 1.0 / 3.0:
                lo = mid
            else:
                hi = mid
        assert abs(lo - float(lmax_s)) < 6e-5


@pytest.mark.parametrize("level", range(25))
def test_product_equals_closed_form(orc, level):
    w = orc.scheme(level)
    M = len(w)
    lam = np.linspace(-1.0, 1.0, 401)
    gp = G_product(w, lam)
    gc = G_closed(M, lam)
    np.testing.assert_allclose(gp, gc, rtol=0, atol=2e-11 * max(1.0, M / 10))
    # G(1) = 1, |G(-1)| = 1/3, |G| <= 1/3 on [-1, l_max]
    assert abs(G_product(w, np.array([1.0]))[0] - 1.0) < 1e-12 * M
    assert abs(abs(G_product(w, np.array([-1.0]))[0]) - 1.0 / 3.0) < 1e-11 * M
    ls = lstar(M)
    lmax = (2.0 - (ls - 1.0)) / (ls + 1.0)  # f(l_max) = 1
    lam2 = np.linspace(-1.0, lmax, 2001)
    assert np.max(np.abs(G_product(w, lam2))) <= 1.0 / 3.0 + 1e-10 * M


@pytest.mark.parametrize("level", [0, 3, 9, 14, 20, 24])
def test_factors_are_reciprocal_roots(orc, level):
    # Eq. (15): omega_j = 1 / (1 - l_j) with G_M(l_j) = 0
    w = orc.scheme(level)
    M = len(w)
    roots = 1.0 - 1.0 / w
    vals = G_closed(M, roots)
    assert np.max(np.abs(vals)) < 1e-9 * M
    assert len(set(np.round(w, 12))) == M  # M distinct factors


@pytest.mark.parametrize("level", range(25))
def test_order_is_permutation_largest_first(orc, level):
    M = orc.level_M(level)
    w = orc.omega_natural(M)
    order = orc.leja_order(M, w)
    assert sorted(order.tolist()) == list(range(M))
    assert order[0] == int(np.argmax(w))
    np.testing.assert_array_equal(orc.scheme(level), w[order])


def test_leja_property_small(orc):
    # every chosen root maximises the product of distances to those before it
    for M in (3, 5, 7, 10, 14):
        w = orc.omega_natural(M)
        p = 1.0 - 1.0 / w
        order = orc.leja_order(M, w).tolist()
        for s in range(1, M):
            chosen = order[:s]
            rest = [j for j in range(M) if j not in chosen]
            score = {j: sum(math.log(abs(p[j] - p[k])) for k in chosen) for j in rest}
            best = max(score.values())
            assert score[order[s]] >= best - 1e-12 * abs(best) - 1e-12
