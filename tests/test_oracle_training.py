"""Pins of the CPU reference for the selector's training data (section 3).

* Every branch's residual norm follows the DST spectral model (Eq. (12) with
  the Appendix A closed form of G_M), which needs no sweeps at all.
* Special draws reduce the random walk to textbook rules: always "up" is the
  increasing rule, always "same" at level 0 is weighted Jacobi (w = 2/3).
* Clustering and the rule fit are checked on hand-made data with known
  answers, and the library's native post-processing (host code, no GPU)
  against the reference.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import training
from spectral import G_closed, appendix_b_M, dst, mu_grid

TOL = 1e-8  # the paper's stopping norm for the data collection


def _norm(v):
    return float(np.sqrt(np.sum(v * v)))


def _available(level, max_level=24):
    return [a for a in (1, 0, -1) if (a != 1 or level + 1 <= max_level) and (a != -1 or level >= 1)]


@pytest.mark.parametrize("N", [10, 20, 50])
def test_branches_follow_spectral_model(N):
    prob = workloads.poisson_1d(N, b=np.ones(N))
    trials, max_steps = 6, 80
    u = workloads.training_draws(trials, max_steps, seed=N)
    out = oracle.collect(prob, u, tol=TOL)
    Ms = appendix_b_M()
    lam = 1.0 - mu_grid(prob)
    for t in range(trials):
        rhat = dst(prob.b, 1)
        r0 = _norm(rhat)
        rhat = rhat * G_closed(1, lam)  # the level-0 start cycle
        rcur, level = _norm(rhat), 0
        rho = rcur / r0
        steps = int(out["steps"][t])
        assert steps >= 1
        for s in range(steps):
            avail = _available(level)
            chosen = avail[min(int(u[t, s] * len(avail)), len(avail) - 1)]
            for j, a in enumerate((1, 0, -1)):
                rec = out["samples"][t, s, j]
                assert (rec["trial"], rec["step"], rec["level"], rec["action"]) == (t, s, level, a)
                assert rec["chosen"] == (a == chosen)
                assert abs(rec["prev_ratio"] - rho) <= 1e-6
                assert abs(rec["r_before"] - rcur) <= 1e-8 * rcur + 1e-11
                if a in avail:
                    M = Ms[level + a]
                    assert rec["M"] == M
                    ra = _norm(rhat * G_closed(M, lam))
                    assert abs(rec["r_after"] - ra) <= 1e-8 * ra + 1e-11, (t, s, a)
                else:
                    assert rec["M"] == 0 and rec["r_after"] == 0.0
            rhat = rhat * G_closed(Ms[level + chosen], lam)
            rnew = _norm(rhat)
            rho, rcur, level = rnew / rcur, rnew, level + chosen
            if s + 1 < steps:
                assert rcur >= TOL * (1 - 1e-6)
        assert rcur < TOL * (1 + 1e-6) or steps == max_steps
        # slots after the last step are untouched
        assert np.all(out["samples"][t, steps:]["M"] == 0)


def test_always_up_is_the_increasing_rule():
    prob = workloads.poisson_1d(20, b=np.ones(20))
    u = np.zeros((1, 60))
    out = oracle.collect(prob, u, tol=TOL)
    ref = oracle.solve(prob, rule="increasing", tol=TOL, tol_mode="absolute", max_cycles=60)
    steps = int(out["steps"][0])
    assert steps == ref["cycles"] - 1
    taken = out["samples"][0, :steps]
    ch = taken[taken["chosen"] == 1]
    assert np.array_equal(ch["action"], np.ones(steps, dtype=np.int32))
    assert np.array_equal(ch["level"], ref["levels"][1:] - 1)
    # bit-identical: same sweeps, same sequential sums
    assert np.array_equal(ch["r_after"], ref["norms"][2:])
    assert np.array_equal(ch["r_before"], ref["norms"][1:-1])


def test_always_same_at_level_0_is_weighted_jacobi():
    prob = workloads.poisson_1d(8, b=np.ones(8))
    u = np.full((1, 2000), 0.999)  # two actions at level 0 (up, same): the second
    out = oracle.collect(prob, u, tol=TOL)
    ref = oracle.solve(prob, rule="fixed", fixed_level=0, tol=TOL, tol_mode="absolute",
                       max_cycles=3000)
    steps = int(out["steps"][0])
    assert steps == ref["cycles"] - 1
    ch = out["samples"][0, :steps]
    ch = ch[ch["chosen"] == 1]
    assert np.all(ch["action"] == 0) and np.all(ch["level"] == 0)
    assert np.array_equal(ch["r_after"], ref["norms"][2:])
    # the down branch never exists at level 0
    assert np.all(out["samples"][0, :steps, 2]["M"] == 0)


def test_top_level_has_no_up_branch():
    prob = workloads.poisson_1d(30, b=np.ones(30))
    u = np.zeros((1, 40))  # always the first available action: up, then same at the top
    out = oracle.collect(prob, u, tol=TOL, max_level=2)
    s = out["samples"][0, :int(out["steps"][0])]
    assert s[0, 0]["level"] == 0 and s[2, 0]["level"] == 2
    top = s[s[:, 1]["level"] == 2]
    assert len(top) > 0
    assert np.all(top[:, 0]["M"] == 0)           # no level 3
    assert np.all(top[:, 1]["chosen"] == 1)      # first available is "same"
    assert np.all(top[:, 2]["M"] == appendix_b_M()[1])


# ---------------------------------------------------------------------------
# Clustering and the rule fit
# ---------------------------------------------------------------------------

def _sample(level, ratio, action, rate, M=4):
    rec = np.zeros((), dtype=oracle.SAMPLE_DTYPE)
    rec["level"], rec["action"], rec["M"] = level, action, M
    rec["prev_ratio"], rec["r_before"] = ratio, 1.0
    rec["r_after"] = math.exp(-rate * M)
    return rec


def test_clusters_by_hand():
    # level 3: eight tuples, n_set = 4 -> two clusters after sorting by ratio;
    # level 5: three tuples -> no whole cluster
    recs = [_sample(3, 0.9, 1, 0.50), _sample(3, 0.1, 0, 0.30), _sample(3, 0.8, 1, 0.52),
            _sample(3, 0.2, 0, 0.31), _sample(3, 0.7, 0, 0.10), _sample(3, 0.3, -1, 0.05),
            _sample(3, 0.6, 0, 0.12), _sample(3, 0.4, -1, 0.06),
            _sample(5, 0.5, 1, 1.0), _sample(5, 0.5, 0, 1.0), _sample(5, 0.5, -1, 1.0)]
    s = np.array(recs, dtype=oracle.SAMPLE_DTYPE)
    cl = training.cluster_samples(s, n_set=4, z=1.96)
    assert [c["level"] for c in cl] == [3, 3]
    lo, hi = cl
    # the lower cluster holds ratios 0.1, 0.2, 0.3, 0.4
    assert lo["mean_ratio"] == pytest.approx(0.25, abs=1e-15)
    assert lo["n"] == [0, 2, 2]
    rate = lambda r, M=4: -math.log(math.exp(-r * M)) / M  # noqa: E731
    assert lo["mean_rate"][1] == pytest.approx((rate(0.30) + rate(0.31)) / 2, rel=1e-15)
    assert lo["mean_rate"][2] == pytest.approx((rate(0.05) + rate(0.06)) / 2, rel=1e-15)
    sd = np.std([rate(0.30), rate(0.31)], ddof=1)
    assert lo["half_width"][1] == pytest.approx(1.96 * sd / math.sqrt(2), rel=1e-12)
    assert lo["best"] == 0  # same level: 0.305 +- 0.0098 clear of 0.055 +- 0.0098
    # the upper cluster: up (0.50, 0.52) against same (0.10, 0.12)
    assert hi["mean_ratio"] == pytest.approx(0.75, abs=1e-15)
    assert hi["n"] == [2, 2, 0] and hi["best"] == 1


def test_overlapping_intervals_leave_the_cluster_undecided():
    rng = np.random.default_rng(3)
    recs = []
    for i in range(400):
        a = (1, 0, -1)[i % 3]
        recs.append(_sample(2, 0.5 + 1e-4 * i, a, 0.2 + 0.05 * rng.standard_normal()))
    cl = training.cluster_samples(np.array(recs, dtype=oracle.SAMPLE_DTYPE), n_set=400)
    assert len(cl) == 1 and cl[0]["best"] == training.NONE
    # the same data with the down action shifted clear of the others
    for r in recs:
        if r["action"] == -1:
            r["r_after"] = r["r_after"] * math.exp(-4 * 0.5)
    cl = training.cluster_samples(np.array(recs, dtype=oracle.SAMPLE_DTYPE), n_set=400)
    assert cl[0]["best"] == -1


def test_rule_fit_recovers_thresholds():
    ratios = np.arange(0.05, 1.0, 0.1)
    clusters = [{"level": 1, "mean_ratio": float(r),
                 "best": training.rule_action(float(r), 0.2, 0.4)} for r in ratios]
    clusters.append({"level": 1, "mean_ratio": 0.5, "best": training.NONE})
    t_low, t_high, agree, decided = training.fit_rule(clusters)
    assert decided == len(ratios) and agree == len(ratios)
    assert t_low == pytest.approx(0.2, abs=1e-12) and t_high == pytest.approx(0.4, abs=1e-12)
    # one disagreeing cluster inside the "up" region costs one agreement, not
    # the thresholds
    clusters[7]["best"] = 0
    t_low2, t_high2, agree2, _ = training.fit_rule(clusters)
    assert agree2 == len(ratios) - 1
    assert (t_low2, t_high2) == pytest.approx((0.2, 0.4), abs=1e-12)


def test_native_postprocessing_matches_reference():
    from paper_2011_06636_amd import abi
    prob = workloads.poisson_1d(30, b=np.ones(30))
    u = workloads.training_draws(40, 60, seed=11)
    out = oracle.collect(prob, u, tol=TOL)
    flat = np.concatenate([out["samples"][t, :out["steps"][t]].reshape(-1)
                           for t in range(len(u))])
    ref = training.cluster_samples(flat, n_set=50)
    got = abi.srj_cluster_samples(flat.astype(abi.SAMPLE_DTYPE), n_set=50, z=1.96)
    assert len(got) == len(ref) > 5
    for g, r in zip(got, ref):
        assert g["level"] == r["level"] and g["count"] == r["count"]
        assert g["mean_ratio"] == r["mean_ratio"] and g["best"] == r["best"]
        assert list(g["n"]) == r["n"]
        for j in range(3):
            if r["n"][j]:
                assert g["mean_rate"][j] == r["mean_rate"][j]
            assert g["half_width"][j] == r["half_width"][j]
    assert abi.srj_fit_rule(got) == training.fit_rule(ref)
