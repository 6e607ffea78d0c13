"""Section 3 post-processing of the selector's training data (CPU reference).

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark baseline); the
library never imports it.

Written from the paper's description (Islam & Wang, arXiv 2011.06636,
section 3): the recorded tuples (state = current level and previous residual
ratio; action; average convergence rate of the action's cycle,
-log(r_after / r_before) / M, the paper's Eq. for the average convergence
rate) are grouped by level, sorted by the previous residual ratio and cut
into clusters of N_set tuples.  In each cluster, the mean rate of every
action gets a 95 % confidence interval; the action with the highest mean is
the cluster's best only if its interval does not overlap the other actions'
intervals.  The rule of Algorithm 1 (ratio above an upper threshold: raise
the level; between the two thresholds: lower it; otherwise keep it) is then
fitted to the clusters that have a best action.

Readings where the paper is silent: the interval is the normal one, mean
+- z s / sqrt(n) with the sample standard deviation s and z = 1.96; a
trailing cluster with fewer than N_set tuples is dropped; ties in the ratio
keep the input order; "does not overlap" is strict; thresholds sit halfway
between the neighbouring clusters' mean ratios, and the first split (in
ascending order) with the most agreeing clusters wins.
"""
from __future__ import annotations

import math

import numpy as np

NONE = 2  # no action is confidently best


def rates(samples: np.ndarray) -> np.ndarray:
    """Average convergence rate of each tuple: -log(r_after / r_before) / M."""
    return np.array([-math.log(s["r_after"] / s["r_before"]) / s["M"] for s in samples],
                    dtype=np.float64)


def usable(samples: np.ndarray) -> np.ndarray:
    """Tuples of branches that ran (M > 0) with positive finite norms, flattened."""
    s = samples.reshape(-1)
    keep = (s["M"] > 0) & (s["r_before"] > 0) & (s["r_after"] > 0) & np.isfinite(s["prev_ratio"])
    keep &= (s["level"] >= 0) & (s["level"] < 25)
    return s[keep]


def cluster_samples(samples: np.ndarray, n_set: int = 10000, z: float = 1.96) -> list:
    """Clusters in level order, then ratio order; one dict per cluster."""
    s = usable(samples)
    r = rates(s) if len(s) else np.zeros(0)
    ok = np.isfinite(r)
    s, r = s[ok], r[ok]
    out = []
    for level in range(25):
        idx = np.nonzero(s["level"] == level)[0]
        idx = idx[np.argsort(s["prev_ratio"][idx], kind="stable")]
        for c0 in range(0, len(idx) - n_set + 1, n_set):
            cl = idx[c0:c0 + n_set]
            ratio_sum = 0.0
            for i in cl:
                ratio_sum = ratio_sum + float(s["prev_ratio"][i])
            n = [0, 0, 0]
            mean = [0.0, 0.0, 0.0]
            half = [math.inf, math.inf, math.inf]
            for j, act in enumerate((1, 0, -1)):
                vals = [float(r[i]) for i in cl if s["action"][i] == act]
                n[j] = len(vals)
                if not vals:
                    continue
                tot = 0.0
                for v in vals:
                    tot = tot + v
                mean[j] = tot / len(vals)
                if len(vals) >= 2:
                    ss = 0.0
                    for v in vals:
                        ss = ss + (v - mean[j]) * (v - mean[j])
                    half[j] = z * math.sqrt(ss / (len(vals) - 1) / len(vals))
            seen = [j for j in range(3) if n[j] > 0]
            best = None
            for j in seen:
                if best is None or mean[j] > mean[best]:
                    best = j
            decided = best is not None and n[best] >= 2
            if decided:
                for j in seen:
                    if j != best and not (mean[best] - half[best] > mean[j] + half[j]):
                        decided = False
            out.append({"level": level, "count": n_set, "mean_ratio": ratio_sum / n_set,
                        "best": (1 - best) if decided else NONE, "n": n, "mean_rate": mean,
                        "half_width": half})
    return out


def rule_action(ratio: float, t_low: float, t_high: float) -> int:
    """Algorithm 1 with thresholds t_low < t_high."""
    if ratio > t_high:
        return 1
    if t_low < ratio < t_high:
        return -1
    return 0


def fit_rule(clusters: list) -> tuple:
    """(t_low, t_high, agree, decided) of the best-agreeing thresholds."""
    d = [c for c in clusters if c["best"] in (-1, 0, 1)]
    order = np.argsort([c["mean_ratio"] for c in d], kind="stable")
    d = [d[i] for i in order]
    m = len(d)
    if m == 0:
        return 0.0, 0.0, 0, 0

    def cut(i):
        if i <= 0:
            return 0.0
        if i >= m:
            return d[m - 1]["mean_ratio"]
        return 0.5 * (d[i - 1]["mean_ratio"] + d[i]["mean_ratio"])

    best = (-1, 0, 0)
    for i in range(m + 1):
        for j in range(i, m + 1):
            agree = sum(1 for c in d[:i] if c["best"] == 0) \
                + sum(1 for c in d[i:j] if c["best"] == -1) \
                + sum(1 for c in d[j:] if c["best"] == 1)
            if agree > best[0]:
                best = (agree, i, j)
    return cut(best[1]), cut(best[2]), best[0], m
