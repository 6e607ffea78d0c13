"""Pins of the oracle's whole solve (no GPU).

* Section 4.1 worked example (1D Poisson N = 100, b = 1, ||r|| < 1e-7):
  the level sequence climbs 0..11 and then alternates 10/11; about 1000
  iterations with the heuristic and over 3000 with the increasing rule.
* Section 3 figure on fixed schemes: M = 63 converges fastest of
  M = 35, 47, 63, 84.
* The spectral model (closed-form G_M on the DST-I eigenbasis, no sweeps)
  gives the same level sequence and cycle-end norms for constant-coefficient
  problems in 1D, 2D and 3D, including anisotropic couplings.
* Table 3 (3D Poisson, f = 1, relative residual < 1e-8): speedup over
  unweighted Jacobi within +-1 of the printed values; Jacobi's count comes from
  the closed form of its residual decay.
* Converged solutions agree with numpy.linalg.solve on tiny grids.
* Error paths: invalid arguments, non-finite input, divergence, caps.
"""
import numpy as np
import pytest

import workloads
from golden_io import keyed, rows
from spectral import dense_matrix, jacobi_sweeps_to_tol, spectral_solve


def test_worked_example_section_4_1(orc):
    g = keyed("section4_1_worked_example.txt")
    N = int(g["N"][0])
    tol = float(g["tol_abs"][0])
    climb = int(g["climb_to_level"][0])
    alt = [int(v) for v in g["alternate_levels"]]
    prob = workloads.poisson_1d(N)
    out = orc.solve(prob, tol=tol, tol_mode="absolute")
    assert out["status"] == "ok"
    lv = out["levels"].tolist()
    assert lv[:climb + 1] == list(range(climb + 1))
    tail = lv[climb + 1:]
    assert len(tail) >= 4
    assert set(tail) == set(alt)
    assert all(tail[i] != tail[i + 1] for i in range(len(tail) - 1))
    # "approximately 1000 iterations": counted per sweep as in the paper's plots
    per_sweep = orc.solve(prob, tol=tol, tol_mode="absolute", stop_per_sweep=True)
    approx = int(g["heuristic_iterations_approx"][0])
    assert abs(per_sweep["sweeps"] - approx) <= 0.1 * approx
    assert out["sweeps"] >= per_sweep["sweeps"]
    inc = orc.solve(prob, tol=tol, tol_mode="absolute", rule="increasing")
    assert inc["status"] == "ok"
    assert inc["sweeps"] > int(g["increasing_iterations_min"][0])
    assert inc["levels"].tolist() == list(range(inc["cycles"]))


def test_fig2_fixed_schemes(orc):
    r = rows("fig2_fixed_schemes.txt")
    fastest = int([x for x in r if x[0] == "fastest"][0][1])
    prob = workloads.poisson_1d(100)
    sweeps = {}
    for M, level in [(int(a), int(b)) for a, b in r if a != "fastest"]:
        assert orc.level_M(level) == M
        out = orc.solve(prob, rule="fixed", fixed_level=level, tol=1e-7, tol_mode="absolute")
        assert out["status"] == "ok"
        sweeps[M] = out["sweeps"]
    assert min(sweeps, key=sweeps.get) == fastest


SPECTRAL_CASES = [
    ("c1", lambda: workloads.c1(), 1e-10),
    ("1d_N100_b1", lambda: workloads.poisson_1d(100), 1e-10),
    ("1d_N400", lambda: workloads.poisson_1d(400, b=np.random.default_rng(3).uniform(-1, 1, (1, 1, 400)))),
    ("2d_c2_recipe_96", lambda: workloads.c2(n=96), 1e-10),
    ("2d_64x40", lambda: workloads.poisson([64, 40], b=np.random.default_rng(4).uniform(-1, 1, (1, 40, 64))), 1e-10),
    ("3d_20", lambda: workloads.poisson([20, 20, 20]), 1e-8),
    ("3d_aniso", lambda: workloads.c5_instance(3, lo=12, hi=24), 1e-8),
]


@pytest.mark.parametrize("case", range(len(SPECTRAL_CASES)))
def test_spectral_model_levels_and_norms(orc, case):
    entry = SPECTRAL_CASES[case]
    prob = entry[1]()
    tol = entry[2] if len(entry) > 2 else 1e-10
    out = orc.solve(prob, tol=tol)
    ref = spectral_solve(prob, tol=tol)
    assert out["status"] == "ok" and ref["converged"]
    np.testing.assert_array_equal(out["levels"], ref["levels"])
    assert out["sweeps"] == ref["sweeps"]
    # relative agreement of cycle-end norms, limited by round-off in the iteration
    rel = np.abs(out["norms"] - ref["norms"]) / ref["norms"][0]
    assert rel.max() < 1e-11, rel.max()


def test_spectral_model_increasing_rule(orc):
    # The increasing rule reaches levels whose round-off amplification is
    # ~1e4 (Leja order, level >= 20); compare the cycles before that.
    prob = workloads.poisson_1d(150)
    out = orc.solve(prob, rule="increasing", tol=1e-9, max_cycles=40)
    ref = spectral_solve(prob, rule="increasing", tol=1e-9)
    k = 18
    np.testing.assert_array_equal(out["levels"][:k], ref["levels"][:k])
    rel = np.abs(out["norms"][:k + 1] - ref["norms"][:k + 1]) / ref["norms"][0]
    assert rel.max() < 1e-11
    assert out["status"] == "ok"


@pytest.mark.parametrize("n", [32, 48])
def test_table3_speedup(orc, n):
    printed = {int(a): int(b) for a, b in rows("table3_speedup_3d.txt")}
    prob = workloads.poisson([n, n, n])
    srj = orc.solve(prob, tol=1e-8, stop_per_sweep=True)
    assert srj["status"] == "ok"
    jac = jacobi_sweeps_to_tol(prob, 1e-8)
    speedup = jac / srj["sweeps"]
    assert abs(speedup - printed[n]) <= 1.0, (jac, srj["sweeps"], speedup)


@pytest.mark.slow
@pytest.mark.parametrize("n", [64, 96])
def test_table3_speedup_larger(orc, n):
    test_table3_speedup(orc, n)


def test_jacobi_rule_matches_closed_form_count(orc):
    prob = workloads.poisson([10, 10, 10])
    out = orc.solve(prob, rule="jacobi", tol=1e-6, stop_per_sweep=True, max_cycles=100000)
    assert out["status"] == "ok"
    assert out["sweeps"] == jacobi_sweeps_to_tol(prob, 1e-6)


TINY = [
    lambda: workloads.poisson([40], b=np.random.default_rng(1).uniform(-1, 1, (1, 1, 40))),
    lambda: workloads.poisson([8, 8], b=np.random.default_rng(2).uniform(-1, 1, (1, 8, 8))),
    lambda: workloads.poisson([4, 4, 4], b=np.random.default_rng(3).uniform(-1, 1, (4, 4, 4))),
    lambda: workloads.anisotropic([5, 4, 4], (1.0, 0.02, 0.5), np.random.default_rng(4).uniform(-1, 1, (4, 4, 5))),
    lambda: workloads.variable_coefficient(4, seed=9, corr_len=2.0),
]


@pytest.mark.parametrize("k", range(len(TINY)))
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_dense_solve_tiny(orc, k, precision):
    prob = TINY[k]()
    A = dense_matrix(prob)
    xs = np.linalg.solve(A, prob.b.ravel())
    tol = 1e-12 if precision == "f64" else 1e-10
    out = orc.solve(prob, tol=tol, precision=precision)
    assert out["status"] == "ok"
    kappa = np.linalg.cond(A)
    err = np.linalg.norm(out["x"].ravel() - xs) / np.linalg.norm(xs)
    assert err <= 2.0 * kappa * tol
    # the reported final norm is the true residual of the returned iterate
    r = np.linalg.norm(prob.b.ravel() - A @ out["x"].ravel())
    assert abs(r - out["r_final"]) <= 1e-9 * out["r0"]


@pytest.mark.parametrize("precision", ["f32", "bf16", "f16"])
def test_refinement_follows_f64_levels(orc, precision):
    # in exact arithmetic a refinement cycle moves the error like an f64 cycle
    prob = workloads.c5_instance(1, lo=9, hi=13)
    ref = orc.solve(prob, tol=1e-8)
    out = orc.solve(prob, tol=1e-8, precision=precision)
    assert out["status"] == "ok"
    n_agree = 6 if precision == "f32" else 3
    np.testing.assert_array_equal(out["levels"][:n_agree], ref["levels"][:n_agree])
    if precision == "f32":
        assert abs(out["cycles"] - ref["cycles"]) <= 2
    rel = np.linalg.norm(out["x"] - ref["x"]) / np.linalg.norm(ref["x"])
    A = dense_matrix(prob) if prob.npoints <= 3000 else None
    bound = 1e-8 * (np.linalg.cond(A) if A is not None else 1e4)
    assert rel <= 4.0 * bound


def test_rounding_f16_matches_numpy(orc):
    rng = np.random.default_rng(0)
    v = np.concatenate([
        rng.standard_normal(4000).astype(np.float32) * np.float32(10.0) ** rng.integers(-9, 6, 4000),
        np.array([0.0, -0.0, 65504.0, 65519.0, 65520.0, 1e9, -1e9, 6.0e-8, 2.9e-8, 3.0e-8,
                  5.96e-8, 6.1e-5, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11], dtype=np.float32),
    ])
    got = orc.round_f16(v)
    with np.errstate(over="ignore"):
        ref = v.astype(np.float16).astype(np.float32)
    np.testing.assert_array_equal(got, ref)


def test_rounding_bf16_matches_torch(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    v = np.concatenate([
        rng.standard_normal(4000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 4000),
        np.array([0.0, -0.0, 3.0e38, 3.39e38, 3.4e38, 1e-40, 1e-44, 1.0 + 2.0 ** -8,
                  1.0 + 3 * 2.0 ** -8], dtype=np.float32),
    ])
    got = orc.round_bf16(v)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(got, ref)


def test_errors_and_caps(orc):
    prob = workloads.poisson_1d(30)
    assert orc.solve(prob, tol=0.0)["status"] == "invalid"
    assert orc.solve(prob, tol=1e-8, start_level=25)["status"] == "invalid"
    assert orc.solve(prob, tol=1e-8, rule="fixed", fixed_level=30)["status"] == "invalid"
    assert orc.solve(prob, tol=1e-8, precision="f32", stop_per_sweep=True)["status"] == "invalid"
    capped = orc.solve(prob, tol=1e-12, max_cycles=2)
    assert capped["status"] == "not_converged" and capped["cycles"] == 2
    assert orc.solve(prob, tol=1e-12, max_sweeps=5)["status"] == "not_converged"
    bad = workloads.poisson_1d(30)
    bad.b = bad.b.copy()
    bad.b[0, 0, 3] = np.nan
    assert orc.solve(bad, tol=1e-8)["status"] == "nonfinite"
    # D scaled down so that rho(B_J) > 1: Jacobi-type iterations diverge
    div = workloads.poisson_1d(30)
    div.dconst = 0.4 * div.dconst
    out = orc.solve(div, tol=1e-8, max_cycles=200)
    assert out["status"] in ("nonfinite", "not_converged")
    assert not out["converged"]
    # zero right-hand side with zero start: converged before any cycle
    z = workloads.poisson_1d(30, b=np.zeros((1, 1, 30)))
    zo = orc.solve(z, tol=1e-8)
    assert zo["status"] == "ok" and zo["cycles"] == 0
