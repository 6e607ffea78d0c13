"""GPU parity of the multigrid V-cycle with SRJ smoothing (srj_mg_*,
through the C ABI) against the oracle's (oracle/srj_mg.c).

Transfers and smoothing evaluate the oracle's fixed-order expressions, so the
iterate must be bit-identical, the smoothing scheme of every V-cycle the
same, the counters (fine sweeps, coarsest-solve sweeps, work) equal, and the
V-cycle norms equal to 1e-12 (sums in another order; on grids of more than
about 9000 points to the error bound of the oracle's sequential sum).  Grids: 1D, 2D with
unequal sides that stop coarsening at an even size, thin 2D and 3D grids
whose coarse levels have one row, 3D, a hierarchy cut by max_levels, fixed
and heuristic smoothing schemes, pre/post counts, and the benchmark's full
2047^2 and 255^3 problems."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(list(n) + [1] * (3 - len(n))))
    return workloads.poisson(n, b=rng.uniform(-1, 1, shape))


CASES = [
    ("1d_255", lambda: workloads.c1(), dict()),
    ("2d_c2_recipe_127", lambda: workloads.c2(n=127), dict()),
    ("2d_95x47_fixed2", lambda: _rand([95, 47], 1), dict(rule="fixed", start_level=2)),
    ("2d_63_pre2_post0", lambda: _rand([63, 63], 2), dict(pre=2, post=0, max_level=5)),
    # two post-smoothing cycles: the interpolating pass, then a plain cycle,
    # and the closing norm in a pass of its own
    ("2d_255_pre1_post2", lambda: _rand([255, 255], 6), dict(pre=1, post=2)),
    ("2d_255_3levels", lambda: _rand([255, 255], 3), dict(max_levels=3, coarse_tol=1e-6)),
    ("3d_31", lambda: _rand([31, 31, 31], 4), dict()),
    ("3d_aniso_63x31x15", lambda: workloads.anisotropic([63, 31, 15], [1.0, 0.3, 0.05],
                                                         np.random.default_rng(5).uniform(-1, 1, (15, 31, 63))),
     dict(rule="fixed", start_level=3)),
    # rows of at least 64 per plane are dealt to the XCDs in bands (3D)
    ("3d_127x127x7", lambda: _rand([127, 127, 7], 9), dict()),
    # thin grids: strips and chunks mostly outside the grid in the fused 2D
    # passes, coarse grids of one row or column, a tail whose coarsest grid
    # has 1023 points, 3D levels of one or three rows and planes
    ("2d_255x7", lambda: _rand([255, 7], 10), dict()),
    ("2d_7x255", lambda: _rand([7, 255], 11), dict()),
    ("2d_2047x3", lambda: _rand([2047, 3], 12), dict()),
    ("3d_1023x3x3", lambda: _rand([1023, 3, 3], 13), dict()),
    ("3d_3x1023x3", lambda: _rand([3, 1023, 3], 14), dict()),
    # the benchmark's grids, as bench.py solves them (graph replays, the
    # one-workgroup tail, the single-wave coarsest solve)
    ("2d_c2_recipe_2047_full", lambda: workloads.c2(n=2047), dict(tol=2e-9)),
    ("3d_255_full", lambda: workloads.poisson([255, 255, 255], b=np.random.default_rng(0).uniform(-1, 1, (255, 255, 255))),
     dict()),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_mg_matches_oracle(torch_cuda, orc, case):
    from paper_2011_06636_amd.solver import MgSolver
    name, make, kw = CASES[case]
    prob = make()
    print(f"mg case {name}: n = {prob.n}", flush=True)
    kw = dict(tol=1e-10) | kw
    ref = orc.mg_solve(prob, **kw)
    s = MgSolver(prob)
    out = s.solve(**kw)
    assert out["status"] == ref["status"], (name, out["status"], ref["status"])
    assert out["levels_grid"] == ref["levels_grid"]
    np.testing.assert_array_equal(out["levels"], ref["levels"])
    assert out["sweeps"] == ref["sweeps"] and out["coarse_sweeps"] == ref["coarse_sweeps"]
    assert out["work"] == ref["work"]
    # the oracle adds the squares in point order, whose relative error is
    # bounded by (n - 1) 2^-53 for n positive terms (the GPU's tree sum by
    # far less); the bar is 1e-12 wherever that bound is below it
    rtol = max(1e-12, prob.npoints * 2.0 ** -53)
    np.testing.assert_allclose(out["norms"], ref["norms"], rtol=rtol, atol=0)
    got = out["x"].cpu().numpy()
    assert np.array_equal(got, ref["x"]), (name, np.max(np.abs(got - ref["x"])))
    s.close()


def test_mg_resumes_from_initial_guess(torch_cuda, orc):
    from paper_2011_06636_amd.solver import MgSolver
    prob = _rand([63, 31], 7)
    x0 = np.random.default_rng(8).uniform(-1, 1, prob.shape)
    ref = orc.mg_solve(prob, x0, tol=1e-9)
    s = MgSolver(prob)
    out = s.solve(s.to_device(x0), tol=1e-9)
    assert np.array_equal(out["x"].cpu().numpy(), ref["x"])
    np.testing.assert_array_equal(out["levels"], ref["levels"])
    s.close()


def test_mg_replays_match_across_solves_options_and_streams(torch_cuda, orc):
    # V-cycles are replayed from graphs cached per smoothing level, starting
    # buffer and options: a second solve on the same solver, a solve with
    # other options, one into another x, and one on a caller's stream must
    # each give the oracle's bits
    import torch
    from paper_2011_06636_amd.solver import MgSolver
    prob = workloads.c2(n=127)
    runs = [dict(tol=1e-10), dict(tol=1e-10), dict(tol=1e-10, pre=2, post=1),
            dict(tol=1e-8, rule="fixed", start_level=1), dict(tol=1e-10)]
    s = MgSolver(prob)
    for i, kw in enumerate(runs):
        ref = orc.mg_solve(prob, **kw)
        x = s.zeros() if i != 4 else s.zeros().clone()
        out = s.solve(x, **kw)
        print(f"mg replay run {i}: {kw}", flush=True)
        np.testing.assert_array_equal(out["levels"], ref["levels"])
        assert out["work"] == ref["work"] and out["coarse_sweeps"] == ref["coarse_sweeps"]
        assert np.array_equal(out["x"].cpu().numpy(), ref["x"]), i
    s.close()
    st = torch.cuda.Stream()
    s = MgSolver(prob, stream=st)
    ref = orc.mg_solve(prob, tol=1e-10)
    for _ in range(2):
        with torch.cuda.stream(st):
            out = s.solve(tol=1e-10)
        st.synchronize()
        assert np.array_equal(out["x"].cpu().numpy(), ref["x"])
        np.testing.assert_array_equal(out["levels"], ref["levels"])
    s.close()


def test_mg_graph_cache_stays_bounded(torch_cuda, orc):
    # every new x gets graphs of its own; past the cache's bound the oldest
    # are dropped, and solves into old and new tensors keep the oracle's bits
    from paper_2011_06636_amd.solver import MgSolver
    prob = workloads.c2(n=127)
    ref = orc.mg_solve(prob, tol=1e-10)
    s = MgSolver(prob)
    xs = [s.zeros() for _ in range(40)]
    for i in list(range(40)) + [0, 1, 39]:
        xs[i].zero_()
        out = s.solve(xs[i], tol=1e-10)
        assert np.array_equal(out["x"].cpu().numpy(), ref["x"]), i
        assert out["work"] == ref["work"], i
    print("mg graph cache: 43 solves into 40 tensors", flush=True)
    s.close()


def test_mg_rejects_what_it_cannot_coarsen(torch_cuda):
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import MgSolver
    with pytest.raises(abi.SrjError) as e:
        MgSolver(workloads.poisson([64, 63]))
    assert e.value.status == abi.SRJ_ERR_UNSUPPORTED
    with pytest.raises(abi.SrjError) as e:
        MgSolver(workloads.variable_coefficient_2d(31, 31, seed=1))
    assert e.value.status == abi.SRJ_ERR_UNSUPPORTED
    s = MgSolver(workloads.poisson([31, 31]))
    for bad in (dict(pre=-1), dict(max_levels=1), dict(rule="increasing"), dict(tol=0.0),
                dict(start_level=5, max_level=3)):
        with pytest.raises(abi.SrjError) as e:
            s.solve(**bad)
        assert e.value.status == abi.SRJ_ERR_INVALID, bad
    s.close()
