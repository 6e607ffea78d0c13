"""GPU parity of batched solves (through the C ABI).

Every instance of a batch must reproduce its own single-problem oracle solve:
the same level at every cycle, the same counters, and a bit-identical
iterate (stricter than the 1e-12 relative bar: the per-point arithmetic is
the same and only the norms' summation order differs).  Batches mix grid sizes, 1D,
2D and 3D instances, and every batch plan (tile shape, sweeps per step,
graph capture or direct launches) must give identical results.
"""
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


def mixed_batch():
    probs = [workloads.c4_instance(i, lo=24, hi=90) for i in range(6)]
    probs += [workloads.c5_instance(i, lo=8, hi=18) for i in range(4)]
    probs.append(workloads.c1(N=100))
    probs.append(workloads.poisson([37, 5], b=np.random.default_rng(3).uniform(-1, 1, (1, 5, 37))))
    return probs


def _check(orc, probs, out, kw):
    for p, inst, x in zip(probs, out["instances"], out["xs"]):
        ref = orc.solve(p, **kw)
        assert inst["converged"] == (ref["status"] == "ok"), p.name
        np.testing.assert_array_equal(inst["levels"], ref["levels"], err_msg=p.name)
        assert inst["sweeps"] == ref["sweeps"] and inst["cycles"] == ref["cycles"], p.name
        got = x.cpu().numpy()
        if np.all(np.isfinite(ref["x"])):
            assert np.array_equal(got, ref["x"]), (p.name, np.max(np.abs(got - ref["x"])))
        assert abs(inst["r_final"] - ref["r_final"]) <= 1e-12 * max(ref["r0"], 1e-300) + \
            1e-12 * abs(ref["r_final"]), p.name


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-10), ("bf16", 1e-8),
                                           ("f16", 1e-8)])
def test_batch_matches_oracle(torch_cuda, orc, precision, tol):
    from paper_2011_06636_amd.solver import BatchSolver
    probs = mixed_batch()
    if precision in ("bf16", "f16"):
        probs = [p for p in probs if p.ndim == 3]  # 16-bit storage: the 3D boxes
    bs = BatchSolver(probs)
    kw = dict(tol=tol, precision=precision, max_cycles=200)
    out = bs.solve(**kw)
    _check(orc, probs, out, kw)
    bs.close()


def test_batch_plans_identical(torch_cuda, orc):
    from paper_2011_06636_amd.solver import BatchSolver
    probs = mixed_batch()
    bs = BatchSolver(probs)
    kw = dict(tol=1e-10, precision="f32", max_cycles=200)
    base = None
    for plan in [(24, 4, 16, True), (16, 2, 3, True), (32, 6, 7, True), (48, 8, 16, True),
                 (24, 1, 5, False), (32, 4, 1, False), (8, 8, 16, True, 8), (8, 3, 5, True, 8),
                 (12, 8, 4, False, 8), (16, 5, 16, True, 4)]:
        assert bs.set_plan(*plan) == 0, plan
        out = bs.solve(**kw)
        got = [x.cpu().numpy() for x in out["xs"]]
        lv = [i["levels"] for i in out["instances"]]
        if base is None:
            base = (got, lv)
            _check(orc, probs, out, kw)
        else:
            for a, b in zip(got, base[0]):
                assert np.array_equal(a, b), plan
            for a, b in zip(lv, base[1]):
                assert np.array_equal(a, b), plan
    bs.close()


TILES3D = [(4, 8), (2, 16), (4, 16), (8, 8), (8, 16)]
PLANS3D = [t + (s,) for s in (2, 1) for t in TILES3D]


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("bf16", 1e-8), ("f32", 1e-10)])
def test_batch_3d_tiles_identical(torch_cuda, orc, precision, tol):
    # every plane tile of the 3D instances, with one or two sweeps per step,
    # gives the same bits: boxes wider than one 60-column tile, ragged in rows
    # and planes, cycles of odd and even length
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import BatchSolver
    probs = [workloads.c5_instance(i, lo=20, hi=70) for i in range(5)]
    assert max(p.n[0] for p in probs) > 62
    bs = BatchSolver(probs)
    assert bs.get_plan3d() == (4, 8, 2)
    kw = dict(tol=tol, precision=precision, max_cycles=200)
    base = None
    for tile in PLANS3D:
        bs.set_plan3d(*tile)
        assert bs.get_plan3d() == tile
        out = bs.solve(**kw)
        got = [x.cpu().numpy() for x in out["xs"]]
        if base is None:
            base = got
            _check(orc, probs, out, kw)
        else:
            for a, b in zip(got, base):
                assert np.array_equal(a, b), tile
    for bad in ((3, 8), (4, 12), (0, 0)):
        with pytest.raises(abi.SrjError) as e:
            bs.set_plan3d(*bad)
        assert e.value.status == abi.SRJ_ERR_UNSUPPORTED
    for sweeps in (0, 3):
        with pytest.raises(abi.SrjError) as e:
            bs.set_plan3d(4, 8, sweeps)
        assert e.value.status == abi.SRJ_ERR_INVALID
    bs.close()


def test_batch_caps_and_errors(torch_cuda, orc):
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import BatchSolver
    probs = [workloads.c4_instance(i, lo=30, hi=60) for i in range(3)]
    bs = BatchSolver(probs)
    out = bs.solve(tol=1e-10, max_cycles=3)
    assert out["status"] == "not_converged"
    assert all(i["cycles"] == 3 and not i["converged"] for i in out["instances"])
    bs.close()
    # a per-point diagonal is not taken by batches
    vc = workloads.variable_coefficient(6, seed=1)
    with pytest.raises(abi.SrjError):
        BatchSolver([vc])


def test_batch_autotune_keeps_results(torch_cuda, orc):
    from paper_2011_06636_amd.solver import BatchSolver
    probs = mixed_batch()
    bs = BatchSolver(probs)
    kw = dict(tol=1e-10, precision="f32", max_cycles=200)
    ref = bs.solve(**kw)
    ref_x = [x.cpu().numpy() for x in ref["xs"]]
    us = bs.autotune("f32", sweeps=24)
    assert us > 0
    rows, T, waves, _, _ = bs.get_plan()
    assert (rows, waves) in ((16, 1), (24, 1), (32, 1), (48, 1), (8, 8), (12, 8), (16, 4)) and T >= 1
    assert bs.get_plan3d() in PLANS3D
    out = bs.solve(**kw)
    for a, b in zip(out["xs"], ref_x):
        assert np.array_equal(a.cpu().numpy(), b)
    bs.close()
