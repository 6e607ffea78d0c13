"""Full-size batched workloads, in the launch configuration that bench.py
times (plans picked by the batch autotuner): 512 2D Poisson squares solved
binary32-refined to 1e-10, and 128 3D anisotropic boxes solved in binary64
and bfloat16-refined to 1e-8.

Every instance must converge.  The oracle solves a sample of the instances
one by one (the two smallest, the ones at a quarter, a half and three
quarters of the size order, and the largest): each must show
the oracle's level at every cycle, its counters and a bit-identical iterate.
Smaller mixed batches, every plan and every precision are checked
instance by instance in test_gpu_batch.py.
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


def _sample(probs):
    order = sorted(range(len(probs)), key=lambda i: (probs[i].npoints, i))
    n = len(order)
    picks = [order[0], order[1], order[n // 4], order[n // 2], order[3 * n // 4], order[-1]]
    return list(dict.fromkeys(picks))


def _run(orc, probs, precision, tol):
    from paper_2011_06636_amd.solver import BatchSolver
    bs = BatchSolver(probs)
    bs.autotune(precision, sweeps=48)
    kw = dict(tol=tol, precision=precision, max_cycles=300)
    out = bs.solve(**kw)
    print(f"full batch {precision}: {len(probs)} instances, plan "
          f"{bs.get_plan() if probs[0].ndim == 2 else bs.get_plan3d()}", flush=True)
    assert all(inst["converged"] for inst in out["instances"])
    for i in _sample(probs):
        p, inst = probs[i], out["instances"][i]
        ref = orc.solve(p, **kw)
        assert ref["status"] == "ok", i
        np.testing.assert_array_equal(inst["levels"], ref["levels"], err_msg=str(i))
        assert inst["sweeps"] == ref["sweeps"] and inst["cycles"] == ref["cycles"], i
        assert np.array_equal(out["xs"][i].cpu().numpy(), ref["x"]), i
        assert abs(inst["r_final"] - ref["r_final"]) <= 1e-12 * ref["r0"], i
    bs.close()


def test_full_512_squares_f32_refined(torch_cuda, orc):
    _run(orc, workloads.c4(), "f32", 1e-10)


@pytest.mark.parametrize("precision", ["f64", "bf16"])
def test_full_128_boxes(torch_cuda, orc, precision):
    _run(orc, workloads.c5(), precision, 1e-8)
