"""Device-array validation at the C ABI (srj_setup, srj_solve, srj_run_cycle,
srj_residual_norm, srj_collect, srj_batch_setup, srj_batch_solve).

Every case passes pinned host memory where device memory is required: the
library must refuse it with SRJ_ERR_INVALID before any device work.  Pinned
memory is reachable from the GPU, so even a missing check would not fault;
the test only observes the status.
"""
import ctypes

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


def _pinned(torch, n):
    return torch.zeros(n, dtype=torch.float64).pin_memory()


def test_setup_refuses_host_b(torch_cuda):
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import make_problem
    torch = torch_cuda
    b = _pinned(torch, 40 * 30)
    p = make_problem(2, [40, 30, 1], [1.0, 1.0, 0.0], 4.0, b)
    ctx = ctypes.c_void_p()
    st = abi.load().srj_setup(ctypes.byref(p), None, ctypes.byref(ctx))
    assert st == abi.SRJ_ERR_INVALID and not ctx.value
    assert b"device memory" in abi.load().srj_last_error()


def test_solve_calls_refuse_host_x(torch_cuda):
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import Solver
    torch = torch_cuda
    s = Solver(workloads.poisson([40, 30], b=np.ones((1, 30, 40))))
    x = _pinned(torch, 40 * 30)
    lib = abi.load()
    r = ctypes.c_double()
    assert lib.srj_run_cycle(s.ctx, ctypes.c_void_p(x.data_ptr()), 3, ctypes.byref(r)) == abi.SRJ_ERR_INVALID
    assert lib.srj_residual_norm(s.ctx, ctypes.c_void_p(x.data_ptr()), ctypes.byref(r)) == abi.SRJ_ERR_INVALID
    o = abi.SrjSolveOpts()
    lib.srj_default_opts(ctypes.byref(o))
    res = abi.SrjSolveResult()
    assert lib.srj_solve(s.ctx, ctypes.c_void_p(x.data_ptr()), ctypes.byref(o), ctypes.byref(res),
                         None, None) == abi.SRJ_ERR_INVALID
    # a device iterate of the right size still works afterwards
    out = s.solve(tol=1e-8)
    assert out["status"] == "ok"
    s.close()


def test_collect_refuses_host_draws(torch_cuda):
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import Solver
    torch = torch_cuda
    s = Solver(workloads.training_problem(10))
    u = _pinned(torch, 4 * 20)
    samples = torch.zeros(4 * 20 * 3 * np.dtype(abi.SAMPLE_DTYPE).itemsize, dtype=torch.uint8,
                          device="cuda")
    steps = torch.zeros(4, dtype=torch.int32, device="cuda")
    st = abi.load().srj_collect(s.ctx, 4, 20, ctypes.c_void_p(u.data_ptr()), ctypes.c_double(1e-8), 24,
                                ctypes.c_void_p(samples.data_ptr()), ctypes.c_void_p(steps.data_ptr()))
    assert st == abi.SRJ_ERR_INVALID
    s.close()


def test_batch_refuses_host_arrays(torch_cuda):
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import BatchSolver, make_problem
    torch = torch_cuda
    # host b at setup
    b = _pinned(torch, 20 * 20)
    probs = (abi.SrjProblem * 1)(make_problem(2, [20, 20, 1], [1.0, 1.0, 0.0], 4.0, b))
    h = ctypes.c_void_p()
    assert abi.load().srj_batch_setup(1, probs, None, ctypes.byref(h)) == abi.SRJ_ERR_INVALID
    # host iterate at solve: refused by the library itself
    bs = BatchSolver([workloads.c4_instance(i, lo=20, hi=40) for i in range(2)])
    xs = bs.zeros()
    xs[1] = _pinned(torch, xs[1].numel()).view(xs[1].shape)
    ptrs = (ctypes.c_void_p * 2)(*[x.data_ptr() for x in xs])
    o = abi.SrjSolveOpts()
    abi.load().srj_default_opts(ctypes.byref(o))
    res = (abi.SrjSolveResult * 2)()
    assert abi.load().srj_batch_solve(bs.handle, ptrs, ctypes.byref(o), res, None) == abi.SRJ_ERR_INVALID
    bs.close()
