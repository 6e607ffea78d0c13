"""srj_residual_norm_noalloc: the residual norm without a context or any
allocation (its partial sums live in a fixed device array per GPU).

Checked through the C ABI against srj_residual_norm of a context built for
the same problem (the same per-block sums folded in the same order, so the
two agree to the last bits; the bar is 1e-15 relative), on two calls in a row
per case, the second on a smaller grid than the first, so that the second
call reads none of the first call's leftover partial sums.  A grid beyond the
fixed array is refused before any device work.
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


def _noalloc_norm(torch, s, x):
    from paper_2011_06636_amd import abi
    out = torch.full((1,), float("nan"), dtype=torch.float64, device=s.device)
    stream = torch.cuda.current_stream(s.device)
    s.stream.synchronize()
    abi.srj_residual_norm_noalloc(s._prob, x.data_ptr(), stream.cuda_stream, out.data_ptr())
    stream.synchronize()
    return float(out.item())


def _pair(torch, prob, seed):
    from paper_2011_06636_amd.solver import Solver
    s = Solver(prob)
    rng = np.random.default_rng(seed)
    x = s.to_device(rng.uniform(-1.0, 1.0, prob.shape))
    ref = s.residual_norm(x)
    got = _noalloc_norm(torch, s, x)
    s.close()
    return got, ref


CASES = [
    # (first problem, second, smaller problem)
    (lambda: workloads.random_faces([300, 41, 19], seed=3),
     lambda: workloads.random_faces([70, 9, 5], seed=4)),
    (lambda: workloads.c2(n=700),
     lambda: workloads.poisson([257, 3])),
    (lambda: workloads.random_faces([513, 77], seed=5),
     lambda: workloads.c1()),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_norm_matches_context_norm(torch_cuda, case):
    first, second = CASES[case]
    for k, make in enumerate((first, second)):
        prob = make()
        print(f"noalloc case {case}.{k}: n = {prob.n}", flush=True)
        got, ref = _pair(torch_cuda, prob, seed=100 * case + k)
        assert np.isfinite(ref) and ref > 0
        assert abs(got - ref) <= 1e-15 * ref, (case, k, got, ref)


def test_noalloc_refuses_grid_beyond_scratch(torch_cuda):
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import make_problem
    torch = torch_cuda
    b = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    # 8 x 2 x 2048 x 20 partial sums of 256 columns x 4 rows (> 2^18): refused
    # on their count, before the (too small) arrays are looked at or any
    # kernel runs
    p = make_problem(3, [257, 65535, 20], [1.0, 1.0, 1.0], 6.0, b)
    st = abi.load().srj_residual_norm_noalloc(p, b.data_ptr(), None, out.data_ptr())
    assert st == abi.SRJ_ERR_UNSUPPORTED
    assert "static scratch" in abi.last_error()
