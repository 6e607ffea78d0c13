"""srj_stream_probe, the streaming kernels that the benchmark's byte rates are
quoted against: they must move exactly what they claim (out = a, out = a + b)
over a length that is not a multiple of a block's share, and refuse bad
arguments before any device work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("n", [2, 4098, 1_000_002])
def test_stream_probe_moves_values(torch_cuda, n):
    from paper_2011_06636_amd import abi
    torch = torch_cuda
    g = torch.Generator(device="cpu").manual_seed(n)
    a = torch.rand(n, dtype=torch.float64, generator=g).cuda()
    b = torch.rand(n, dtype=torch.float64, generator=g).cuda()
    out = torch.full((n + 2,), -7.0, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    abi.srj_stream_probe(0, a.data_ptr(), b.data_ptr(), out.data_ptr(), n, st)
    torch.cuda.synchronize()
    assert torch.equal(out[:n], a) and torch.all(out[n:] == -7.0)
    abi.srj_stream_probe(1, a.data_ptr(), b.data_ptr(), out.data_ptr(), n, st)
    torch.cuda.synchronize()
    ref = (a.cpu().numpy() + b.cpu().numpy())
    assert np.array_equal(out[:n].cpu().numpy(), ref) and torch.all(out[n:] == -7.0)


def test_stream_probe_refuses_bad_arguments(torch_cuda):
    from paper_2011_06636_amd import abi
    torch = torch_cuda
    a = torch.zeros(16, dtype=torch.float64, device="cuda")
    lib = abi.load()
    assert lib.srj_stream_probe(2, a.data_ptr(), a.data_ptr(), a.data_ptr(), 16, None) == abi.SRJ_ERR_INVALID
    assert lib.srj_stream_probe(0, a.data_ptr(), a.data_ptr(), a.data_ptr(), 15, None) == abi.SRJ_ERR_INVALID
    h = torch.zeros(16, dtype=torch.float64).pin_memory()
    assert lib.srj_stream_probe(0, h.data_ptr(), a.data_ptr(), a.data_ptr(), 16, None) == abi.SRJ_ERR_INVALID
