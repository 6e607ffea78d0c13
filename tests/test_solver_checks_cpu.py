"""Host-side argument checks of the torch wrapper (no GPU needed): an
iterate that is not a contiguous float64 tensor of the problem's size on
the solver's device is refused before its address reaches the library."""
import pytest
import torch

from paper_2011_06636_amd.solver import check_iterate


def test_cpu_tensor_is_refused_for_a_gpu_solver():
    with pytest.raises(ValueError, match="is on cpu"):
        check_iterate(torch.zeros(10, dtype=torch.float64), "cuda:0", 10)


@pytest.mark.parametrize("x,msg", [
    (torch.zeros(10, dtype=torch.float32), "float64"),
    (torch.zeros(4, 6, dtype=torch.float64).t(), "contiguous"),
    (torch.zeros(9, dtype=torch.float64), "holds 9 values"),
])
def test_layout_checks(x, msg):
    with pytest.raises(ValueError, match=msg):
        check_iterate(x, "cpu", x.numel() if msg != "holds 9 values" else 10)


def test_not_a_tensor():
    with pytest.raises(TypeError):
        check_iterate([0.0] * 10, "cpu", 10)


def test_good_tensor_passes():
    check_iterate(torch.zeros(3, 4, dtype=torch.float64), "cpu", 12)
