"""The autotuner: picks a valid plan by timing, never changes results, and
reuses cached choices (GPU)."""
import os

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


@pytest.mark.parametrize("which,precision", [(0, "f64"), (1, "f32")])
@pytest.mark.parametrize("case", ["2d", "3d"])
def test_autotune_single(torch_cuda, tmp_path, monkeypatch, which, precision, case):
    from paper_2011_06636_amd.solver import Solver
    monkeypatch.setenv("SRJ_TUNE_CACHE", str(tmp_path / "tune.txt"))
    prob = workloads.c2(n=300) if case == "2d" else workloads.variable_coefficient(30, seed=3)
    s = Solver(prob)
    ref = s.solve(tol=1e-10, precision=precision)
    us = s.autotune(which=which, sweeps=24, use_cache=True)
    assert us > 0
    plan = s.get_plan(which)
    out = s.solve(tol=1e-10, precision=precision)
    assert np.array_equal(out["levels"], ref["levels"])
    assert np.array_equal(out["x"].cpu().numpy(), ref["x"].cpu().numpy())
    lines = open(tmp_path / "tune.txt").read().strip().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:5] == [str(v) for v in plan]
    # a second context reuses the cached plan without timing
    s2 = Solver(prob)
    us2 = s2.autotune(which=which, sweeps=24, use_cache=True)
    assert us2 == pytest.approx(float(lines[0].split()[5]))
    assert s2.get_plan(which) == plan
    s.close()
    s2.close()
