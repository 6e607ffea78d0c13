"""The C ABI from plain C: tests/c_abi/solve_c.c (built by
__graft_entry__.build() with gcc, no Python or torch in it) solves a 2D
Poisson problem through include/srj.h on the default stream; its levels,
sweep count, norms and iterate sum must equal those of the same solve
through the Python binding, and the solve must converge."""
import os
import subprocess

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

BINARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "solve_c")


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _parse(text):
    out = {}
    for line in text.splitlines():
        key, *vals = line.split()
        if key == "status":
            out.update(status=int(vals[0]), converged=int(vals[2]), cycles=int(vals[4]),
                       sweeps=int(vals[6]))
        elif key == "r0":
            out.update(r0=float(vals[0]), r_final=float(vals[2]))
        elif key == "levels":
            out["levels"] = [int(v) for v in vals]
        elif key == "sum":
            out["sum"] = float(vals[0])
    return out


@pytest.mark.parametrize("n0,n1", [(300, 200), (64, 1000), (45, 30)])
def test_plain_c_solve_matches_binding(torch_cuda, n0, n1):
    from paper_2011_06636_amd.solver import Solver
    assert os.path.exists(BINARY), "tests/c_abi/solve_c is not built (run __graft_entry__.build())"
    tol = 1e-8
    run = subprocess.run([BINARY, str(n0), str(n1), repr(tol)], capture_output=True, text=True,
                         timeout=120)
    assert run.returncode == 0, run.stderr + run.stdout
    got = _parse(run.stdout)
    assert got["status"] == 0 and got["converged"] == 1
    b = 1.0 + 0.001 * (np.arange(n0 * n1) % 7).astype(np.float64)
    prob = workloads.poisson([n0, n1], b=b.reshape(1, n1, n0))
    s = Solver(prob)
    out = s.solve(tol=tol, max_cycles=400)
    x = out["x"].cpu().numpy().reshape(-1)
    s.close()
    assert out["status"] == "ok"
    assert got["cycles"] == out["cycles"] and got["sweeps"] == out["sweeps"]
    assert got["levels"] == [int(v) for v in out["levels"]]
    assert got["r0"] == out["r0"] and got["r_final"] == out["r_final"]
    total = 0.0
    for v in x:  # index order, as the C program sums
        total += float(v)
    assert got["sum"] == total
    assert got["r_final"] < tol * got["r0"]
