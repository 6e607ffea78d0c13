"""GPU parity on general sparse matrices (srj_setup_csr).

* A stencil written as a sparse matrix runs through the ELL kernels and
  reproduces the stencil kernels' solve bit for bit (levels and iterates;
  norms to summation-order rounding): an oracle-free check of the per-row
  expression order.
* Finite element systems on unstructured meshes and random tridiagonal
  systems against the CPU reference: the same levels and iterates (bit for
  bit), norms within summation-order rounding, on the multi-kernel path
  (one sweep per launch) and the one-workgroup path for small systems.
* The training-data collector takes sparse problems too.
* Structure errors are rejected at setup; refinement and the update test are
  refused for sparse matrices.
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


def _solve(prob, resident=True, **kw):
    from paper_2011_06636_amd.solver import Solver
    s = Solver(prob)
    try:
        s.set_resident(resident)
        x = s.zeros()
        out = s.solve(x, **kw)
        return out, x.cpu().numpy().reshape(-1)
    finally:
        s.close()


@pytest.mark.parametrize("make", [
    lambda: workloads.poisson([301, 97], b=np.random.default_rng(1).uniform(-1, 1, (1, 97, 301))),
    lambda: workloads.variable_coefficient(24, seed=2, corr_len=3.0),
    lambda: workloads.random_tridiagonal(5000, seed=3),
], ids=["2d_poisson", "3d_varcoef", "1d_tridiagonal"])
def test_stencil_as_csr_matches_stencil_kernels(torch_cuda, make):
    prob = make()
    kw = dict(tol=1e-10, max_cycles=300)
    a, xa = _solve(prob, resident=False, **kw)
    b, xb = _solve(workloads.to_csr(prob), resident=False, **kw)
    assert np.array_equal(a["levels"], b["levels"])
    assert np.array_equal(xa, xb)
    # the two residual kernels group their partial sums differently
    np.testing.assert_allclose(a["norms"], b["norms"], rtol=1e-12, atol=0)


CASES = [
    ("fem_plate_0.025", lambda: workloads.fem_poisson("plate_hole", 0.025, seed=0), False),
    ("fem_disk_0.025", lambda: workloads.fem_poisson("disk", 0.025, seed=1), False),
    ("fem_disk_0.05_resident", lambda: workloads.fem_poisson("disk", 0.05, seed=2), True),
    ("tridiag_1000_resident", lambda: workloads.random_tridiagonal(1000, seed=4), True),
    ("tridiag_1000", lambda: workloads.random_tridiagonal(1000, seed=5), False),
]


@pytest.mark.parametrize("name,make,resident", CASES, ids=[c[0] for c in CASES])
def test_sparse_solve_matches_reference(torch_cuda, orc, name, make, resident):
    prob = make()
    kw = dict(tol=1e-9, tol_mode="absolute", max_cycles=2000)
    got, gx = _solve(prob, resident=resident, **kw)
    ref = orc.solve(prob, **kw)
    assert got["status"] == ref["status"] == "ok"
    assert np.array_equal(got["levels"], ref["levels"])
    assert got["sweeps"] == ref["sweeps"]
    assert np.array_equal(gx, ref["x"].reshape(-1))
    np.testing.assert_allclose(got["norms"], ref["norms"], rtol=1e-11, atol=0)


def test_collect_on_a_sparse_problem(torch_cuda, orc):
    import torch

    from paper_2011_06636_amd.solver import Solver
    prob = workloads.fem_poisson("disk", 0.1, seed=0)
    assert prob.npoints <= 1024
    u = workloads.training_draws(6, 120, seed=5)
    s = Solver(prob)
    got = s.collect(torch.from_numpy(u).cuda())
    s.close()
    ref = orc.collect(prob, u)
    assert np.array_equal(got["steps"], ref["steps"])
    for t, n in enumerate(ref["steps"]):
        for f in ("level", "action", "M", "chosen", "prev_ratio", "r_before", "r_after"):
            assert np.array_equal(got["samples"][t, :n][f], ref["samples"][t, :n][f]), (t, f)


def _bad(rp, col, val):
    return workloads.csr_problem(np.array(rp), np.array(col), np.array(val), np.ones(len(rp) - 1))


@pytest.mark.parametrize("prob", [
    _bad([0, 1, 2], [0, 0], [2.0, -1.0]),            # row 1 has no diagonal
    _bad([0, 2, 3], [0, 0, 1], [2.0, 1.0, 2.0]),      # diagonal twice
    _bad([0, 2, 3], [0, 5, 1], [2.0, -1.0, 2.0]),     # column out of range
    _bad([0, 1, 2], [0, 1], [2.0, -1.0]),             # diagonal <= 0
    _bad([0, 1, 2], [0, 1], [2.0, np.inf]),           # non-finite entry
], ids=["no_diag", "diag_twice", "col_range", "diag_sign", "inf"])
def test_bad_structure_is_rejected(torch_cuda, prob):
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import Solver
    with pytest.raises(abi.SrjError) as e:
        Solver(prob)
    assert e.value.status == abi.SRJ_ERR_INVALID


def test_sparse_refuses_refinement_and_update_test(torch_cuda):
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import Solver
    s = Solver(workloads.to_csr(workloads.random_tridiagonal(50, seed=0)))
    for kw in (dict(precision="f32"), dict(tol_mode="update_inf")):
        with pytest.raises(abi.SrjError) as e:
            s.solve(s.zeros(), tol=1e-8, **kw)
        assert e.value.status == abi.SRJ_ERR_UNSUPPORTED
    s.close()
