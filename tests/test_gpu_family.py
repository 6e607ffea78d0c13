"""GPU tests of srj_set_scheme_family (a user-supplied scheme family).

* The one-level family {w = 1} turns every cycle into one unweighted Jacobi
  sweep (section 2, Eq. 2): the solve must match the CPU reference's Jacobi
  rule bit for bit, through the fused block kernels (T = 1 launches) and the
  one-workgroup solver.
* The paper's factors in their natural index order (instead of the execution
  order) must give the same iterate as the reference's sweeps applied in that
  order.
* Restoring the paper's family gives back a fresh context's results; bad
  families and levels outside a family are rejected.
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


@pytest.mark.parametrize("make,resident", [
    (lambda: workloads.poisson([70, 64], b=np.random.default_rng(1).uniform(-1, 1, (1, 64, 70))), False),
    (lambda: workloads.poisson([40], b=np.random.default_rng(2).uniform(-1, 1, (1, 1, 40))), True),
], ids=["2d_fused", "1d_resident"])
def test_jacobi_family_matches_reference_jacobi(torch_cuda, orc, make, resident):
    from paper_2011_06636_amd.solver import Solver
    prob = make()
    s = Solver(prob)
    s.set_resident(resident)
    s.set_scheme_family([[1.0]])
    kw = dict(tol=1e-4, max_cycles=20000)
    x = s.zeros()
    got = s.solve(x, **kw)
    gx = x.cpu().numpy().reshape(-1)
    s.close()
    ref = orc.solve(prob, rule="jacobi", **kw)
    assert got["status"] == ref["status"]
    assert got["sweeps"] == ref["sweeps"] == got["cycles"]
    assert np.all(got["levels"] == 0)
    assert np.array_equal(gx, ref["x"].reshape(-1))
    np.testing.assert_allclose(got["norms"], ref["norms"], rtol=1e-11, atol=0)


def test_natural_order_family(torch_cuda, orc):
    from paper_2011_06636_amd.solver import Solver
    prob = workloads.poisson([97, 61], b=np.random.default_rng(3).uniform(-1, 1, (1, 61, 97)))
    levels = [orc.omega_natural(orc.level_M(l)) for l in range(12)]
    s = Solver(prob)
    s.set_scheme_family(levels)
    x0 = np.random.default_rng(4).uniform(-1, 1, prob.shape)
    x = s.to_device(x0)
    for lv in (3, 7, 11):
        s.run_cycle(x, lv)
    got = x.cpu().numpy().reshape(-1)
    s.close()
    ref = x0.copy()
    for lv in (3, 7, 11):
        for w in levels[lv]:
            ref = orc.sweep(prob, ref, float(w))
    assert np.array_equal(got, ref.reshape(-1))


def test_restore_paper_family(torch_cuda):
    from paper_2011_06636_amd.solver import Solver
    prob = workloads.c2(n=128)
    fresh = Solver(prob)
    a = fresh.solve(tol=1e-9)
    fresh.close()
    s = Solver(prob)
    s.set_scheme_family([[1.0], [0.5, 1.5]])
    s.set_scheme_family(None)
    b = s.solve(tol=1e-9)
    s.close()
    assert np.array_equal(a["levels"], b["levels"])
    assert np.array_equal(a["x"].cpu().numpy(), b["x"].cpu().numpy())


def test_family_errors(torch_cuda):
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import Solver
    s = Solver(workloads.poisson([20, 20], b=np.ones((1, 20, 20))))
    for bad in ([[]], [[1.0]] * 26, [[float("nan")]]):
        with pytest.raises(abi.SrjError) as e:
            s.set_scheme_family(bad)
        assert e.value.status == abi.SRJ_ERR_INVALID
    s.set_scheme_family([[1.0], [0.6, 1.3]])
    for kw in (dict(start_level=2), dict(rule="fixed", fixed_level=5)):
        with pytest.raises(abi.SrjError) as e:
            s.solve(tol=1e-6, **kw)
        assert e.value.status == abi.SRJ_ERR_INVALID
    with pytest.raises(abi.SrjError):
        s.run_cycle(s.zeros(), 2)
    out = s.solve(tol=1e-6, max_cycles=50000)  # the top level is clamped to 1
    assert out["levels"].max() <= 1
    s.close()
