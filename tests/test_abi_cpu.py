"""Host-side checks of the C ABI library (no GPU needed).

* libsrj.so loads and exports every entry point declared in include/srj.h.
* srj_scheme (host code of the library) returns the same factors in the same
  order as the oracle, bit for bit, at all 25 levels; its value for M = 1..7
  matches Table 2.
* Argument validation happens before any device call: invalid problems and
  options return SRJ_ERR_INVALID with a message.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2011_06636_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "srj.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(srj_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = abi.load()
    names = header_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(abi.EXPORTS) == names


def test_scheme_table_matches_oracle_bitwise(orc):
    for level in range(25):
        got = np.array(abi.srj_scheme(level))
        ref = orc.scheme(level)
        assert got.shape == ref.shape
        assert np.array_equal(got, ref), level


def test_scheme_invalid_level():
    lib = abi.load()
    M = ctypes.c_int32()
    buf = (ctypes.c_double * 4)()
    assert lib.srj_scheme(25, buf, 4, ctypes.byref(M)) == abi.SRJ_ERR_INVALID
    assert lib.srj_scheme(-1, buf, 4, ctypes.byref(M)) == abi.SRJ_ERR_INVALID
    assert "level" in abi.last_error()
    # cap smaller than M: only cap values written, M reported
    assert lib.srj_scheme(3, buf, 2, ctypes.byref(M)) == abi.SRJ_OK and M.value == 5


def test_default_opts():
    o = abi.srj_default_opts()
    assert o.rule == abi.RULE["heuristic"] and o.tol == 1e-10 and o.max_level == 24
    assert o.precision == abi.PREC["f64"] and o.max_cycles == 10000


def _prob(**kw):
    p = abi.SrjProblem()
    p.ndim = kw.get("ndim", 1)
    n = kw.get("n", (8, 1, 1))
    for d in range(3):
        p.n[d] = n[d]
        p.cconst[d] = kw.get("c", 1.0) if d == 0 else 1.0
        p.face[d] = None
    p.dconst = kw.get("dconst", 2.0)
    p.diag = None
    p.b = kw.get("b", 0x1000)  # never dereferenced: validation fails first
    return p


@pytest.mark.parametrize("kw", [
    dict(ndim=0), dict(ndim=4), dict(n=(0, 1, 1)), dict(ndim=1, n=(8, 2, 1)),
    dict(dconst=0.0), dict(dconst=-1.0), dict(dconst=float("nan")), dict(b=None),
    dict(c=float("inf")), dict(c=float("nan")), dict(c=-1.0),
    dict(ndim=2, n=(8, 65536, 1)), dict(n=(2 ** 38 + 1, 1, 1)), dict(n=(2 ** 62, 1, 1)),
    dict(ndim=3, n=(2 ** 7, 65535, 65535)),
])
def test_setup_rejects_invalid_problem(kw):
    lib = abi.load()
    h = ctypes.c_void_p()
    st = lib.srj_setup(ctypes.byref(_prob(**kw)), None, ctypes.byref(h))
    assert st == abi.SRJ_ERR_INVALID
    assert not h.value
    assert abi.last_error()


@pytest.mark.parametrize("kw", [
    dict(ndim=0), dict(n=(0, 1, 1)), dict(dconst=0.0), dict(b=None), dict(c=float("inf")),
    dict(n=(2 ** 38 + 1, 1, 1)), dict(n=(2 ** 62, 1, 1)), dict(ndim=3, n=(2 ** 40, 2 ** 40, 2 ** 40)),
])
def test_batch_setup_rejects_invalid_problem(kw):
    lib = abi.load()
    h = ctypes.c_void_p()
    probs = (abi.SrjProblem * 2)(_prob(), _prob(**kw))
    st = lib.srj_batch_setup(2, probs, None, ctypes.byref(h))
    assert st == abi.SRJ_ERR_INVALID
    assert not h.value
    assert abi.last_error()


def test_batch_setup_rejects_too_many_points_in_total():
    lib = abi.load()
    h = ctypes.c_void_p()
    probs = (abi.SrjProblem * 3)(*[_prob(n=(2 ** 37, 1, 1)) for _ in range(3)])
    assert lib.srj_batch_setup(3, probs, None, ctypes.byref(h)) == abi.SRJ_ERR_INVALID
    assert "2^38" in abi.last_error()


def test_null_context_calls_are_invalid():
    lib = abi.load()
    nrm = ctypes.c_double()
    assert lib.srj_run_cycle(None, None, 0, ctypes.byref(nrm)) == abi.SRJ_ERR_INVALID
    assert lib.srj_residual_norm(None, None, ctypes.byref(nrm)) == abi.SRJ_ERR_INVALID
    o = abi.srj_default_opts()
    res = abi.SrjSolveResult()
    assert lib.srj_solve(None, None, ctypes.byref(o), ctypes.byref(res), None, None) == abi.SRJ_ERR_INVALID
    assert lib.srj_destroy(None) == abi.SRJ_OK
