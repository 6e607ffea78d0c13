"""Grids of more than 2^31 points (2D: 65536 x 32769; 3D: 2048 x 1024 x
1025, swept two sweeps per launch): every index on the path must be 64-bit.

From x0 = 0 with b = 1 and unit couplings, after one level-1 cycle (two
sweeps) a point's value depends only on its distance to each boundary, up to
2, and its residual up to 3.  A 9 x 9 grid computed by the CPU reference
therefore holds every value the big grid can take: big index i maps to i
near the low boundary, to 8 - (n - 1 - i) near the high one and to 4
elsewhere.  Sampled points (corners, edges, rows around the 2^31-th value,
the last row) must equal the mapped reference values bit for bit, and the
cycle-end norm must equal the weighted sum of the reference residuals.
"""
import ctypes
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

N0, N1 = 65536, 32769


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _map(i, n):
    return i if i < 4 else (8 - (n - 1 - i) if i >= n - 4 else 4)


def _hip():
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return hip


# Sampled rows are read with HIP runtime copies on the raw addresses, with
# explicit bounds: the check involves no kernel besides the library's own.
def _row(ptr, j):
    """Row j of a float64 N1 x N0 device array."""
    assert 0 <= j < N1, j
    out = np.empty(N0, dtype=np.float64)
    assert _hip().hipMemcpy(out.ctypes.data, ptr + 8 * j * N0, 8 * N0, 2) == 0  # device to host
    return out


def test_more_than_2_31_points(torch_cuda, orc):
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import make_problem
    torch = torch_cuda
    assert N0 * N1 > 2 ** 31
    small = workloads.anisotropic([9, 9], (1.0, 1.0), np.ones((1, 9, 9)))
    xs = np.zeros(small.shape)
    for w in orc.scheme(1):
        xs = orc.sweep(small, xs, float(w))
    rs = (small.b - orc.apply(small, xs)).reshape(9, 9)
    xs = xs.reshape(9, 9)
    wt = np.array([1.0] * 4 + [0.0] + [1.0] * 4)
    w0, w1 = wt.copy(), wt.copy()
    w0[4], w1[4] = N0 - 8, N1 - 8
    want_norm = math.sqrt(float(np.sum(w1[:, None] * w0[None, :] * rs * rs)))

    b = torch.ones(N1 * N0, dtype=torch.float64, device="cuda")
    x = torch.zeros(N1 * N0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    flat = (2 ** 31) // N0  # the row holding the 2^31-th value (the last row here)
    assert flat == N1 - 1
    rows = [0, 1, 2, 3, 4, 5, N1 // 2, N1 - 6, N1 - 5, N1 - 4, N1 - 3, N1 - 2, flat]
    cols = [0, 1, 2, 3, 4, 7, N0 // 2, N0 - 5, N0 - 4, N0 - 3, N0 - 1]
    for j in rows:
        assert np.all(_row(b.data_ptr(), j) == 1.0) and np.all(_row(x.data_ptr(), j) == 0.0), j
    p = make_problem(2, [N0, N1, 1], [1.0, 1.0, 0.0], 4.0, b)
    ctx = abi.srj_setup(p, torch.cuda.current_stream().cuda_stream)
    try:
        nrm = abi.srj_run_cycle(ctx, x.data_ptr(), 1)
        torch.cuda.synchronize()
        got = np.stack([_row(x.data_ptr(), j)[cols] for j in rows])
        want = np.array([[xs[_map(j, N1), _map(i, N0)] for i in cols] for j in rows])
        assert np.array_equal(got, want)
        assert nrm == pytest.approx(want_norm, rel=1e-10)
    finally:
        abi.srj_destroy(ctx)
    del x, b
    torch.cuda.empty_cache()


M0, M1, M2 = 2048, 1024, 1025


@pytest.mark.parametrize("faces", [False, True])
def test_3d_more_than_2_31_points(torch_cuda, orc, faces):
    # the same construction in 3D: a level-1 cycle (two sweeps, one launch of
    # the two-sweep plane kernel: constant coefficients, or unit face arrays
    # and a diagonal array of 6, about 140 GB in all) on a 2048 x 1024 x 1025
    # box, checked against a 9 x 9 x 9 reference box on sampled rows, and the
    # norm as a weighted sum
    from paper_2011_06636_amd import abi
    from paper_2011_06636_amd.solver import make_problem
    torch = torch_cuda
    npts = M0 * M1 * M2
    assert npts > 2 ** 31
    small = workloads.anisotropic([9, 9, 9], (1.0, 1.0, 1.0), np.ones((9, 9, 9)))
    xs = np.zeros(small.shape)
    for w in orc.scheme(1):
        xs = orc.sweep(small, xs, float(w))
    rs = (small.b - orc.apply(small, xs)).reshape(9, 9, 9)
    xs = xs.reshape(9, 9, 9)
    wt = np.array([1.0] * 4 + [0.0] + [1.0] * 4)
    w0, w1, w2 = wt.copy(), wt.copy(), wt.copy()
    w0[4], w1[4], w2[4] = M0 - 8, M1 - 8, M2 - 8
    want_norm = math.sqrt(float(np.sum(w2[:, None, None] * w1[None, :, None] * w0[None, None, :]
                                       * rs * rs)))
    b = torch.ones(npts, dtype=torch.float64, device="cuda")
    x = torch.zeros(npts, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    arrays = []
    if faces:
        arrays = [torch.ones(npts, dtype=torch.float64, device="cuda") for _ in range(3)]
        arrays.append(torch.full((npts,), 6.0, dtype=torch.float64, device="cuda"))
        p = make_problem(3, [M0, M1, M2], [0.0, 0.0, 0.0], 1.0, b, faces=arrays[:3],
                         diag=arrays[3])
    else:
        p = make_problem(3, [M0, M1, M2], [1.0, 1.0, 1.0], 6.0, b)
    torch.cuda.synchronize()
    ctx = abi.srj_setup(p, torch.cuda.current_stream().cuda_stream)
    try:
        assert abi.srj_get_plan(ctx, 0)[0] == (12 if faces else 11)
        nrm = abi.srj_run_cycle(ctx, x.data_ptr(), 1)
        torch.cuda.synchronize()
        planes = [0, 1, 3, 4, M2 // 2, (2 ** 31) // (M0 * M1), M2 - 4, M2 - 2, M2 - 1]
        rows = [0, 2, 4, M1 // 2, M1 - 3, M1 - 1]
        cols = [0, 1, 3, 4, M0 // 2, M0 - 4, M0 - 1]
        hip = _hip()
        for k in planes:
            for j in rows:
                assert 0 <= k < M2 and 0 <= j < M1, (k, j)
                out = np.empty(M0, dtype=np.float64)
                ofs = 8 * (k * M1 * M0 + j * M0)
                assert ofs + 8 * M0 <= 8 * npts
                assert hip.hipMemcpy(out.ctypes.data, x.data_ptr() + ofs, 8 * M0, 2) == 0
                want = np.array([xs[_map(k, M2), _map(j, M1), _map(i, M0)] for i in cols])
                assert np.array_equal(out[cols], want), (k, j)
        assert nrm == pytest.approx(want_norm, rel=1e-10)
    finally:
        abi.srj_destroy(ctx)
    del x, b, arrays
    torch.cuda.empty_cache()
