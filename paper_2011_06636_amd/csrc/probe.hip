// Streaming kernels of known traffic: the achievable HBM ceiling that the
// sweep kernels' byte rates are quoted against, and the reference dispatch
// that scales the hardware byte counters (FETCH_SIZE, WRITE_SIZE).
//
// kind 0: out[i] = a[i]            (read 8 B, write 8 B per value)
// kind 1: out[i] = a[i] + b[i]     (read 16 B, write 8 B per value: the
//                                   read/write mix of a one-sweep launch)
// Each thread moves 4 pairs of binary64 values with 16-byte accesses;
// consecutive lanes touch consecutive 16-byte words.
#include "internal.h"

namespace srj {

namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeUnroll = 4;

struct alignas(16) D2 {
    double v[2];
};

template <int KIND>
__global__ __launch_bounds__(kProbeBlock) void k_stream(const D2 *__restrict__ a,
                                                        const D2 *__restrict__ b,
                                                        D2 *__restrict__ out, int64_t npairs)
{
    const int64_t base = (int64_t)blockIdx.x * (kProbeBlock * kProbeUnroll) + threadIdx.x;
    D2 va[kProbeUnroll], vb[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kProbeBlock;
        if (i < npairs) {
            va[u] = a[i];
            if (KIND == 1) vb[u] = b[i];
        }
    }
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kProbeBlock;
        if (i < npairs) {
            D2 o = va[u];
            if (KIND == 1) {
                o.v[0] = va[u].v[0] + vb[u].v[0];
                o.v[1] = va[u].v[1] + vb[u].v[1];
            }
            out[i] = o;
        }
    }
}

}  // namespace

}  // namespace srj

using namespace srj;

extern "C" {

srj_status srj_stream_probe(int32_t kind, const double *a, const double *b, double *out, int64_t n,
                            void *hip_stream)
{
    if (kind != 0 && kind != 1) return fail(SRJ_ERR_INVALID, "kind must be 0 (copy) or 1 (a + b)");
    if (n < 2 || n % 2 != 0) return fail(SRJ_ERR_INVALID, "n must be even and >= 2");
    if (n > (int64_t(1) << 36)) return fail(SRJ_ERR_INVALID, "n must be <= 2^36");
    int dev = 0;
    SRJ_HIP_CHECK(hipGetDevice(&dev));
    const size_t bytes = sizeof(double) * (size_t)n;
    srj_status st = check_device_array(a, bytes, dev, "a");
    if (st == SRJ_OK && kind == 1) st = check_device_array(b, bytes, dev, "b");
    if (st == SRJ_OK) st = check_device_array(out, bytes, dev, "out");
    if (st != SRJ_OK) return st;
    if ((uintptr_t)a % 16 || (kind == 1 && (uintptr_t)b % 16) || (uintptr_t)out % 16)
        return fail(SRJ_ERR_INVALID, "arrays must be 16-byte aligned");
    const int64_t npairs = n / 2;
    const int64_t per_block = kProbeBlock * kProbeUnroll;
    const int64_t blocks = (npairs + per_block - 1) / per_block;
    if (blocks > INT32_MAX) return fail(SRJ_ERR_INVALID, "n too large for one launch");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const D2 *pa = reinterpret_cast<const D2 *>(a);
    const D2 *pb = reinterpret_cast<const D2 *>(kind == 1 ? b : a);
    D2 *po = reinterpret_cast<D2 *>(out);
    if (kind == 0)
        hipLaunchKernelGGL(k_stream<0>, dim3((unsigned)blocks), dim3(kProbeBlock), 0, s, pa, pb, po,
                           npairs);
    else
        hipLaunchKernelGGL(k_stream<1>, dim3((unsigned)blocks), dim3(kProbeBlock), 0, s, pa, pb, po,
                           npairs);
    SRJ_HIP_CHECK(hipGetLastError());
    return SRJ_OK;
}

}  // extern "C"
