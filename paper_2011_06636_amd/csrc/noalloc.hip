// Residual norm without any allocation: the L2 norm of b - A x of a stencil
// problem (the norm of sections 3 and 4 that drives the scheme choice and the
// stopping tests), for callers that cannot allocate device memory.
//
// The per-block partial sums live in a file-scope device array, one copy per
// GPU for the life of the process.  Host code never passes the array's name
// to a kernel (on the host it is a stand-in, not a device address): the
// device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and kept.
#include <mutex>

#include "internal.h"

namespace srj {

// Partial sums for up to 2^18 workgroups of the residual norm (2 MiB), one
// per 256 columns x 4 rows of a plane, rows counted per eighth of the plane
// when it has at least 64 rows: 8 ceil(n0 / 256) ceil(ceil(n1 / 8) / 4) n2
// partials then, else ceil(n0 / 256) ceil(n1 / 4) n2.  A 16384^2 grid, a
// 512^3 box or a 2D grid with n0 <= 256 and n1 <= 2^20 rows fits.
constexpr int64_t kScratchPartials = int64_t(1) << 18;

static __device__ __align__(256) double scratch[kScratchPartials];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

srj_status scratch_for(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SRJ_ERR_UNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SRJ_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                         hipGetErrorString(e));
        g_scratch[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch[dev];
    return SRJ_OK;
}

}  // namespace

}  // namespace srj

using namespace srj;

extern "C" {

srj_status srj_residual_norm_noalloc(const srj_problem *p, const double *x, void *hip_stream,
                                     double *norm_out)
{
    srj_status st = validate_problem(p);
    if (st != SRJ_OK) return st;
    DevProblem P;
    fill_dev_problem(p, P);
    if (residual_blocks(P) > kScratchPartials)
        return fail(SRJ_ERR_UNSUPPORTED,
                    "grid needs " + std::to_string(residual_blocks(P)) +
                        " partial sums (one per 256 columns x 4 rows of a plane); the static "
                        "scratch holds " + std::to_string(kScratchPartials));
    int dev = 0;
    SRJ_HIP_CHECK(hipGetDevice(&dev));
    if ((st = check_problem_arrays(p, dev)) != SRJ_OK) return st;
    const size_t nb = sizeof(double) * (size_t)(p->n[0] * p->n[1] * p->n[2]);
    if ((st = check_device_array(x, nb, dev, "x")) != SRJ_OK) return st;
    if ((st = check_device_array(norm_out, sizeof(double), dev, "norm_out")) != SRJ_OK) return st;
    double *partials = nullptr;
    if ((st = scratch_for(dev, &partials)) != SRJ_OK) return st;
    SRJ_HIP_CHECK(launch_residual_norm_into(P, x, partials, kScratchPartials, norm_out,
                                            static_cast<hipStream_t>(hip_stream)));
    return SRJ_OK;
}

}  // extern "C"
