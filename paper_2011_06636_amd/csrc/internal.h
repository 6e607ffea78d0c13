// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "srj.h"

namespace srj {

struct Refine;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
srj_status fail(srj_status st, const std::string &msg);

// The per-cycle solve log (log.cpp): whether SRJ_LOG asks for it, and the
// lines of one ended solve from its level and norm histories (norms holds
// cycles + 1 values, level_sweeps the sweeps of each of nlevels levels).
bool log_enabled();
void log_cycles(const char *what, srj_status st, int cycles, const int32_t *levels,
                const int32_t *level_sweeps, int nlevels, const double *norms, int64_t sweeps,
                double r0, double r_final);

// Does [p, p + bytes) lie inside one allocation of device (or managed)
// memory of device dev?  Host memory, pinned or not, is refused: the kernels
// would fault on pageable memory.  Returns SRJ_OK, or SRJ_ERR_INVALID with a
// message naming `what`.
srj_status check_device_array(const void *p, size_t bytes, int dev, const char *what);

// Largest number of points of one grid (and of all instances of a batch):
// 2^38 binary64 values are 2 TiB, far beyond one device, so every byte count
// and launch dimension derived from it fits its type.
constexpr int64_t kMaxPoints = int64_t(1) << 38;
// n[0] n[1] n[2] <= kMaxPoints without overflow (each n[d] >= 1).
inline bool points_fit(const int64_t n[3])
{
    return n[1] <= kMaxPoints && n[2] <= kMaxPoints / n[1] && n[0] <= kMaxPoints / (n[1] * n[2]);
}

#define SRJ_HIP_CHECK(expr)                                                              \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess)                                                            \
            return ::srj::fail(SRJ_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

// ---------------------------------------------------------------------------
// Scheme family (host): Appendix B levels, Eq. (17) factors, Leja order.
// ---------------------------------------------------------------------------
int level_m(int level);                      // -1 if outside 0..24
const std::vector<double> &level_factors(int level);  // execution order, cached
// Concatenated table of all levels in execution order; offsets[l]..offsets[l+1].
void full_table(std::vector<double> &omega, std::vector<int32_t> &offsets);

// ---------------------------------------------------------------------------
// Device view of a problem
// ---------------------------------------------------------------------------
struct DevProblem {
    int32_t ndim;
    int32_t pad_;
    int64_t n0, n1, n2;
    double c[3];
    const double *face[3];  // nullptr: constant coupling c[d]
    double dconst, dinvconst;
    const double *diag;     // nullptr: constant diagonal
    const double *dinv;     // 1/diag (library-owned) when diag != nullptr
    const double *b;
    // General sparse matrix (srj_setup_csr): ndim = 1, n0 rows, diag and dinv
    // library-owned, off-diagonal entries in a column-major ELL layout,
    // entry j of row p at [j * n0 + p], in the row's storage order.
    const int32_t *ell_len;  // off-diagonal entries per row; nullptr: stencil problem
    const int32_t *ell_col;
    const double *ell_val;
    int32_t ell_width, pad2_;
};

// Binary32 operator used by the refinement inner cycles.
struct DevProblem32 {
    int32_t ndim;
    int32_t pad_;
    int64_t n0, n1, n2;
    float c[3];
    const float *face[3];
    float dconst, dinvconst;
    const float *diag;
    const float *dinv;
};

// Reduction scratch: per-block partial sums and the final sum.
struct ReduceScratch {
    double *partials = nullptr;
    int64_t capacity = 0;
    double *sum = nullptr;       // the device's address of host_sum, where the fold writes
    double *host_sum = nullptr;  // pinned host scalar, valid after the stream is synchronized
};

// ---------------------------------------------------------------------------
// Kernel launchers (sweep.hip, reduce.hip, refine.hip)
// ---------------------------------------------------------------------------
hipError_t compute_dinv(const double *diag, double *dinv, int64_t n, hipStream_t s);

// One binary64 sweep x -> xo with factor w, T sweeps fused when possible.
struct SweepPlan {
    int kind = 0;   // 0 = one sweep per launch; 1 = 2D register tiles; 2 = 2D tiles, b in LDS
    int T = 1;      // sweeps fused per launch
    int bx = 0, by = 0;
    int occ = 1;    // kernel's minimum waves per SIMD (register budget)
};
hipError_t launch_sweep_generic(const DevProblem &P, const double *x, double *xo, double w,
                                hipStream_t s);
// Device state of the per-sweep update test: the largest |x' - x| of sweep g
// accumulates in slot g % 3, spread over kUpdStripes stripes one 128-byte
// line apart so that the blocks' atomic merges do not all hit one address
// (bit patterns of non-negative doubles order like the values; a NaN orders
// above everything).  The first launch that finds the previous sweep's
// maximum below tol sets flag and stop = g - 1.
constexpr int kUpdStripes = 64, kUpdStride = 16;
struct UpdState {
    unsigned long long maxbits[3 * kUpdStripes * kUpdStride];
    int32_t flag, pad_;
    int64_t stop;
};
// One sweep (global index g) that also reduces max |x' - x| and exits early
// once an earlier sweep met the test.
hipError_t launch_sweep_upd(const DevProblem &P, const double *x, double *xo, double w, double tol,
                            UpdState *st, int64_t g, hipStream_t s);
// The update test with fused sweeps (plan kind 10): a launch of T <= kUpdFMaxT
// sweeps accumulates the largest |x' - x| of its k-th sweep in slot [ring][k]
// (kUpdFStripes stripes one 128-byte line apart); a one-workgroup check after
// each launch folds that launch's slots in sweep order, and the first sweep
// below tol sets flag and stop (its global index); launches that find flag
// set do nothing.  The check also clears the slots of the other ring.
constexpr int kUpdFStripes = 16, kUpdFMaxT = 16;
struct UpdFState {
    unsigned long long maxbits[2][kUpdFMaxT][kUpdFStripes * kUpdStride];
    int32_t flag, pad_;
    int64_t stop;
};
// T fused sweeps with the test (kind 10 plans); ring: slot set of this launch.
hipError_t launch_sweep_fused_upd(const DevProblem &P, const SweepPlan &plan, const double *x,
                                  double *xo, const double *w_dev, int T, UpdFState *st, int ring,
                                  hipStream_t s, bool reverse);
bool fused_upd_supported(const DevProblem &P, const SweepPlan &plan);
// Folds the T sweeps of the launch that used `ring` (first global index g0),
// sets flag/stop on the first below tol, and clears the other ring.  T = 0
// only clears.  With pub non-null, also writes flag and stop to pub[0] and
// pub[1] (pinned host memory, through its device mapping).
hipError_t launch_upd_check(UpdFState *st, int ring, int T, int64_t g0, double tol, int64_t *pub,
                            hipStream_t s);
// Fused sweeps: applies w[0..T-1] (device pointer into the scheme table).
// reverse alternates the block order of the block kernels (callers flip it
// every launch); results do not depend on it.
hipError_t launch_sweep_fused(const DevProblem &P, const SweepPlan &plan, const double *x,
                              double *xo, const double *w_dev, int T, hipStream_t s,
                              bool reverse = false);
bool fused_supported(const DevProblem &P, const SweepPlan &plan);
// Lists the fused variants as (kind, rows, halo, occ); returns how many exist.
int plan_variants(int32_t *out, int cap);

// srj_problem checks (api.hip): the description (SRJ_ERR_INVALID with a
// message), its device arrays on device dev, and its device view (dinv unset).
srj_status validate_problem(const srj_problem *p);
srj_status check_problem_arrays(const srj_problem *p, int dev);
void fill_dev_problem(const srj_problem *p, DevProblem &P);

// Sum of (b - A x)^2 into scratch.sum (device).  residual_blocks: the
// partial sums (one per workgroup of the norm, and of the refinement's outer
// pass, which uses the same units) that the scratch must hold.
int64_t residual_blocks(const DevProblem &P);
hipError_t launch_residual_sumsq(const DevProblem &P, const double *x, ReduceScratch &rs,
                                 hipStream_t s);
// The same residual with its L2 norm (square root of the fixed-order sum)
// written to norm_out (device); partials holds at least residual_blocks(P)
// values.  Stencil problems only.
hipError_t launch_residual_norm_into(const DevProblem &P, const double *x, double *partials,
                                     int64_t capacity, double *norm_out, hipStream_t s);
// Folds rs.partials[0..nblocks) into rs.sum in a fixed order.
hipError_t launch_fold(ReduceScratch &rs, int64_t nblocks, hipStream_t s);
// Block-level fixed-order sums used by every reduction kernel.
__device__ __forceinline__ double wave_sum64(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

}  // namespace srj

// ---------------------------------------------------------------------------
// Solver context (the opaque srj_ctx of the C ABI)
// ---------------------------------------------------------------------------
struct srj_ctx {
    srj::DevProblem P{};
    hipStream_t stream = nullptr;
    int device = 0;                // current device at setup; caller arrays must live there
    bool reverse = false;          // block order of the next fused launch (flips every launch)
    int64_t npoints = 0;
    double *ws = nullptr;          // ping-pong partner of the caller's x
    double *dinv = nullptr;        // 1/diag when diag is given
    double *omega_dev = nullptr;   // all levels, execution order (binary64)
    float *omega32_dev = nullptr;  // the same table rounded to binary32
    std::vector<int32_t> offsets;  // level -> first factor in the tables
    // the scheme family in use: the paper's Appendix B levels with the Eq.
    // (17) factors in execution order, or one set by srj_set_scheme_family
    int nlevels = 0;
    std::vector<int32_t> levelM;
    std::vector<std::vector<double>> factors;
    srj::ReduceScratch rs;
    srj::SweepPlan plan;        // binary64 sweeps
    bool resident = false;      // binary64 solves of small grids run in one workgroup
    srj::SweepPlan plan_inner;  // inner sweeps of the refinement modes
    struct srj::Refine *refine = nullptr;  // refinement workspaces (lazily allocated)
    srj::UpdState *upd = nullptr;          // per-sweep update test (lazily allocated)
    srj::UpdFState *updf = nullptr;        // the same for fused sweeps (lazily allocated)
    int64_t *updf_pub = nullptr;           // its flag and stop in pinned host memory
    int64_t *updf_pub_dev = nullptr;       // (the device mapping of updf_pub)
    // one-workgroup solves: result record and level/offset tables (fixed
    // size), level and norm histories (grown to the largest max_cycles seen)
    void *rs_fixed = nullptr;
    int32_t *rs_levels = nullptr;
    double *rs_norms = nullptr;
    int64_t rs_cap = 0;
    // what the tables of rs_fixed hold (level sizes, then offsets; empty
    // before the first upload), and a pinned host mirror of the record and
    // the histories that one launch fills after each solve (rs_host_dev: its
    // device mapping)
    std::vector<int32_t> rs_tables;
    void *rs_host = nullptr, *rs_host_dev = nullptr;
    // library copies of a general sparse matrix (srj_setup_csr)
    double *csr_diag = nullptr, *csr_b = nullptr, *csr_val = nullptr;
    int32_t *csr_len = nullptr, *csr_col = nullptr;
    // Profiling: HIP events around the sweep launches of each cycle.
    bool profiling = false;
    bool prof_pending = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double prof_ms = 0.0;
    int64_t prof_launches = 0, prof_sweeps = 0, prof_pending_launches = 0, prof_pending_sweeps = 0;
};

namespace srj {
srj_status run_sweeps(srj_ctx *c, double **cur, double **nxt, int level);
srj_status residual_norm(srj_ctx *c, const double *x, double *out);
// The L2 norm from n partial sums of squares (device) that a kernel left:
// folded in a fixed order on c's stream, host result, blocking.
srj_status fold_norm(srj_ctx *c, double *partials, int64_t n, double *out);
srj_status collect_profile(srj_ctx *c);
int next_level(srj_rule rule, int level, double ratio, int max_level);
// Refinement (refine.hip).
srj_status refine_solve(srj_ctx *ctx, double *x, const srj_solve_opts *o, srj_solve_result *res,
                        int32_t *levels_out, double *norms_out);
void refine_free(srj_ctx *ctx);
bool inner_fused_supported(const DevProblem &P, const SweepPlan &plan);
srj_status time_inner_plan(srj_ctx *c, const SweepPlan &plan, int sweeps, const float *w_dev,
                           float *ms);
// Whole binary64 solve of a small grid in one workgroup (resident.hip).
constexpr int64_t kResidentMax = 4000;
bool resident_fits(const DevProblem &P);
srj_status resident_solve(srj_ctx *c, double *x, const srj_solve_opts *o, srj_solve_result *res,
                          int32_t *levels_out, double *norms_out);
// The same solve launched with no host work (so that it can be captured in
// a graph): the residual stopping test only, opts already validated and
// clamped as srj_solve does, buffers made by resident_prepare for at least
// o->max_cycles cycles.  The kernel appends its sweep count to rec.sweeps
// (at index *rec.count, kept while below rec.cap; *rec.count is incremented)
// and stores any status other than SRJ_OK and SRJ_ERR_NOT_CONVERGED in
// *rec.bad, in stream order.
struct ResidentRecord {
    int64_t *sweeps = nullptr;
    int32_t *count = nullptr;
    int32_t *bad = nullptr;
    int32_t cap = 0;
};
srj_status resident_prepare(srj_ctx *c, int max_cycles);
// The options of a resident solve of c's grid as the kernels take them, and
// the device tables of level sizes and factor offsets that resident_prepare
// made (for solves run by other kernels, such as the multigrid tail's).
struct ResidentArgs;
srj_status resident_tables(srj_ctx *c, const srj_solve_opts *o, ResidentArgs *a,
                           const int32_t **level_m, const int32_t **offsets);
srj_status resident_launch_recorded(srj_ctx *c, double *x, const srj_solve_opts *o,
                                    const ResidentRecord &rec);
// Autotuner cache (tune.hip): key -> plan and time per sweep.
std::string tune_key(const char *what, int which, int ndim, const int64_t n[3], bool faces,
                     bool diag);
bool tune_cache_get(const std::string &key, SweepPlan &plan, double &us);
void tune_cache_put(const std::string &key, const SweepPlan &plan, double us);
int inner_plan_variants(int32_t *out, int cap);
}  // namespace srj

