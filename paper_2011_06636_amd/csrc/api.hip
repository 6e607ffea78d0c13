// C ABI entry points and the host side of the solve loop.
//
// Method: Islam & Wang, arXiv 2011.06636.  A cycle is M relaxed Jacobi
// sweeps with the factors of one scheme level (section 2, Eq. 7 and
// Eq. (17); levels from Appendix B).  After each cycle the L2 residual norm
// is reduced on the device and read back; Algorithm 1 (section 3) picks the
// next level from the ratio of the norms after and before the cycle.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "internal.h"
#include "plane3d.h"

namespace srj {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

srj_status fail(srj_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

srj_status check_device_array(const void *p, size_t bytes, int dev, const char *what)
{
    if (!p) return fail(SRJ_ERR_INVALID, std::string(what) + " is NULL");
    hipPointerAttribute_t a{};
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SRJ_ERR_INVALID, std::string(what) + " is not device memory");
    }
    const bool devmem = a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
    if (!devmem || a.device != dev)
        return fail(SRJ_ERR_INVALID, std::string(what) + " is not device memory of the context's GPU");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SRJ_ERR_INVALID, std::string(what) + " is not inside a device allocation");
    }
    const uintptr_t lo = (uintptr_t)base, at = (uintptr_t)p;
    if (at < lo || bytes > size - (at - lo))
        return fail(SRJ_ERR_INVALID, std::string(what) + " extends past the end of its allocation");
    return SRJ_OK;
}

}  // namespace srj

namespace srj {

srj_status validate_problem(const srj_problem *p)
{
    if (!p) return fail(SRJ_ERR_INVALID, "problem is NULL");
    if (p->ndim < 1 || p->ndim > 3) return fail(SRJ_ERR_INVALID, "ndim must be 1, 2 or 3");
    for (int d = 0; d < 3; ++d) {
        if (p->n[d] < 1) return fail(SRJ_ERR_INVALID, "every n[d] must be >= 1");
        if (d >= p->ndim && p->n[d] != 1) return fail(SRJ_ERR_INVALID, "n[d] must be 1 for d >= ndim");
        if (d < p->ndim && !p->face[d] && !(p->cconst[d] >= 0.0 && isfinite(p->cconst[d])))
            return fail(SRJ_ERR_INVALID, "cconst[d] must be finite and >= 0");
    }
    if (p->n[1] > 65535 || p->n[2] > 65535)
        return fail(SRJ_ERR_INVALID, "n[1] and n[2] must be <= 65535");
    if (!points_fit(p->n)) return fail(SRJ_ERR_INVALID, "n[0] n[1] n[2] must be <= 2^38");
    if (!p->b) return fail(SRJ_ERR_INVALID, "b is NULL");
    if (!p->diag && !(p->dconst > 0.0) ) return fail(SRJ_ERR_INVALID, "dconst must be > 0");
    if (!p->diag && !isfinite(p->dconst)) return fail(SRJ_ERR_INVALID, "dconst must be finite");
    return SRJ_OK;
}

srj_status check_problem_arrays(const srj_problem *p, int dev)
{
    const size_t nb = sizeof(double) * (size_t)(p->n[0] * p->n[1] * p->n[2]);
    srj_status st = check_device_array(p->b, nb, dev, "b");
    if (st == SRJ_OK && p->diag) st = check_device_array(p->diag, nb, dev, "diag");
    for (int d = 0; st == SRJ_OK && d < p->ndim; ++d)
        if (p->face[d]) st = check_device_array(p->face[d], nb, dev, "face[d]");
    return st;
}

void fill_dev_problem(const srj_problem *p, DevProblem &P)
{
    P = DevProblem{};
    P.ndim = p->ndim;
    P.n0 = p->n[0];
    P.n1 = p->n[1];
    P.n2 = p->n[2];
    for (int d = 0; d < 3; ++d) {
        P.c[d] = d < p->ndim ? p->cconst[d] : 0.0;
        P.face[d] = d < p->ndim ? p->face[d] : nullptr;
    }
    P.dconst = p->diag ? 0.0 : p->dconst;
    P.dinvconst = p->diag ? 0.0 : 1.0 / p->dconst;
    P.diag = p->diag;
    P.b = p->b;
}

}  // namespace srj

using namespace srj;

namespace {

srj_status validate_opts(const srj_solve_opts *o)
{
    if (!o) return fail(SRJ_ERR_INVALID, "opts is NULL");
    if (o->rule < SRJ_RULE_HEURISTIC || o->rule > SRJ_RULE_FIXED)
        return fail(SRJ_ERR_INVALID, "unknown rule");
    if (o->rule == SRJ_RULE_FIXED && (o->fixed_level < 0 || o->fixed_level >= SRJ_NUM_LEVELS))
        return fail(SRJ_ERR_INVALID, "fixed_level outside 0..24");
    if (o->tol_mode != SRJ_TOL_RELATIVE && o->tol_mode != SRJ_TOL_ABSOLUTE &&
        o->tol_mode != SRJ_TOL_UPDATE_INF)
        return fail(SRJ_ERR_INVALID, "unknown tol_mode");
    if (!(o->tol > 0.0)) return fail(SRJ_ERR_INVALID, "tol must be > 0");
    if (o->max_cycles < 1) return fail(SRJ_ERR_INVALID, "max_cycles must be >= 1");
    if (o->max_sweeps < 1) return fail(SRJ_ERR_INVALID, "max_sweeps must be >= 1");
    if (o->max_level < 0 || o->max_level >= SRJ_NUM_LEVELS)
        return fail(SRJ_ERR_INVALID, "max_level outside 0..24");
    if (o->start_level < 0 || o->start_level > o->max_level)
        return fail(SRJ_ERR_INVALID, "start_level outside 0..max_level");
    if (o->precision < SRJ_PREC_F64 || o->precision > SRJ_PREC_BF16_REFINE)
        return fail(SRJ_ERR_INVALID, "unknown precision");
    if (!(o->scale_target >= 0.0)) return fail(SRJ_ERR_INVALID, "scale_target must be >= 0");
    return SRJ_OK;
}

// Plane chunk of the per-face two-sweep tiles (4 rows, 60 columns): 16 when
// the grid still gives at least 4096 waves with it (measured 7 % faster than
// 8 at 256^3), else 8 (1.6x faster at 96^3, where 16 leaves too few waves).
int per_face_chunk(const DevProblem &P)
{
    const int64_t waves = ((P.n0 + 59) / 60) * ((P.n1 + 3) / 4) * ((P.n2 + 15) / 16);
    return waves >= 4096 ? 16 : 8;
}

SweepPlan default_inner_plan(const DevProblem &P)
{
    SweepPlan pl;
    if (P.ndim == 3) {
        if (!P.face[0] && !P.face[1] && !P.face[2] && !P.diag) {
            pl.kind = 11;  // two-sweep plane tiles: 8 rows, 8 planes per chunk
            pl.by = 8;
            pl.T = 2;
            pl.occ = 8;
        } else if (plane3d_fits(P.ndim, P.face[0], P.face[1], P.face[2], P.diag)) {
            // per-face two-sweep plane tiles of 4 rows: chunks of 16 planes
            // where they still give at least 4096 waves, else 8
            pl.kind = 12;
            pl.by = 4;
            pl.T = 2;
            pl.occ = per_face_chunk(P);
        } else {
            pl.kind = 3;
            pl.by = 16;
        }
        return pl;
    }
    if (P.ndim == 2 && !P.face[0] && !P.face[1] && !P.diag && P.n0 >= 64 && P.n1 >= 64) {
        pl.kind = 7;  // blocks of 8 waves x 8 rows, 8 sweeps per launch
        pl.by = 8;
        pl.T = 8;
        pl.occ = 8;
    }
    if (P.ndim == 2 && P.face[0] && P.face[1] && P.diag && P.n0 >= 64 && P.n1 >= 64) {
        pl.kind = 10;  // per-face blocks of 8 waves x 8 rows, 8 sweeps per launch
        pl.by = 8;
        pl.T = 8;
        pl.occ = 8;
    }
    return pl;
}

SweepPlan default_plan(const DevProblem &P)
{
    SweepPlan pl;
    pl.kind = 0;
    pl.T = 1;
    if (P.ndim == 3) {
        if (!P.face[0] && !P.face[1] && !P.face[2] && !P.diag) {
            pl.kind = 11;  // two-sweep plane tiles: 4 rows, 8 planes per chunk
            pl.by = 4;
            pl.T = 2;
            pl.occ = 8;
        } else if (plane3d_fits(P.ndim, P.face[0], P.face[1], P.face[2], P.diag)) {
            // per-face two-sweep plane tiles of 4 rows: chunks of 16 planes
            // where they still give at least 4096 waves, else 8
            pl.kind = 12;
            pl.by = 4;
            pl.T = 2;
            pl.occ = per_face_chunk(P);
        } else {
            pl.kind = 3;
            pl.by = 16;
        }
        return pl;
    }
    if (P.ndim == 2 && !P.face[0] && !P.face[1] && !P.diag && P.n0 >= 64 && P.n1 >= 64) {
        // blocks of 8 waves x 8 rows.  Grids of at least 512 blocks of 108 x 44
        // written points (two per CU) take two columns per lane and 10 sweeps
        // per launch; smaller grids, where a launch lasts about one block, take
        // one column per lane and 8 sweeps per launch (shorter blocks).
        const int64_t wide_blocks = ((P.n0 + 107) / 108) * ((P.n1 + 43) / 44);
        pl.kind = wide_blocks >= 512 ? 8 : 7;
        pl.by = 8;
        pl.T = wide_blocks >= 512 ? 10 : 8;
        pl.occ = 8;
    }
    if (P.ndim == 2 && P.face[0] && P.face[1] && P.diag && P.n0 >= 64 && P.n1 >= 64) {
        // per-face blocks (kind 10): 8 waves x 8 rows, 8 sweeps per launch
        // (48 x 48 written points) on grids of at least 1024 such blocks;
        // smaller grids take 16 waves x 4 rows and 12 sweeps (40 x 40 written
        // points), fewer launches per cycle for about as many blocks
        const int64_t blocks = ((P.n0 + 47) / 48) * ((P.n1 + 47) / 48);
        pl.kind = 10;
        pl.by = blocks >= 1024 ? 8 : 4;
        pl.T = blocks >= 1024 ? 8 : 12;
        pl.occ = blocks >= 1024 ? 8 : 16;
    }
    return pl;
}

}  // namespace

namespace srj {

// Sweeps of one cycle.  *cur holds the iterate; the pointers are swapped
// after every launch so that *cur always names the latest iterate.
srj_status run_sweeps(srj_ctx *c, double **cur, double **nxt, int level)
{
    const std::vector<double> &w = c->factors[level];
    const int M = static_cast<int>(w.size());
    const double *wdev = c->omega_dev + c->offsets[level];
    int64_t launches = 0;
    if (c->profiling) SRJ_HIP_CHECK(hipEventRecord(c->ev0, c->stream));
    if (c->plan.kind != 0 && fused_supported(c->P, c->plan)) {
        for (int done = 0; done < M;) {
            const int T = std::min(c->plan.T, M - done);
            SRJ_HIP_CHECK(
                launch_sweep_fused(c->P, c->plan, *cur, *nxt, wdev + done, T, c->stream, c->reverse));
            c->reverse = !c->reverse;
            std::swap(*cur, *nxt);
            done += T;
            ++launches;
        }
    } else {
        for (int k = 0; k < M; ++k) {
            SRJ_HIP_CHECK(launch_sweep_generic(c->P, *cur, *nxt, w[k], c->stream));
            std::swap(*cur, *nxt);
            ++launches;
        }
    }
    if (c->profiling) {
        SRJ_HIP_CHECK(hipEventRecord(c->ev1, c->stream));
        c->prof_pending = true;
        c->prof_pending_launches = launches;
        c->prof_pending_sweeps = M;
    }
    return SRJ_OK;
}

// Folds the last cycle's event pair into the profile (after a stream sync).
srj_status collect_profile(srj_ctx *c)
{
    if (!c->profiling || !c->prof_pending) return SRJ_OK;
    float ms = 0.f;
    SRJ_HIP_CHECK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->prof_ms += ms;
    c->prof_launches += c->prof_pending_launches;
    c->prof_sweeps += c->prof_pending_sweeps;
    c->prof_pending = false;
    return SRJ_OK;
}

srj_status residual_norm(srj_ctx *c, const double *x, double *out)
{
    SRJ_HIP_CHECK(launch_residual_sumsq(c->P, x, c->rs, c->stream));
    SRJ_HIP_CHECK(hipStreamSynchronize(c->stream));  // the fold wrote *rs.host_sum
    *out = sqrt(*c->rs.host_sum);
    return collect_profile(c);
}

srj_status fold_norm(srj_ctx *c, double *partials, int64_t n, double *out)
{
    ReduceScratch rs = c->rs;  // its device and pinned scalars
    rs.partials = partials;
    rs.capacity = n;
    SRJ_HIP_CHECK(launch_fold(rs, n, c->stream));
    SRJ_HIP_CHECK(hipStreamSynchronize(c->stream));  // the fold wrote *rs.host_sum
    *out = sqrt(*c->rs.host_sum);
    return collect_profile(c);
}

int next_level(srj_rule rule, int level, double ratio, int max_level)
{
    int nl = level;
    if (rule == SRJ_RULE_HEURISTIC) {
        if (ratio > 0.4)
            nl = level + 1;
        else if (ratio < 0.4 && ratio > 0.2)
            nl = level - 1;
    } else if (rule == SRJ_RULE_INCREASING) {
        nl = level + 1;
    }
    return std::max(0, std::min(nl, max_level));
}

}  // namespace srj

extern "C" {

void srj_default_opts(srj_solve_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->rule = SRJ_RULE_HEURISTIC;
    o->fixed_level = 0;
    o->tol_mode = SRJ_TOL_RELATIVE;
    o->tol = 1e-10;
    o->max_cycles = 10000;
    o->max_sweeps = 50000000;
    o->precision = SRJ_PREC_F64;
    o->start_level = 0;
    o->max_level = SRJ_NUM_LEVELS - 1;
    o->scale_target = 0.0;
    o->r0 = 0.0;
}

const char *srj_last_error(void) { return g_last_error.c_str(); }

srj_status srj_scheme(int32_t level, double *omega_out, int32_t cap, int32_t *M_out)
{
    if (level < 0 || level >= SRJ_NUM_LEVELS) return fail(SRJ_ERR_INVALID, "level outside 0..24");
    if (!M_out || (cap > 0 && !omega_out)) return fail(SRJ_ERR_INVALID, "NULL output pointer");
    const std::vector<double> &w = level_factors(level);
    *M_out = static_cast<int32_t>(w.size());
    const int n = std::min<int>(cap, static_cast<int>(w.size()));
    for (int i = 0; i < n; ++i) omega_out[i] = w[i];
    return SRJ_OK;
}

srj_status srj_destroy(srj_ctx *c)
{
    if (!c) return SRJ_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    refine_free(c);
    (void)hipFree(c->upd);
    (void)hipFree(c->updf);
    (void)hipHostFree(c->updf_pub);
    (void)hipFree(c->rs_fixed);
    (void)hipFree(c->rs_levels);
    (void)hipFree(c->rs_norms);
    (void)hipHostFree(c->rs_host);
    for (void *q : {(void *)c->csr_diag, (void *)c->csr_b, (void *)c->csr_val, (void *)c->csr_len,
                    (void *)c->csr_col})
        (void)hipFree(q);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    (void)hipFree(c->ws);
    (void)hipFree(c->dinv);
    (void)hipFree(c->omega_dev);
    (void)hipFree(c->omega32_dev);
    (void)hipFree(c->rs.partials);
    (void)hipHostFree(c->rs.host_sum);  // rs.sum is its device mapping
    delete c;
    return SRJ_OK;
}

static srj_status ctx_finish(srj_ctx *c);

// The paper's family: Appendix B levels, Eq. (17) factors in execution order.
static void paper_family(srj_ctx *c)
{
    c->nlevels = SRJ_NUM_LEVELS;
    c->levelM.resize(SRJ_NUM_LEVELS);
    c->factors.resize(SRJ_NUM_LEVELS);
    for (int l = 0; l < SRJ_NUM_LEVELS; ++l) {
        c->levelM[l] = level_m(l);
        c->factors[l] = level_factors(l);
    }
}

// Concatenates the family into the device tables (binary64 and binary32) and
// the per-level offsets; replaces earlier tables.  Synchronises the stream.
static srj_status upload_family(srj_ctx *c)
{
    std::vector<double> table;
    std::vector<int32_t> offs;
    for (int l = 0; l < c->nlevels; ++l) {
        offs.push_back((int32_t)table.size());
        table.insert(table.end(), c->factors[l].begin(), c->factors[l].end());
    }
    offs.push_back((int32_t)table.size());
    std::vector<float> table32(table.size());
    for (size_t i = 0; i < table.size(); ++i) table32[i] = static_cast<float>(table[i]);
    SRJ_HIP_CHECK(hipStreamSynchronize(c->stream));  // no kernel may still read the old tables
    (void)hipFree(c->omega_dev);
    (void)hipFree(c->omega32_dev);
    c->omega_dev = nullptr;
    c->omega32_dev = nullptr;
    if (hipMalloc(&c->omega_dev, sizeof(double) * table.size()) != hipSuccess ||
        hipMalloc(&c->omega32_dev, sizeof(float) * table.size()) != hipSuccess)
        return fail(SRJ_ERR_NOMEM, "hipMalloc failed for the scheme tables");
    SRJ_HIP_CHECK(hipMemcpy(c->omega_dev, table.data(), sizeof(double) * table.size(),
                            hipMemcpyHostToDevice));
    SRJ_HIP_CHECK(hipMemcpy(c->omega32_dev, table32.data(), sizeof(float) * table32.size(),
                            hipMemcpyHostToDevice));
    c->offsets = offs;
    return SRJ_OK;
}

srj_status srj_setup(const srj_problem *p, void *hip_stream, srj_ctx **out)
{
    if (!out) return fail(SRJ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    srj_status st = validate_problem(p);
    if (st != SRJ_OK) return st;
    int dev = 0;
    SRJ_HIP_CHECK(hipGetDevice(&dev));
    if ((st = check_problem_arrays(p, dev)) != SRJ_OK) return st;

    srj_ctx *c = new srj_ctx();
    c->device = dev;
    c->stream = static_cast<hipStream_t>(hip_stream);
    DevProblem &P = c->P;
    fill_dev_problem(p, P);
    c->npoints = P.n0 * P.n1 * P.n2;
    const size_t bytes = sizeof(double) * (size_t)c->npoints;

    auto nomem = [&](const char *what) {
        srj_destroy(c);
        return fail(SRJ_ERR_NOMEM, std::string("hipMalloc failed for ") + what);
    };
    if (hipMalloc(&c->ws, bytes) != hipSuccess) return nomem("ping-pong buffer");
    if (p->diag) {
        if (hipMalloc(&c->dinv, bytes) != hipSuccess) return nomem("1/D");
        hipError_t e = compute_dinv(p->diag, c->dinv, c->npoints, c->stream);
        if (e != hipSuccess) {
            srj_destroy(c);
            return fail(SRJ_ERR_HIP, std::string("1/D kernel: ") + hipGetErrorString(e));
        }
        P.dinv = c->dinv;
    }
    st = ctx_finish(c);
    if (st == SRJ_OK) *out = c;
    return st;
}

// Scheme tables, reduction scratch and plans: the part of a context that does
// not depend on how the matrix was given.  Destroys c on failure.
static srj_status ctx_finish(srj_ctx *c)
{
    DevProblem &P = c->P;
    auto nomem = [&](const char *what) {
        srj_destroy(c);
        return fail(SRJ_ERR_NOMEM, std::string("hipMalloc failed for ") + what);
    };
    paper_family(c);
    srj_status fs = upload_family(c);
    if (fs != SRJ_OK) {
        srj_destroy(c);
        return fs;
    }
    hipError_t e = hipSuccess;
    c->rs.capacity = residual_blocks(P);
    if (e == hipSuccess && hipMalloc(&c->rs.partials, sizeof(double) * c->rs.capacity) != hipSuccess)
        return nomem("reduction partials");
    if (e == hipSuccess && hipHostMalloc(&c->rs.host_sum, sizeof(double), 0) != hipSuccess)
        return nomem("pinned scalar");
    // the fold writes the sum straight into the pinned scalar through its
    // device mapping: no copy launch after each norm
    if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&c->rs.sum, c->rs.host_sum, 0);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        srj_destroy(c);
        return fail(SRJ_ERR_HIP, std::string("setup: ") + hipGetErrorString(e));
    }
    c->plan = default_plan(P);
    c->plan_inner = default_inner_plan(P);
    c->resident = resident_fits(P);
    return SRJ_OK;
}

srj_status srj_set_scheme_family(srj_ctx *c, int32_t nlevels, const int32_t *M, const double *omegas)
{
    if (!c) return fail(SRJ_ERR_INVALID, "ctx is NULL");
    if (nlevels == 0) {  // back to the paper's family
        paper_family(c);
        return upload_family(c);
    }
    if (nlevels < 0 || nlevels > SRJ_NUM_LEVELS) return fail(SRJ_ERR_INVALID, "nlevels outside 0..25");
    if (!M || !omegas) return fail(SRJ_ERR_INVALID, "NULL argument");
    int64_t total = 0;
    for (int l = 0; l < nlevels; ++l) {
        if (M[l] < 1 || M[l] > (1 << 20)) return fail(SRJ_ERR_INVALID, "M must be 1 .. 2^20");
        total += M[l];
    }
    if (total > (1 << 24)) return fail(SRJ_ERR_INVALID, "too many factors");
    for (int64_t i = 0; i < total; ++i)
        if (!isfinite(omegas[i])) return fail(SRJ_ERR_INVALID, "factors must be finite");
    c->nlevels = nlevels;
    c->levelM.assign(M, M + nlevels);
    c->factors.assign(nlevels, {});
    for (int l = 0, k = 0; l < nlevels; k += M[l], ++l)
        c->factors[l].assign(omegas + k, omegas + k + M[l]);
    return upload_family(c);
}

srj_status srj_setup_csr(const srj_csr_problem *p, void *hip_stream, srj_ctx **out)
{
    if (!out) return fail(SRJ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!p || !p->rowptr || !p->col || !p->val || !p->b) return fail(SRJ_ERR_INVALID, "NULL argument");
    if (p->n < 1 || p->n > ((int64_t)1 << 31) - 1) return fail(SRJ_ERR_INVALID, "n must be 1 .. 2^31 - 1");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int64_t n = p->n;
    int dev = 0;
    SRJ_HIP_CHECK(hipGetDevice(&dev));
    srj_status chk = check_device_array(p->rowptr, sizeof(int64_t) * ((size_t)n + 1), dev, "rowptr");
    if (chk == SRJ_OK) chk = check_device_array(p->b, sizeof(double) * (size_t)n, dev, "b");
    if (chk != SRJ_OK) return chk;
    // the structure is checked on the host: copy it
    std::vector<int64_t> rp((size_t)n + 1);
    SRJ_HIP_CHECK(hipStreamSynchronize(stream));
    SRJ_HIP_CHECK(hipMemcpy(rp.data(), p->rowptr, sizeof(int64_t) * rp.size(), hipMemcpyDeviceToHost));
    if (rp[0] != 0) return fail(SRJ_ERR_INVALID, "rowptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return fail(SRJ_ERR_INVALID, "rowptr must be non-decreasing");
    const int64_t nnz = rp[n];
    if (nnz > ((int64_t)1 << 31) - 1) return fail(SRJ_ERR_INVALID, "too many entries");
    std::vector<int32_t> col((size_t)nnz);
    std::vector<double> val((size_t)nnz);
    if (nnz > 0) {
        chk = check_device_array(p->col, sizeof(int32_t) * col.size(), dev, "col");
        if (chk == SRJ_OK) chk = check_device_array(p->val, sizeof(double) * val.size(), dev, "val");
        if (chk != SRJ_OK) return chk;
        SRJ_HIP_CHECK(hipMemcpy(col.data(), p->col, sizeof(int32_t) * col.size(), hipMemcpyDeviceToHost));
        SRJ_HIP_CHECK(hipMemcpy(val.data(), p->val, sizeof(double) * val.size(), hipMemcpyDeviceToHost));
    }
    // diagonal, 1/D and the off-diagonal entries in storage order (ELL, column-major)
    std::vector<double> d((size_t)n), dinv((size_t)n);
    std::vector<int32_t> len((size_t)n);
    int32_t width = 0;
    for (int64_t i = 0; i < n; ++i) {
        int ndiag = 0;
        int32_t off = 0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (col[k] < 0 || col[k] >= n) return fail(SRJ_ERR_INVALID, "column index out of range");
            if (!isfinite(val[k])) return fail(SRJ_ERR_INVALID, "entries must be finite");
            if (col[k] == i) {
                ++ndiag;
                d[i] = val[k];
            } else {
                ++off;
            }
        }
        if (ndiag != 1) return fail(SRJ_ERR_INVALID, "every row must hold its diagonal exactly once");
        if (!(d[i] > 0.0)) return fail(SRJ_ERR_INVALID, "diagonal entries must be > 0");
        dinv[i] = 1.0 / d[i];
        len[i] = off;
        width = std::max(width, off);
    }
    if ((int64_t)width * n > ((int64_t)1 << 40)) return fail(SRJ_ERR_INVALID, "matrix too wide");
    std::vector<int32_t> ecol((size_t)std::max<int64_t>(1, (int64_t)width * n));
    std::vector<double> evalv(ecol.size(), 0.0);
    for (int64_t i = 0; i < n; ++i) {
        int j = 0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (col[k] != i) {
                ecol[(size_t)j * n + i] = col[k];
                evalv[(size_t)j * n + i] = val[k];
                ++j;
            }
        for (; j < width; ++j) ecol[(size_t)j * n + i] = (int32_t)i;  // never read
    }
    srj_ctx *c = new srj_ctx();
    c->device = dev;
    c->stream = stream;
    c->npoints = n;
    auto nomem = [&](const char *what) {
        srj_destroy(c);
        return fail(SRJ_ERR_NOMEM, std::string("hipMalloc failed for ") + what);
    };
    const size_t bytes = sizeof(double) * (size_t)n;
    if (hipMalloc(&c->ws, bytes) != hipSuccess) return nomem("ping-pong buffer");
    if (hipMalloc(&c->csr_diag, bytes) != hipSuccess || hipMalloc(&c->dinv, bytes) != hipSuccess ||
        hipMalloc(&c->csr_b, bytes) != hipSuccess ||
        hipMalloc(&c->csr_len, sizeof(int32_t) * (size_t)n) != hipSuccess ||
        hipMalloc(&c->csr_col, sizeof(int32_t) * ecol.size()) != hipSuccess ||
        hipMalloc(&c->csr_val, sizeof(double) * evalv.size()) != hipSuccess)
        return nomem("sparse matrix copy");
    hipError_t e = hipMemcpy(c->csr_diag, d.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->dinv, dinv.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->csr_b, p->b, bytes, hipMemcpyDeviceToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->csr_len, len.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->csr_col, ecol.data(), sizeof(int32_t) * ecol.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->csr_val, evalv.data(), sizeof(double) * evalv.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        srj_destroy(c);
        return fail(SRJ_ERR_HIP, std::string("sparse matrix copy: ") + hipGetErrorString(e));
    }
    DevProblem &P = c->P;
    P.ndim = 1;
    P.n0 = n;
    P.n1 = P.n2 = 1;
    P.diag = c->csr_diag;
    P.dinv = c->dinv;
    P.b = c->csr_b;
    P.ell_len = c->csr_len;
    P.ell_col = c->csr_col;
    P.ell_val = c->csr_val;
    P.ell_width = width;
    srj_status st = ctx_finish(c);
    if (st == SRJ_OK) *out = c;
    return st;
}

srj_status srj_set_plan(srj_ctx *c, int32_t which, int32_t kind, int32_t tile_rows,
                        int32_t sweeps_per_launch, int32_t waves_per_simd)
{
    if (!c) return fail(SRJ_ERR_INVALID, "ctx is NULL");
    if (which != 0 && which != 1) return fail(SRJ_ERR_INVALID, "which must be 0 or 1");
    SweepPlan pl;
    pl.kind = kind;
    pl.by = tile_rows;
    pl.T = sweeps_per_launch;
    pl.occ = waves_per_simd;
    SweepPlan &dst = which == 0 ? c->plan : c->plan_inner;
    if (kind == 0) {
        dst = SweepPlan{};
        return SRJ_OK;
    }
    const bool ok = which == 0 ? fused_supported(c->P, pl) : inner_fused_supported(c->P, pl);
    if (!ok) return fail(SRJ_ERR_UNSUPPORTED, "plan not supported for this problem");
    dst = pl;
    return SRJ_OK;
}

srj_status srj_get_plan(srj_ctx *c, int32_t which, int32_t *kind, int32_t *tile_rows,
                        int32_t *sweeps_per_launch, int32_t *waves_per_simd)
{
    if (!c || !kind || !tile_rows || !sweeps_per_launch || !waves_per_simd)
        return fail(SRJ_ERR_INVALID, "NULL argument");
    if (which != 0 && which != 1) return fail(SRJ_ERR_INVALID, "which must be 0 or 1");
    const SweepPlan &pl = which == 0 ? c->plan : c->plan_inner;
    *kind = pl.kind;
    *tile_rows = pl.by;
    *sweeps_per_launch = pl.T;
    *waves_per_simd = pl.occ;
    return SRJ_OK;
}

srj_status srj_set_resident(srj_ctx *c, int32_t enable)
{
    if (!c) return fail(SRJ_ERR_INVALID, "ctx is NULL");
    if (enable && !resident_fits(c->P))
        return fail(SRJ_ERR_UNSUPPORTED, "grid too large for a one-workgroup solve");
    c->resident = enable != 0;
    return SRJ_OK;
}

srj_status srj_plan_variants(int32_t which, int32_t *out, int32_t cap, int32_t *count)
{
    if (!count || (cap > 0 && !out)) return fail(SRJ_ERR_INVALID, "NULL argument");
    if (which != 0 && which != 1) return fail(SRJ_ERR_INVALID, "which must be 0 or 1");
    *count = which == 0 ? plan_variants(out, cap) : inner_plan_variants(out, cap);
    return SRJ_OK;
}

srj_status srj_set_profiling(srj_ctx *c, int32_t enable)
{
    if (!c) return fail(SRJ_ERR_INVALID, "ctx is NULL");
    if (enable && !c->ev0) {
        SRJ_HIP_CHECK(hipEventCreate(&c->ev0));
        SRJ_HIP_CHECK(hipEventCreate(&c->ev1));
    }
    c->profiling = enable != 0;
    c->prof_pending = false;
    c->prof_ms = 0.0;
    c->prof_launches = c->prof_sweeps = 0;
    return SRJ_OK;
}

srj_status srj_get_profile(srj_ctx *c, double *sweep_ms, int64_t *launches, int64_t *sweeps)
{
    if (!c || !sweep_ms || !launches || !sweeps) return fail(SRJ_ERR_INVALID, "NULL argument");
    *sweep_ms = c->prof_ms;
    *launches = c->prof_launches;
    *sweeps = c->prof_sweeps;
    return SRJ_OK;
}

srj_status srj_residual_norm(srj_ctx *c, const double *x, double *norm_out)
{
    if (!c || !x || !norm_out) return fail(SRJ_ERR_INVALID, "NULL argument");
    srj_status st = check_device_array(x, sizeof(double) * (size_t)c->npoints, c->device, "x");
    if (st != SRJ_OK) return st;
    return residual_norm(c, x, norm_out);
}

// Solve with the per-sweep update test (section 4.2.2, Eq. (25)): one sweep
// per launch, sweep g reading buffer g % 2 and writing buffer (g + 1) % 2
// (buffer 0 is x); the selector runs on cycle-end residual ratios as usual.
// After each cycle the host reads the test state: a launch inside the cycle
// may have found that an earlier sweep met the test (later launches then did
// nothing), or the cycle's last sweep met it.
// The update test with fused sweeps (plan kind 10): each launch of T sweeps
// records the largest |x' - x| of each of its sweeps, a check after it finds
// the first sweep below tol, and later launches do nothing.  A launch reads
// one buffer and writes the other, and the launches after the stop write
// nothing, so the input of the launch that held the stop is intact: the
// iterate of the stop sweep is formed again from it (the same sweeps, so the
// same bits) unless the stop is that launch's last sweep.
static srj_status solve_update_inf_fused(srj_ctx *c, double *x, const srj_solve_opts *o,
                                         srj_solve_result *res, int32_t *levels_out,
                                         double *norms_out)
{
    if (!c->updf && hipMalloc(&c->updf, sizeof(UpdFState)) != hipSuccess) {
        c->updf = nullptr;
        return fail(SRJ_ERR_NOMEM, "hipMalloc failed for the update test state");
    }
    if (!c->updf_pub) {
        if (hipHostMalloc((void **)&c->updf_pub, 2 * sizeof(int64_t), 0) != hipSuccess) {
            c->updf_pub = nullptr;
            return fail(SRJ_ERR_NOMEM, "pinned allocation failed for the update test flag");
        }
        if (hipHostGetDevicePointer((void **)&c->updf_pub_dev, c->updf_pub, 0) != hipSuccess) {
            (void)hipHostFree(c->updf_pub);
            c->updf_pub = c->updf_pub_dev = nullptr;
            return fail(SRJ_ERR_HIP, "no device mapping of the update test flag");
        }
    }
    SRJ_HIP_CHECK(hipMemsetAsync(c->updf, 0, sizeof(UpdFState), c->stream));
    SRJ_HIP_CHECK(launch_upd_check(c->updf, 1, 0, 0, o->tol, c->updf_pub_dev, c->stream));  // clears ring 0
    double norm0 = 0.0;
    srj_status st = residual_norm(c, x, &norm0);
    if (st != SRJ_OK) return st;
    res->r0 = o->r0 > 0.0 ? o->r0 : norm0;
    res->r_final = norm0;
    if (norms_out) norms_out[0] = norm0;
    if (!isfinite(norm0)) return fail(SRJ_ERR_NONFINITE, "initial residual norm is not finite");
    if (norm0 == 0.0) {
        res->converged = 1;  // x solves the system: every update is zero
        return SRJ_OK;
    }
    struct Launch {
        int64_t g0;
        int T, done;
        double *in, *out;
    };
    std::vector<Launch> launches;
    srj_status status = SRJ_ERR_NOT_CONVERGED;
    int level = o->start_level;
    double prev = norm0;
    double *cur = x, *nxt = c->ws;
    double *result = x;  // the iterate of the last sweep that counts
    int64_t g = 0;       // sweeps enqueued
    int64_t nl = 0;      // launches enqueued
    for (int cycle = 0; cycle < o->max_cycles; ++cycle) {
        const int lv = o->rule == SRJ_RULE_FIXED ? o->fixed_level : level;
        const int M = static_cast<int>(c->factors[lv].size());
        if (g + M > o->max_sweeps) break;
        const double *wdev = c->omega_dev + c->offsets[lv];
        launches.clear();
        for (int done = 0; done < M; ++nl) {
            const int T = std::min(c->plan.T, M - done);
            const int ring = (int)(nl & 1);
            SRJ_HIP_CHECK(launch_sweep_fused_upd(c->P, c->plan, cur, nxt, wdev + done, T, c->updf,
                                                 ring, c->stream, c->reverse));
            SRJ_HIP_CHECK(launch_upd_check(c->updf, ring, T, g, o->tol, c->updf_pub_dev, c->stream));
            c->reverse = !c->reverse;
            launches.push_back({g, T, done, cur, nxt});
            std::swap(cur, nxt);
            g += T;
            done += T;
        }
        double norm = 0.0;
        st = residual_norm(c, cur, &norm);  // synchronises the stream
        if (st != SRJ_OK) return st;
        // the cycle's last k_upd_check left flag and stop in pinned memory
        const int32_t flag = (int32_t)c->updf_pub[0];
        const int64_t stop = flag ? c->updf_pub[1] : -1;
        res->cycles = cycle + 1;
        res->final_level = lv;
        if (levels_out) levels_out[cycle] = lv;
        if (flag) {
            const Launch *hit = nullptr;
            for (const Launch &L : launches)
                if (stop >= L.g0 && stop < L.g0 + L.T) hit = &L;
            if (!hit) return fail(SRJ_ERR_HIP, "update test stop outside the cycle's launches");
            result = hit->out;
            const int Tstop = (int)(stop - hit->g0) + 1;
            if (Tstop != hit->T || hit != &launches.back()) {
                if (Tstop != hit->T)  // the stop sweep's iterate, formed again
                    SRJ_HIP_CHECK(launch_sweep_fused(c->P, c->plan, hit->in, hit->out,
                                                     wdev + hit->done, Tstop, c->stream,
                                                     c->reverse));
                st = residual_norm(c, result, &norm);
                if (st != SRJ_OK) return st;
            }
            res->sweeps = stop + 1;
            res->r_final = norm;
            if (norms_out) norms_out[cycle + 1] = norm;
            res->converged = 1;
            status = SRJ_OK;
            break;
        }
        result = cur;
        res->sweeps = g;
        res->r_final = norm;
        if (norms_out) norms_out[cycle + 1] = norm;
        if (!isfinite(norm)) {
            status = fail(SRJ_ERR_NONFINITE, "residual norm is not finite");
            break;
        }
        const double ratio = norm / prev;
        prev = norm;
        if (o->rule == SRJ_RULE_HEURISTIC) {
            const double m = std::min(fabs(ratio - 0.2), fabs(ratio - 0.4));
            res->min_margin = std::min(res->min_margin, m);
        }
        level = next_level(o->rule, level, ratio, o->max_level);
    }
    if (status == SRJ_ERR_NOT_CONVERGED) set_error("cycle or sweep cap reached");
    if (result != x)
        SRJ_HIP_CHECK(hipMemcpyAsync(x, result, sizeof(double) * (size_t)c->npoints,
                                     hipMemcpyDeviceToDevice, c->stream));
    SRJ_HIP_CHECK(hipStreamSynchronize(c->stream));
    return status;
}

static srj_status solve_update_inf(srj_ctx *c, double *x, const srj_solve_opts *o, srj_solve_result *res,
                                   int32_t *levels_out, double *norms_out)
{
    if (c->plan.kind != 0 && fused_upd_supported(c->P, c->plan))
        return solve_update_inf_fused(c, x, o, res, levels_out, norms_out);
    if (!c->upd && hipMalloc(&c->upd, sizeof(UpdState)) != hipSuccess) {
        c->upd = nullptr;
        return fail(SRJ_ERR_NOMEM, "hipMalloc failed for the update test state");
    }
    SRJ_HIP_CHECK(hipMemsetAsync(c->upd, 0, sizeof(UpdState), c->stream));
    double *buf[2] = {x, c->ws};
    double norm0 = 0.0;
    srj_status st = residual_norm(c, x, &norm0);
    if (st != SRJ_OK) return st;
    res->r0 = o->r0 > 0.0 ? o->r0 : norm0;
    res->r_final = norm0;
    if (norms_out) norms_out[0] = norm0;
    if (!isfinite(norm0)) return fail(SRJ_ERR_NONFINITE, "initial residual norm is not finite");
    if (norm0 == 0.0) {
        res->converged = 1;  // x solves the system: every update is zero
        return SRJ_OK;
    }
    srj_status status = SRJ_ERR_NOT_CONVERGED;
    int level = o->start_level;
    double prev = norm0;
    int64_t g = 0;       // sweeps enqueued
    int64_t last = -1;   // the sweep whose iterate is the result
    for (int cycle = 0; cycle < o->max_cycles; ++cycle) {
        const int lv = o->rule == SRJ_RULE_FIXED ? o->fixed_level : level;
        const std::vector<double> &w = c->factors[lv];
        const int M = static_cast<int>(w.size());
        if (g + M > o->max_sweeps) break;
        for (int k = 0; k < M; ++k, ++g)
            SRJ_HIP_CHECK(launch_sweep_upd(c->P, buf[g % 2], buf[(g + 1) % 2], w[k], o->tol, c->upd,
                                           g, c->stream));
        double norm = 0.0;
        st = residual_norm(c, buf[g % 2], &norm);  // synchronises the stream
        if (st != SRJ_OK) return st;
        static thread_local UpdState h;
        SRJ_HIP_CHECK(hipMemcpy(&h, c->upd, sizeof(h), hipMemcpyDeviceToHost));
        unsigned long long lastmax = 0;  // fold the stripes of the cycle's last sweep
        for (int k = 0; k < kUpdStripes; ++k)
            lastmax = std::max(lastmax, h.maxbits[((g - 1) % 3) * kUpdStripes * kUpdStride + k * kUpdStride]);
        int64_t stop = -1;
        if (h.flag)
            stop = h.stop;
        else if (__builtin_bit_cast(double, lastmax) < o->tol)
            stop = g - 1;
        res->cycles = cycle + 1;
        res->final_level = lv;
        if (levels_out) levels_out[cycle] = lv;
        if (stop >= 0) {
            last = stop;
            res->sweeps = stop + 1;
            if (stop != g - 1) {  // the cycle-end norm belongs to a later, skipped sweep
                st = residual_norm(c, buf[(stop + 1) % 2], &norm);
                if (st != SRJ_OK) return st;
            }
            res->r_final = norm;
            if (norms_out) norms_out[cycle + 1] = norm;
            res->converged = 1;
            status = SRJ_OK;
            break;
        }
        last = g - 1;
        res->sweeps = g;
        res->r_final = norm;
        if (norms_out) norms_out[cycle + 1] = norm;
        if (!isfinite(norm)) {
            status = fail(SRJ_ERR_NONFINITE, "residual norm is not finite");
            break;
        }
        const double ratio = norm / prev;
        prev = norm;
        if (o->rule == SRJ_RULE_HEURISTIC) {
            const double m = std::min(fabs(ratio - 0.2), fabs(ratio - 0.4));
            res->min_margin = std::min(res->min_margin, m);
        }
        level = next_level(o->rule, level, ratio, o->max_level);
    }
    if (status == SRJ_ERR_NOT_CONVERGED) set_error("cycle or sweep cap reached");
    double *result = last >= 0 ? buf[(last + 1) % 2] : x;
    if (result != x)
        SRJ_HIP_CHECK(hipMemcpyAsync(x, result, sizeof(double) * (size_t)c->npoints,
                                     hipMemcpyDeviceToDevice, c->stream));
    SRJ_HIP_CHECK(hipStreamSynchronize(c->stream));
    return status;
}

srj_status srj_run_cycle(srj_ctx *c, double *x, int32_t level, double *resnorm_out)
{
    if (!c || !x || !resnorm_out) return fail(SRJ_ERR_INVALID, "NULL argument");
    if (level < 0 || level >= c->nlevels) return fail(SRJ_ERR_INVALID, "level outside the scheme family");
    srj_status chk = check_device_array(x, sizeof(double) * (size_t)c->npoints, c->device, "x");
    if (chk != SRJ_OK) return chk;
    double *cur = x, *nxt = c->ws;
    srj_status st = run_sweeps(c, &cur, &nxt, level);
    if (st != SRJ_OK) return st;
    if (cur != x)
        SRJ_HIP_CHECK(hipMemcpyAsync(x, cur, sizeof(double) * (size_t)c->npoints,
                                     hipMemcpyDeviceToDevice, c->stream));
    return residual_norm(c, x, resnorm_out);
}

static srj_status solve_dispatch(srj_ctx *c, double *x, const srj_solve_opts *o,
                                 srj_solve_result *res, int32_t *levels_out, double *norms_out);

srj_status srj_solve(srj_ctx *c, double *x, const srj_solve_opts *o, srj_solve_result *res,
                     int32_t *levels_out, double *norms_out)
{
    // the per-cycle log (SRJ_LOG) needs the histories: the solve then fills
    // arrays of its own where the caller passes none
    if (!log_enabled() || !c || !x || !o || !res || o->max_cycles < 1 || o->max_cycles > (1 << 24))
        return solve_dispatch(c, x, o, res, levels_out, norms_out);
    std::vector<int32_t> lv;
    std::vector<double> nv;
    if (!levels_out) {
        lv.resize((size_t)o->max_cycles);
        levels_out = lv.data();
    }
    if (!norms_out) {
        nv.resize((size_t)o->max_cycles + 1);
        norms_out = nv.data();
    }
    const srj_status st = solve_dispatch(c, x, o, res, levels_out, norms_out);
    if (st == SRJ_OK || st == SRJ_ERR_NOT_CONVERGED || st == SRJ_ERR_NONFINITE)
        log_cycles("solve", st, res->cycles, levels_out, c->levelM.data(), (int)c->levelM.size(),
                   norms_out, res->sweeps, res->r0, res->r_final);
    return st;
}

static srj_status solve_dispatch(srj_ctx *c, double *x, const srj_solve_opts *o,
                                 srj_solve_result *res, int32_t *levels_out, double *norms_out)
{
    if (!c || !x || !res) return fail(SRJ_ERR_INVALID, "NULL argument");
    srj_status st = validate_opts(o);
    if (st != SRJ_OK) return st;
    st = check_device_array(x, sizeof(double) * (size_t)c->npoints, c->device, "x");
    if (st != SRJ_OK) return st;
    // the context's scheme family bounds the levels: the top level is clamped
    // to it, a start or fixed level beyond it is an error
    if (o->start_level >= c->nlevels || (o->rule == SRJ_RULE_FIXED && o->fixed_level >= c->nlevels))
        return fail(SRJ_ERR_INVALID, "level outside the scheme family");
    srj_solve_opts oc = *o;
    oc.max_level = std::min(o->max_level, c->nlevels - 1);
    o = &oc;
    memset(res, 0, sizeof(*res));
    res->min_margin = INFINITY;
    if (c->P.ell_len && (o->precision != SRJ_PREC_F64 || o->tol_mode == SRJ_TOL_UPDATE_INF))
        return fail(SRJ_ERR_UNSUPPORTED, "general sparse matrices take binary64 and a residual test");
    if (o->tol_mode == SRJ_TOL_UPDATE_INF) {
        if (o->precision != SRJ_PREC_F64)
            return fail(SRJ_ERR_UNSUPPORTED, "the update test needs precision F64");
        if (c->resident && resident_fits(c->P))
            return resident_solve(c, x, o, res, levels_out, norms_out);
        return solve_update_inf(c, x, o, res, levels_out, norms_out);
    }
    if (o->precision != SRJ_PREC_F64) return refine_solve(c, x, o, res, levels_out, norms_out);
    if (c->resident && resident_fits(c->P)) return resident_solve(c, x, o, res, levels_out, norms_out);

    double *cur = x, *nxt = c->ws;
    double norm0 = 0.0;
    st = residual_norm(c, x, &norm0);
    if (st != SRJ_OK) return st;
    const double r0 = o->r0 > 0.0 ? o->r0 : norm0;
    res->r0 = r0;
    res->r_final = norm0;
    if (norms_out) norms_out[0] = norm0;
    const double target = o->tol_mode == SRJ_TOL_RELATIVE ? o->tol * r0 : o->tol;
    srj_status status = SRJ_ERR_NOT_CONVERGED;
    int level = o->start_level;
    double prev = norm0;
    if (!isfinite(norm0)) {
        status = fail(SRJ_ERR_NONFINITE, "initial residual norm is not finite");
    } else if (norm0 == 0.0 || norm0 < target) {
        res->converged = 1;
        status = SRJ_OK;
    } else {
        for (int cycle = 0; cycle < o->max_cycles; ++cycle) {
            const int lv = o->rule == SRJ_RULE_FIXED ? o->fixed_level : level;
            const int M = c->levelM[lv];
            if (res->sweeps + M > o->max_sweeps) break;
            st = run_sweeps(c, &cur, &nxt, lv);
            if (st != SRJ_OK) return st;
            res->sweeps += M;
            double norm = 0.0;
            st = residual_norm(c, cur, &norm);
            if (st != SRJ_OK) return st;
            res->cycles = cycle + 1;
            res->r_final = norm;
            res->final_level = lv;
            if (levels_out) levels_out[cycle] = lv;
            if (norms_out) norms_out[cycle + 1] = norm;
            if (!isfinite(norm)) {
                status = fail(SRJ_ERR_NONFINITE, "residual norm is not finite");
                break;
            }
            if (norm < target) {
                res->converged = 1;
                status = SRJ_OK;
                break;
            }
            const double ratio = norm / prev;
            prev = norm;
            if (o->rule == SRJ_RULE_HEURISTIC) {
                const double m = std::min(fabs(ratio - 0.2), fabs(ratio - 0.4));
                res->min_margin = std::min(res->min_margin, m);
            }
            level = next_level(o->rule, level, ratio, o->max_level);
        }
        if (status == SRJ_ERR_NOT_CONVERGED) set_error("cycle or sweep cap reached");
    }
    if (cur != x)
        SRJ_HIP_CHECK(hipMemcpyAsync(x, cur, sizeof(double) * (size_t)c->npoints,
                                     hipMemcpyDeviceToDevice, c->stream));
    SRJ_HIP_CHECK(hipStreamSynchronize(c->stream));
    return status;
}

}  // extern "C"
