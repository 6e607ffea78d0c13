// Autotuner: times every kernel plan that fits a problem on the problem
// itself (HIP events on the context's stream), keeps the fastest, and
// remembers the choice per GPU architecture, CU count and problem shape class
// in a text cache (file named by the SRJ_TUNE_CACHE environment variable;
// one "key kind rows sweeps occupancy us_per_sweep" line per entry).  Every
// plan gives bit-identical iterates, so tuning never changes results.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace srj {

namespace {

std::mutex g_tune_mu;

std::string arch_tag()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string arch(prop.gcnArchName);
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    return arch + "_cu" + std::to_string(prop.multiProcessorCount);
}

int size_class(int64_t n)
{
    int k = 0;
    while ((int64_t(1) << k) < n) ++k;
    return k;
}

std::map<std::string, std::pair<SweepPlan, double>> load_cache(const char *path)
{
    std::map<std::string, std::pair<SweepPlan, double>> m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        SweepPlan p;
        double us = 0.0;
        if (is >> key >> p.kind >> p.by >> p.T >> p.occ >> us) m[key] = {p, us};
    }
    return m;
}

}  // namespace

std::string tune_key(const char *what, int which, int ndim, const int64_t n[3], bool faces,
                     bool diag)
{
    std::ostringstream os;
    os << arch_tag() << '/' << what << "/w" << which << "/d" << ndim << "/n" << size_class(n[0])
       << 'x' << size_class(n[1]) << 'x' << size_class(n[2]) << "/f" << (faces ? 1 : 0) << "/g"
       << (diag ? 1 : 0);
    return os.str();
}

bool tune_cache_get(const std::string &key, SweepPlan &plan, double &us)
{
    const char *path = getenv("SRJ_TUNE_CACHE");
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto m = load_cache(path);
    auto it = m.find(key);
    if (it == m.end()) return false;
    plan = it->second.first;
    us = it->second.second;
    return true;
}

void tune_cache_put(const std::string &key, const SweepPlan &plan, double us)
{
    const char *path = getenv("SRJ_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto m = load_cache(path);
    m[key] = {plan, us};
    std::ofstream f(path, std::ios::trunc);
    for (const auto &kv : m)
        f << kv.first << ' ' << kv.second.first.kind << ' ' << kv.second.first.by << ' '
          << kv.second.first.T << ' ' << kv.second.first.occ << ' ' << kv.second.second << '\n';
}

}  // namespace srj

using namespace srj;

namespace {

// Candidate plans for `which`: one sweep per launch plus every fused variant
// that fits, at its full halo and at about half of it.
std::vector<SweepPlan> candidates(srj_ctx *c, int which)
{
    std::vector<SweepPlan> out;
    out.push_back(SweepPlan{});
    std::vector<int32_t> v(4 * 256);
    const int n = which == 0 ? plan_variants(v.data(), 256) : inner_plan_variants(v.data(), 256);
    for (int i = 0; i < n && i < 256; ++i) {
        const int kind = v[4 * i], rows = v[4 * i + 1], halo = v[4 * i + 2], occ = v[4 * i + 3];
        for (int T : {halo, (halo + 1) / 2}) {
            SweepPlan p;
            p.kind = kind;
            p.by = rows;
            p.T = T;
            p.occ = occ;
            const bool ok = which == 0 ? fused_supported(c->P, p) : inner_fused_supported(c->P, p);
            bool dup = false;
            for (const SweepPlan &q : out)
                dup = dup || (q.kind == p.kind && q.by == p.by && q.T == p.T && q.occ == p.occ);
            if (ok && !dup) out.push_back(p);
        }
    }
    return out;
}

srj_status time_f64_plan(srj_ctx *c, const SweepPlan &plan, int sweeps, double *scratch,
                         const double *w_dev, float *ms)
{
    const bool fused = plan.kind != 0;
    double *a = c->ws, *b = scratch;
    SRJ_HIP_CHECK(hipMemsetAsync(a, 0, sizeof(double) * (size_t)c->npoints, c->stream));
    bool reverse = false;
    auto run = [&](int n) -> srj_status {
        for (int done = 0; done < n;) {
            const int T = fused ? std::min(plan.T, n - done) : 1;
            if (fused) {
                SRJ_HIP_CHECK(launch_sweep_fused(c->P, plan, a, b, w_dev, T, c->stream, reverse));
                reverse = !reverse;
            } else {
                SRJ_HIP_CHECK(launch_sweep_generic(c->P, a, b, 2.0 / 3.0, c->stream));
            }
            std::swap(a, b);
            done += T;
        }
        return SRJ_OK;
    };
    srj_status st = run(fused ? plan.T : 1);  // warm-up
    if (st != SRJ_OK) return st;
    SRJ_HIP_CHECK(hipEventRecord(c->ev0, c->stream));
    st = run(sweeps);
    if (st != SRJ_OK) return st;
    SRJ_HIP_CHECK(hipEventRecord(c->ev1, c->stream));
    SRJ_HIP_CHECK(hipEventSynchronize(c->ev1));
    SRJ_HIP_CHECK(hipEventElapsedTime(ms, c->ev0, c->ev1));
    return SRJ_OK;
}

}  // namespace

extern "C" srj_status srj_autotune(srj_ctx *c, int32_t which, int32_t sweeps, int32_t use_cache,
                                   double *best_us_per_sweep)
{
    if (!c || !best_us_per_sweep) return fail(SRJ_ERR_INVALID, "NULL argument");
    if (which != 0 && which != 1) return fail(SRJ_ERR_INVALID, "which must be 0 or 1");
    if (sweeps < 1 || sweeps > 100000) return fail(SRJ_ERR_INVALID, "sweeps must be 1..100000");
    const int64_t n[3] = {c->P.n0, c->P.n1, c->P.n2};
    const bool faces = c->P.face[0] || c->P.face[1] || c->P.face[2];
    const std::string key = tune_key("single", which, c->P.ndim, n, faces, c->P.diag != nullptr);
    SweepPlan cached;
    double cached_us = 0.0;
    if (use_cache && tune_cache_get(key, cached, cached_us)) {
        const bool ok = cached.kind == 0 ||
                        (which == 0 ? fused_supported(c->P, cached) : inner_fused_supported(c->P, cached));
        if (ok) {
            (which == 0 ? c->plan : c->plan_inner) = cached;
            *best_us_per_sweep = cached_us;
            return SRJ_OK;
        }
    }
    const bool had_profiling = c->profiling;
    if (!c->ev0) {
        SRJ_HIP_CHECK(hipEventCreate(&c->ev0));
        SRJ_HIP_CHECK(hipEventCreate(&c->ev1));
    }
    c->profiling = false;  // the events are used for timing here
    // factors: the same value repeated (a contraction, so the scratch iterate stays bounded)
    double *w64 = nullptr, *scratch = nullptr;
    float *w32 = nullptr;
    std::vector<double> wl(64, 2.0 / 3.0);
    std::vector<float> wf(64, static_cast<float>(2.0 / 3.0));
    srj_status st = SRJ_OK;
    if (hipMalloc(&w64, sizeof(double) * 64) != hipSuccess ||
        hipMalloc(&w32, sizeof(float) * 64) != hipSuccess ||
        (which == 0 && hipMalloc(&scratch, sizeof(double) * (size_t)c->npoints) != hipSuccess))
        st = fail(SRJ_ERR_NOMEM, "autotune scratch");
    if (st == SRJ_OK &&
        (hipMemcpyAsync(w64, wl.data(), sizeof(double) * 64, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
         hipMemcpyAsync(w32, wf.data(), sizeof(float) * 64, hipMemcpyHostToDevice, c->stream) != hipSuccess))
        st = fail(SRJ_ERR_HIP, "autotune upload");
    SweepPlan best;
    double best_us = INFINITY;
    if (st == SRJ_OK) {
        for (const SweepPlan &p : candidates(c, which)) {
            float ms = 0.f;
            st = which == 0 ? time_f64_plan(c, p, sweeps, scratch, w64, &ms)
                            : time_inner_plan(c, p, sweeps, w32, &ms);
            if (st != SRJ_OK) break;
            const double us = 1e3 * ms / sweeps;
            if (us < best_us) {
                best_us = us;
                best = p;
            }
        }
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(w64);
    (void)hipFree(w32);
    (void)hipFree(scratch);
    c->profiling = had_profiling;
    if (st != SRJ_OK) return st;
    (which == 0 ? c->plan : c->plan_inner) = best;
    *best_us_per_sweep = best_us;
    tune_cache_put(key, best, best_us);
    return SRJ_OK;
}
