// Per-cycle solve log, switched on by the environment variable SRJ_LOG.
//
// For every cycle a solve ran, one line gives the level Algorithm 1 used, its
// number of sweeps M, the cycle-end residual norm, the ratio to the previous
// norm (the quantity Algorithm 1 compares with 0.2 and 0.4, section 3) and
// the cycle's average convergence rate per sweep as section 3 defines it for
// the training data, -log(ratio) / M; a last line gives the status and the
// counters.  SRJ_LOG=1 or
// SRJ_LOG=stderr writes to standard error, any other value except 0 names a
// file that lines are appended to.  The lines are formed from the level and
// norm histories a solve returns, after it has ended, so the solve itself is
// unchanged.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "internal.h"

namespace srj {

namespace {

std::mutex g_log_mu;

// the stream named by SRJ_LOG, or null when logging is off; *close is set
// when the caller must fclose it
FILE *log_open(bool *close)
{
    *close = false;
    const char *v = getenv("SRJ_LOG");
    if (!v || !*v || strcmp(v, "0") == 0) return nullptr;
    if (strcmp(v, "1") == 0 || strcmp(v, "stderr") == 0) return stderr;
    FILE *f = fopen(v, "a");
    if (f) *close = true;
    return f;
}

}  // namespace

bool log_enabled()
{
    const char *v = getenv("SRJ_LOG");
    return v && *v && strcmp(v, "0") != 0;
}

void log_cycles(const char *what, srj_status st, int cycles, const int32_t *levels,
                const int32_t *level_sweeps, int nlevels, const double *norms, int64_t sweeps,
                double r0, double r_final)
{
    std::lock_guard<std::mutex> lock(g_log_mu);
    bool close = false;
    FILE *f = log_open(&close);
    if (!f) return;
    for (int k = 0; k < cycles; ++k) {
        const int lv = levels[k];
        const int M = lv >= 0 && lv < nlevels ? level_sweeps[lv] : 0;
        const double ratio = norms[k] > 0.0 ? norms[k + 1] / norms[k] : NAN;
        const double rate = M > 0 && ratio > 0.0 ? -log(ratio) / M : NAN;
        fprintf(f, "srj %s: cycle %d level %d sweeps %d norm %.17g ratio %.6g rate %.6g\n", what,
                k, lv, M, norms[k + 1], ratio, rate);
    }
    fprintf(f, "srj %s: status %d cycles %d sweeps %lld r0 %.17g r_final %.17g\n", what, (int)st,
            cycles, (long long)sweeps, r0, r_final);
    if (close) fclose(f);
}

}  // namespace srj
