// Batched solves of many independent problems.
#include "internal.h"

extern "C" {

srj_status srj_batch_setup(int32_t, const srj_problem *, void *, srj_batch **out)
{
    if (out) *out = nullptr;
    return srj::fail(SRJ_ERR_UNSUPPORTED, "batched solves are not built yet");
}

srj_status srj_batch_solve(srj_batch *, double *const *, const srj_solve_opts *, srj_solve_result *,
                           int32_t *)
{
    return srj::fail(SRJ_ERR_UNSUPPORTED, "batched solves are not built yet");
}

srj_status srj_batch_destroy(srj_batch *) { return SRJ_OK; }

}
