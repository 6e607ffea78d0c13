// Mixed-precision iterative refinement (binary32 / 16-bit inner SRJ cycles).
#include "internal.h"

struct srj_ctx;

namespace srj {

srj_status refine_solve(srj_ctx *, double *, const srj_solve_opts *, srj_solve_result *,
                        int32_t *, double *)
{
    return fail(SRJ_ERR_UNSUPPORTED, "refinement modes are not built yet");
}

void refine_free(srj_ctx *) {}

}  // namespace srj
