/* A plain C consumer of the library's C ABI (include/srj.h): device memory
 * from the HIP runtime, no Python.  Solves the 2D Poisson problem of
 * n0 x n1 interior points on the unit square (couplings (n_d + 1)^2, D their
 * doubled sum) with b_p = 1 + 0.001 (p mod 7), x0 = 0, to a relative
 * residual tol (Algorithm 1 level choice, default options otherwise), and
 * prints the result in a fixed text form:
 *   status <s> converged <c> cycles <k> sweeps <m>
 *   r0 <r0> r_final <r>            (%.17g)
 *   levels <l1> <l2> ...
 *   sum <sum of x in index order>  (%.17g)
 * Usage: solve_c n0 n1 tol.  Exit status 0 on SRJ_OK, 1 otherwise, 2 on a
 * usage or HIP error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "srj.h"

#define MAX_CYCLES 400

int main(int argc, char **argv)
{
    if (argc != 4) {
        fprintf(stderr, "usage: solve_c n0 n1 tol\n");
        return 2;
    }
    const int64_t n0 = atoll(argv[1]), n1 = atoll(argv[2]);
    const double tol = atof(argv[3]);
    if (n0 < 1 || n1 < 1 || n0 * n1 > ((int64_t)1 << 26) || !(tol > 0.0)) {
        fprintf(stderr, "bad arguments\n");
        return 2;
    }
    const size_t n = (size_t)(n0 * n1);
    double *hb = malloc(n * sizeof(double));
    double *hx = malloc(n * sizeof(double));
    if (!hb || !hx) return 2;
    for (size_t p = 0; p < n; ++p) hb[p] = 1.0 + 0.001 * (double)(p % 7);
    double *db = NULL, *dx = NULL;
    if (hipMalloc((void **)&db, n * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&dx, n * sizeof(double)) != hipSuccess ||
        hipMemcpy(db, hb, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(dx, 0, n * sizeof(double)) != hipSuccess) {
        fprintf(stderr, "HIP allocation or copy failed\n");
        return 2;
    }
    srj_problem prob = {0};
    prob.ndim = 2;
    prob.n[0] = n0;
    prob.n[1] = n1;
    prob.n[2] = 1;
    prob.cconst[0] = (double)((n0 + 1) * (n0 + 1));
    prob.cconst[1] = (double)((n1 + 1) * (n1 + 1));
    prob.dconst = 2.0 * (prob.cconst[0] + prob.cconst[1]);
    prob.b = db;
    srj_ctx *ctx = NULL;
    srj_status st = srj_setup(&prob, NULL, &ctx);
    if (st != SRJ_OK) {
        fprintf(stderr, "srj_setup: %d %s\n", (int)st, srj_last_error());
        return 1;
    }
    srj_solve_opts opts;
    srj_default_opts(&opts);
    opts.tol = tol;
    opts.max_cycles = MAX_CYCLES;
    srj_solve_result res;
    int32_t levels[MAX_CYCLES];
    double norms[MAX_CYCLES + 1];
    st = srj_solve(ctx, dx, &opts, &res, levels, norms);
    printf("status %d converged %d cycles %d sweeps %lld\n", (int)st, (int)res.converged,
           (int)res.cycles, (long long)res.sweeps);
    printf("r0 %.17g r_final %.17g\n", res.r0, res.r_final);
    printf("levels");
    for (int k = 0; k < res.cycles; ++k) printf(" %d", (int)levels[k]);
    printf("\n");
    if (hipMemcpy(hx, dx, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 2;
    double sum = 0.0;
    for (size_t p = 0; p < n; ++p) sum += hx[p];
    printf("sum %.17g\n", sum);
    srj_destroy(ctx);
    hipFree(dx);
    hipFree(db);
    free(hb);
    free(hx);
    return st == SRJ_OK ? 0 : 1;
}
