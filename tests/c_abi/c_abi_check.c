/*
 * c_abi_check.c -- a plain C client of liblbm (no Python, no C++): the
 * library's interface used exactly as a C program would use it, checked against
 * closed forms on the GPU.  Built by the repository's build step; run by
 * tests/test_gpu_c_abi.py.  Exit status 0 when every check holds.
 *
 *  1. Uniform flow is a fixed point of streaming plus collision (Eqs. 1-5), and
 *     mass and momentum are conserved (Eq. 1) up to the rounding of the FP32
 *     store.
 *  2. One solid sample at rest in a uniform stream U (rho = 1): the trilinear
 *     interpolation of a constant is the constant, so the penalty force of
 *     Eq. 7 with gain gamma and area a totals F = -a gamma U, and the torque
 *     about the coordinate origin is x_s x F (Alg. 2 (c)).
 *  3. Invalid calls return their error codes and leave a message.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "lbm.h"

static int failures = 0;

#define HIP_OK(x)                                                                 \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "c-abi: %s failed: %s\n", #x, hipGetErrorString(e_)); \
            exit(2);                                                              \
        }                                                                         \
    } while (0)
#define LBM_OK_(ctx, x)                                                                          \
    do {                                                                                         \
        lbm_status s_ = (x);                                                                     \
        if (s_ != LBM_OK) {                                                                      \
            fprintf(stderr, "c-abi: %s returned %d: %s\n", #x, (int)s_, lbm_last_error(ctx));    \
            exit(2);                                                                             \
        }                                                                                        \
    } while (0)

static void check(int ok, const char *what, double got, double want)
{
    printf("c-abi: %-52s got % .9e want % .9e  %s\n", what, got, want, ok ? "ok" : "FAIL");
    if (!ok) failures++;
}

static void uniform_state(lbm_ctx *ctx, int N, float ux, float uy, float uz, float *rho_d, float *u_d)
{
    float *rho = (float *)malloc(sizeof(float) * N), *u = (float *)malloc(sizeof(float) * 3 * N);
    for (int k = 0; k < N; ++k) {
        rho[k] = 1.0f;
        u[k] = ux;
        u[N + k] = uy;
        u[2 * N + k] = uz;
    }
    HIP_OK(hipMemcpy(rho_d, rho, sizeof(float) * N, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(u_d, u, sizeof(float) * 3 * N, hipMemcpyHostToDevice));
    LBM_OK_(ctx, lbm_init_equilibrium(ctx, rho_d, u_d));
    free(rho);
    free(u);
}

int main(void)
{
    const int nx = 24, ny = 16, nz = 12, N = nx * ny * nz;
    lbm_params p;
    LBM_OK_(NULL, lbm_default_params(&p, nx, ny, nz, 0.02));
    size_t bytes = 0;
    LBM_OK_(NULL, lbm_workspace_size(&p, &bytes));
    void *ws = NULL;
    HIP_OK(hipMalloc(&ws, bytes));
    hipStream_t st;
    HIP_OK(hipStreamCreate(&st));
    lbm_ctx *ctx = NULL;
    LBM_OK_(NULL, lbm_create(&p, ws, bytes, (void *)st, &ctx));
    float *rho_d = NULL, *u_d = NULL;
    HIP_OK(hipMalloc((void **)&rho_d, sizeof(float) * N));
    HIP_OK(hipMalloc((void **)&u_d, sizeof(float) * 3 * N));

    /* 1. uniform flow: fixed point, conservation */
    const float U0[3] = {0.05f, 0.02f, -0.01f};
    uniform_state(ctx, N, U0[0], U0[1], U0[2], rho_d, u_d);
    double c0[4], c1[4];
    LBM_OK_(ctx, lbm_conserved(ctx, c0));
    LBM_OK_(ctx, lbm_step(ctx, 50));
    LBM_OK_(ctx, lbm_conserved(ctx, c1));
    LBM_OK_(ctx, lbm_macros(ctx, rho_d, u_d));
    float *rho = (float *)malloc(sizeof(float) * N), *u = (float *)malloc(sizeof(float) * 3 * N);
    HIP_OK(hipStreamSynchronize(st));
    HIP_OK(hipMemcpy(rho, rho_d, sizeof(float) * N, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(u, u_d, sizeof(float) * 3 * N, hipMemcpyDeviceToHost));
    double du = 0.0, dr = 0.0;
    for (int k = 0; k < N; ++k) {
        dr = fmax(dr, fabs(rho[k] - 1.0));
        for (int a = 0; a < 3; ++a) du = fmax(du, fabs(u[a * N + k] - U0[a]));
    }
    check(du <= 1e-6, "uniform flow, 50 steps: max |u - U|", du, 0.0);
    check(dr <= 1e-6, "uniform flow, 50 steps: max |rho - 1|", dr, 0.0);
    /* the collision conserves them exactly; the FP32 store rounds each of the
     * N*27 deviations every step, so the totals may drift by at most
     * N*27*steps*2^-24*max|d| (about 4e-6 of the mass here): gate 1e-7 */
    check(fabs(c1[0] - c0[0]) <= 1e-7 * c0[0], "mass after 50 steps", c1[0], c0[0]);
    for (int a = 1; a < 4; ++a) check(fabs(c1[a] - c0[a]) <= 1e-7 * c0[0], "momentum component after 50 steps", c1[a], c0[a]);

    /* 2. one sample at rest in a uniform stream */
    const float U = 0.05f, area = 0.7f, gain = 1.3f;
    const float xs[3] = {10.25f, 7.5f, 4.75f};
    uniform_state(ctx, N, U, 0.0f, 0.0f, rho_d, u_d);
    float *smp_d = NULL;
    HIP_OK(hipMalloc((void **)&smp_d, sizeof(float) * 8));
    const float smp[8] = {xs[0], xs[1], xs[2], 0.0f, 0.0f, 0.0f, area, gain};  /* xyz, ub, area, gain */
    HIP_OK(hipMemcpy(smp_d, smp, sizeof(smp), hipMemcpyHostToDevice));
    size_t mbytes = 0;
    LBM_OK_(ctx, lbm_solids_ws_size(ctx, 1, &mbytes));
    void *mws = NULL;
    HIP_OK(hipMalloc(&mws, mbytes));
    LBM_OK_(ctx, lbm_set_solids(ctx, 1, smp_d, smp_d + 3, smp_d + 6, smp_d + 7, mws, mbytes));
    LBM_OK_(ctx, lbm_step(ctx, 1));
    double F[3], T[3];
    LBM_OK_(ctx, lbm_ib_force(ctx, F));
    LBM_OK_(ctx, lbm_ib_torque(ctx, T));
    const double Fx = -(double)area * gain * U;
    check(fabs(F[0] - Fx) <= 1e-5 * fabs(Fx), "sample force F_x = -a gamma U", F[0], Fx);
    check(fabs(F[1]) <= 1e-7 && fabs(F[2]) <= 1e-7, "sample force F_y, F_z = 0 (largest shown)", fmax(fabs(F[1]), fabs(F[2])), 0.0);
    check(fabs(T[1] - xs[2] * Fx) <= 1e-5 * fabs(xs[2] * Fx), "torque T_y = z_s F_x", T[1], xs[2] * Fx);
    check(fabs(T[2] + xs[1] * Fx) <= 1e-5 * fabs(xs[1] * Fx), "torque T_z = -y_s F_x", T[2], -xs[1] * Fx);

    /* 3. error paths */
    check(lbm_step(ctx, -1) == LBM_E_INVAL && strlen(lbm_last_error(ctx)) > 0, "lbm_step(-1) -> LBM_E_INVAL", 0, 0);
    check(lbm_set_solids(ctx, 1, smp_d, NULL, NULL, NULL, (char *)mws + 4, mbytes) == LBM_E_INVAL,
          "misaligned sample workspace -> LBM_E_INVAL", 0, 0);
    check(lbm_set_solids(ctx, 1, smp_d, NULL, NULL, NULL, mws, 16) == LBM_E_NOMEM, "too small sample workspace -> LBM_E_NOMEM", 0, 0);
    lbm_params bad = p;
    bad.nx = 0;
    size_t b2 = 0;
    check(lbm_workspace_size(&bad, &b2) == LBM_E_INVAL, "nx = 0 -> LBM_E_INVAL", 0, 0);

    lbm_destroy(ctx);
    HIP_OK(hipFree(mws));
    HIP_OK(hipFree(smp_d));
    HIP_OK(hipFree(rho_d));
    HIP_OK(hipFree(u_d));
    HIP_OK(hipFree(ws));
    HIP_OK(hipStreamDestroy(st));
    free(rho);
    free(u);
    printf("c-abi: %s\n", failures ? "FAILED" : "all checks hold");
    return failures ? 1 : 0;
}
