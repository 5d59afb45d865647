/*
 * A closed loop through the C ABI alone: no Python and no PyTorch, device memory from the
 * HIP runtime.  Reads a flat-ground model, controller parameters, an initial state and a
 * nominal plan from a text file (whitespace separated):
 *   16 model values   trunk size (3), trunk mass, hip x, hip y, thigh length and mass,
 *                     calf length and mass, foot radius, gravity, contact k, c, mu, v_slip
 *   16 parameters     K, H, n_knots, dt, sigma, lambda, kp, kd, w_height, h_ref,
 *                     w_upright, w_vel, v_ref, w_torque, seed, instance
 *   steps
 *   37 state values, then 12 * n_knots knots (joint-major)
 * runs `steps` control steps (mppi_step, Algorithm 1) each followed by one plant step
 * (mppi_sim_step), and prints the final state and the last first control, one value per
 * line.  Exit status 77 when no GPU is visible, 1 on an error, 0 otherwise.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "mppi.h"

#define NX 37

static int fail(const char *what, mppi_status s)
{
    fprintf(stderr, "%s: %s (%s)\n", what, mppi_status_str(s), mppi_last_error(NULL));
    return 1;
}

static int hip_fail(const char *what, hipError_t e)
{
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 1;
}

#define MPPI(call)                                   \
    do {                                             \
        mppi_status s_ = (call);                     \
        if (s_ < 0) return fail(#call, s_);          \
    } while (0)
#define HIP(call)                                    \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) return hip_fail(#call, e_); \
    } while (0)

static int read_values(FILE *f, double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (fscanf(f, "%lf", &v[i]) != 1) return 0;
    return 1;
}

int main(int argc, char **argv)
{
    if (argc != 2) {
        fprintf(stderr, "usage: %s input.txt\n", argv[0]);
        return 1;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        fprintf(stderr, "no GPU visible\n");
        return 77;
    }
    FILE *f = fopen(argv[1], "r");
    if (!f) {
        perror(argv[1]);
        return 1;
    }
    double mv[16], pv[16], sv[1], x0[NX], knots[96];
    if (!read_values(f, mv, 16) || !read_values(f, pv, 16) || !read_values(f, sv, 1) || !read_values(f, x0, NX)) {
        fprintf(stderr, "malformed input\n");
        fclose(f);
        return 1;
    }
    const int nk = (int)pv[2], steps = (int)sv[0], D = 12 * nk;
    if (nk < 2 || nk > 8 || steps < 1 || !read_values(f, knots, D)) {
        fprintf(stderr, "malformed input\n");
        fclose(f);
        return 1;
    }
    fclose(f);

    mppi_model_desc d = {0};
    for (int i = 0; i < 3; ++i) d.trunk_size[i] = (float)mv[i];
    d.trunk_mass = (float)mv[3];
    d.hip_x = (float)mv[4];
    d.hip_y = (float)mv[5];
    d.thigh_len = (float)mv[6];
    d.thigh_mass = (float)mv[7];
    d.calf_len = (float)mv[8];
    d.calf_mass = (float)mv[9];
    d.foot_r = (float)mv[10];
    d.gravity = (float)mv[11];
    d.contact_k = (float)mv[12];
    d.contact_c = (float)mv[13];
    d.friction_mu = (float)mv[14];
    d.slip_velocity = (float)mv[15];
    d.scene = MPPI_SCENE_FLAT;

    mppi_params p = {0};
    p.K = (int32_t)pv[0];
    p.H = (int32_t)pv[1];
    p.n_knots = nk;
    p.dt = (float)pv[3];
    p.sigma = (float)pv[4];
    p.lambda = (float)pv[5];
    p.kp = (float)pv[6];
    p.kd = (float)pv[7];
    p.w_height = (float)pv[8];
    p.h_ref = (float)pv[9];
    p.w_upright = (float)pv[10];
    p.w_vel = (float)pv[11];
    p.v_ref = (float)pv[12];
    p.w_torque = (float)pv[13];
    p.seed = (uint64_t)pv[14];
    p.instance = (uint32_t)pv[15];
    p.arith = MPPI_ARITH_FP64;
    p.basis = MPPI_BASIS_CUBIC;

    mppi_model *model = NULL;
    mppi_ctx *ctx = NULL;
    MPPI(mppi_model_create(&d, &model));
    MPPI(mppi_create(model, &p, &ctx));

    hipStream_t stream;
    void *ws;
    float *dx[2], *du, *dk;
    const size_t ws_bytes = mppi_workspace_bytes(ctx);
    HIP(hipStreamCreate(&stream));
    HIP(hipMalloc(&ws, ws_bytes));  /* the runtime aligns allocations to at least 256 bytes */
    HIP(hipMalloc((void **)&dx[0], sizeof(float) * NX));
    HIP(hipMalloc((void **)&dx[1], sizeof(float) * NX));
    HIP(hipMalloc((void **)&du, sizeof(float) * 12));
    HIP(hipMalloc((void **)&dk, sizeof(float) * D));
    MPPI(mppi_bind(ctx, ws, ws_bytes, stream));

    float hx[NX], hu[12], hk[96];
    for (int i = 0; i < NX; ++i) hx[i] = (float)x0[i];
    for (int i = 0; i < D; ++i) hk[i] = (float)knots[i];
    HIP(hipMemcpy(dx[0], hx, sizeof(hx), hipMemcpyHostToDevice));
    HIP(hipMemcpy(dk, hk, sizeof(float) * D, hipMemcpyHostToDevice));
    MPPI(mppi_set_nominal(ctx, dk));

    int cur = 0;
    for (int s = 0; s < steps; ++s) {
        MPPI(mppi_step(ctx, dx[cur], du));
        MPPI(mppi_sim_step(model, MPPI_ARITH_FP64, 1, dx[cur], du, p.kp, p.kd, p.dt, dx[1 - cur], NULL, NULL,
                           stream));
        cur = 1 - cur;
    }
    const mppi_status st = mppi_sync_status(ctx);
    if (st < 0) return fail("mppi_sync_status", st);
    HIP(hipMemcpy(hx, dx[cur], sizeof(hx), hipMemcpyDeviceToHost));
    HIP(hipMemcpy(hu, du, sizeof(hu), hipMemcpyDeviceToHost));
    for (int i = 0; i < NX; ++i) printf("%.9g\n", hx[i]);
    for (int i = 0; i < 12; ++i) printf("%.9g\n", hu[i]);

    mppi_destroy(ctx);
    mppi_model_destroy(model);
    (void)hipFree(dk);
    (void)hipFree(du);
    (void)hipFree(dx[1]);
    (void)hipFree(dx[0]);
    (void)hipFree(ws);
    (void)hipStreamDestroy(stream);
    return 0;
}
