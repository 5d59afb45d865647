/*
 * Oracle of the tracking cost -- plain FP64 C.  TEST INFRASTRUCTURE ONLY (tests,
 * smoke check, CPU baseline); the product library never links or calls it.
 *
 * What it follows:
 *   - Eq. 3 (Sec. IV-B): a quadratic penalty on the deviation of the state from a
 *     reference (desired base position and attitude) plus a quadratic penalty on the
 *     deviation of the controls from a time-varying joint reference u_ref(t), both with
 *     diagonal weights.
 *   - u_ref(t) is a trotting gait whose footholds follow the Raibert heuristic (the
 *     paper names the heuristic and the gait, not the formulas): diagonal leg pairs
 *     alternate between stance and swing; a foot lands half a stance-length ahead of the
 *     hip along the commanded velocity, corrected by a gain times the velocity error; in
 *     stance it sweeps back at the commanded speed; in swing it returns along a raised
 *     arc.  Foot targets become joint targets by closed-form leg inverse kinematics.
 *   - Eq. 4 (Sec. IV-D): the box-push cost adds a weighted l1 distance of the box
 *     position from its target.
 * Readings where the paper is silent (the form of the attitude error, the time pairing
 * of states and controls, the gait constants) are stated next to the code.
 */
#include "mppi_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* diagonal legs move together: FL with RR, FR with RL */
static const double kPhaseOffset[4] = {0.0, 0.5, 0.5, 0.0};

void orc_leg_ik(const orc_model *m, const double *p, double *q)
{
    double l1 = m->thigh_len, l2 = m->calf_len;
    /* abduction about the trunk x axis turns the leg plane; the foot lies at distance r
       below the hip inside that plane */
    double r = sqrt(p[1] * p[1] + p[2] * p[2]);
    double a = atan2(p[1], -p[2]);
    double xs = p[0], zs = -r;
    /* two-link reach, clamped inside the workspace (reading: 5% of the total length from
       the inner limit, 0.1% from full extension) */
    double d = sqrt(xs * xs + zs * zs);
    double dmin = fabs(l1 - l2) + 0.05 * (l1 + l2), dmax = 0.999 * (l1 + l2);
    if (d < dmin) d = dmin;
    if (d > dmax) d = dmax;
    double ck = (d * d - l1 * l1 - l2 * l2) / (2 * l1 * l2);
    if (ck > 1) ck = 1;
    if (ck < -1) ck = -1;
    double k = -acos(ck); /* knee bent backwards, as in the standing pose */
    /* rotation about y by angle h maps the hanging direction (0, 0, -1) to
       (-sin h, 0, -cos h); the foot direction from the hip is at angle atan2(-xs, -zs) */
    double h = atan2(-xs, -zs) - atan2(l2 * sin(k), l1 + l2 * cos(k));
    q[0] = a;
    q[1] = h;
    q[2] = k;
}

void orc_gait_foot(const orc_tracking *c, int leg, double t, const double *v_h, const double *cmd_h, double *p)
{
    if (c->gait == 0) {
        p[0] = 0; p[1] = 0; p[2] = -c->stand_height;
        return;
    }
    double T = c->period, duty = c->duty, Tst = duty * T;
    double ph = t / T + kPhaseOffset[leg];
    ph -= floor(ph);
    double land[2], lift = 0, xy[2];
    for (int i = 0; i < 2; ++i) land[i] = 0.5 * cmd_h[i] * Tst + c->raibert_k * (v_h[i] - cmd_h[i]);
    if (ph < duty) {
        double s = ph / duty; /* stance: the foot moves back under the advancing hip */
        for (int i = 0; i < 2; ++i) xy[i] = land[i] - cmd_h[i] * Tst * s;
    } else {
        double s = (ph - duty) / (1 - duty); /* swing: back to the next foothold on an arc */
        double w = 0.5 * (1 - cos(M_PI * s));
        for (int i = 0; i < 2; ++i) {
            double lo = land[i] - cmd_h[i] * Tst;
            xy[i] = lo + (land[i] - lo) * w;
        }
        lift = c->swing_height * sin(M_PI * s);
    }
    p[0] = xy[0];
    p[1] = xy[1];
    p[2] = -c->stand_height + lift;
}

/* heading (yaw) of the trunk and the rotation of world xy vectors into the heading frame */
static void to_heading(const double *x, const double *vw, double *out)
{
    double qw = x[3], qx = x[4], qy = x[5], qz = x[6];
    double psi = atan2(2 * (qw * qz + qx * qy), 1 - 2 * (qy * qy + qz * qz));
    double c = cos(psi), s = sin(psi);
    out[0] = c * vw[0] + s * vw[1];
    out[1] = -s * vw[0] + c * vw[1];
}

void orc_gait_reference(const orc_model *m, const orc_tracking *c, double t, const double *x0, double *u_ref)
{
    double v_h[2], cmd_h[2], p[3];
    double vw[2] = {x0[ORC_NQ], x0[ORC_NQ + 1]};
    to_heading(x0, vw, v_h);
    to_heading(x0, c->v_cmd, cmd_h);
    for (int leg = 0; leg < 4; ++leg) {
        orc_gait_foot(c, leg, t, v_h, cmd_h, p);
        orc_leg_ik(m, p, u_ref + 3 * leg);
    }
}

/* reading: the state term pairs the post-step state x_{k+1} with the joint reference
   at its own time; the control term pairs u_k with u_ref(t_k) */
static double stage(const orc_model *m, const orc_tracking *c, double t_x, const double *x, const double *q_ref,
                    const double *u, const double *u_ref)
{
    double e[36];
    double pref[3] = {c->p_ref0[0] + c->v_cmd[0] * t_x, c->p_ref0[1] + c->v_cmd[1] * t_x, c->p_ref0[2]};
    for (int i = 0; i < 3; ++i) e[i] = x[i] - pref[i];
    /* attitude against upright with zero yaw: twice the vector part of the unit
       quaternion, sign-fixed so that q and -q give the same error (small-angle rotation
       vector) */
    double sg = x[3] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < 3; ++i) e[3 + i] = 2 * sg * x[4 + i];
    for (int j = 0; j < 12; ++j) e[6 + j] = x[7 + j] - q_ref[j];
    e[18] = x[ORC_NQ] - c->v_cmd[0];
    e[19] = x[ORC_NQ + 1] - c->v_cmd[1];
    e[20] = x[ORC_NQ + 2];
    for (int i = 0; i < 3; ++i) e[21 + i] = x[ORC_NQ + 3 + i];
    for (int j = 0; j < 12; ++j) e[24 + j] = x[ORC_NQ + 6 + j];
    double l = 0;
    for (int i = 0; i < 36; ++i) l += c->Q[i] * e[i] * e[i];
    for (int j = 0; j < 12; ++j) l += c->R[j] * (u[j] - u_ref[j]) * (u[j] - u_ref[j]);
    if (m->scene == ORC_SCENE_FREE_BOX)
        l += c->box_w * (fabs(c->box_goal[0] - x[ORC_NX]) + fabs(c->box_goal[1] - x[ORC_NX + 1]));
    return l;
}

double orc_tracking_stage(const orc_model *m, const orc_tracking *c, double t_x, const double *x,
                          const double *q_ref, const double *u, const double *u_ref)
{
    return stage(m, c, t_x, x, q_ref, u, u_ref);
}

double orc_tracking_cost(const orc_model *m, const orc_params *p, const orc_tracking *c, uint32_t step,
                         const double *traj, const double *u)
{
    int H = p->H, nx = orc_nx(m);
    double *ref = malloc(sizeof(double) * 12 * (H + 1));
    for (int k = 0; k <= H; ++k) orc_gait_reference(m, c, ((double)step + k) * p->dt, traj, ref + 12 * k);
    double L = 0;
    for (int k = 0; k < H; ++k) {
        double t_x = ((double)step + k + 1) * p->dt;
        L += p->dt * stage(m, c, t_x, traj + (size_t)(k + 1) * nx, ref + 12 * (k + 1), u + 12 * k, ref + 12 * k);
    }
    free(ref);
    return isfinite(L) ? L : INFINITY;
}

double orc_rollout_tracking(const orc_model *m, const orc_params *p, const orc_tracking *c, uint32_t step,
                            const double *x0, const double *theta, double *traj)
{
    int H = p->H, nk = p->nk, nx = orc_nx(m);
    double *tr = traj ? traj : malloc(sizeof(double) * (size_t)(H + 1) * nx);
    double *B = malloc(sizeof(double) * H * nk), *u = malloc(sizeof(double) * 12 * H);
    double L = orc_rollout(m, p, x0, theta, tr);
    if (isfinite(L)) {
        orc_basis_matrix(p->basis, nk, H, p->dt, B);
        for (int k = 0; k < H; ++k)
            for (int j = 0; j < 12; ++j) {
                double s = 0;
                for (int i = 0; i < nk; ++i) s += B[k * nk + i] * theta[j * nk + i];
                u[12 * k + j] = s;
            }
        L = orc_tracking_cost(m, p, c, step, tr, u);
    }
    free(B);
    free(u);
    if (!traj) free(tr);
    return L;
}

int orc_mppi_step_tracking(const orc_model *m, const orc_params *p, const orc_tracking *c, uint32_t step,
                           const double *x0, double *mu, double *u0, double *costs, int nthreads)
{
    int K = p->K, D = 12 * p->nk;
    double *eps = malloc(sizeof(double) * (size_t)K * D);
    double *L = costs ? costs : malloc(sizeof(double) * K);
    double mup[96];
    orc_sample_eps(p, step, eps);
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int n = 0; n < K; ++n) {
        double theta[96];
        for (int d = 0; d < D; ++d) theta[d] = mu[d] + (n ? p->sigma * eps[(size_t)n * D + d] : 0.0);
        L[n] = orc_rollout_tracking(m, p, c, step, x0, theta, NULL);
    }
    (void)nthreads;
    int rc = orc_update(p, L, mu, eps, mup, NULL);
    orc_shift(p, mup, mu, u0);
    free(eps);
    if (!costs) free(L);
    return rc;
}
