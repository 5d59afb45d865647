/*
 * Oracle for whole-body MPPI: a plain, slow FP64 CPU implementation of what the
 * GPU hot path computes.  TEST INFRASTRUCTURE ONLY: it is used by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark, never by the product
 * library, and it shares no code with it.
 *
 * Method: MPPI (paper Sec. II-B, Eqs. 1-2, Algorithm 1) over cubic-spline knots
 * (Sec. III-B) with whole-body floating-base dynamics and penalty contact in place
 * of the MuJoCo simulator (Sec. III-A).
 *
 * State layout (robot, 37 doubles):
 *   [p_w(3), quat wxyz(4), q_joint(12), v_w(3), omega_body(3), qd_joint(12)]
 * joints ordered FL, FR, RL, RR x (abduction, flexion, knee).
 * Scene 3 (free box) appends [p(3), quat wxyz(4), v_w(3), omega_body(3)] -> 50.
 */
#ifndef MPPI_ORACLE_H
#define MPPI_ORACLE_H
#include <stdint.h>

#define ORC_NB 13
#define ORC_NQ 19
#define ORC_NV 18
#define ORC_NX 37
#define ORC_NX_BOX 50

enum { ORC_SCENE_FLAT = 0, ORC_SCENE_HEIGHTFIELD = 1, ORC_SCENE_STATIC_BOX = 2, ORC_SCENE_FREE_BOX = 3 };

typedef struct orc_model {
    double trunk_size[3];
    double trunk_mass;
    double hip_x, hip_y;
    double thigh_len, thigh_mass;
    double calf_len, calf_mass;
    double foot_r;
    double gravity;
    double k, c, mu, vs;          /* contact stiffness, damping, friction, slip velocity */
    int32_t scene;
    int32_t hf_nx, hf_ny, pad0;
    double hf_cell, hf_x0, hf_y0;
    const double *hf;             /* heights, hf[iy*nx + ix] */
    double sbox_center[3], sbox_half[3];   /* static (climb) box, axis aligned */
    double box_half[3], box_mass;          /* free box */
} orc_model;

typedef struct orc_params {
    int32_t K, H, nk;
    int32_t basis;                /* knot interpolation: 0 cubic (not-a-knot), 1 linear, 2 zeroth order, 3 direct */
    double dt, sigma, lambda, kp, kd;
    double w_h, h_ref, w_o, w_v, v_ref, w_tau, w_reach, w_box;
    double goal[2];
    uint64_t seed;
    uint32_t instance, pad1;
} orc_params;

int  orc_nx(const orc_model *m);

/* Counter-based generator (Salmon et al., SC'11) and the Gaussian map. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_sample_eps(const orc_params *p, uint32_t step, double *eps /* K x 12nk */);
void orc_philox_raw(const orc_params *p, uint32_t step, uint32_t *raw /* K x 4*ceil(D/4) */);

/* Spline (Sec. III-B): basis H x nk, shift nk x nk. */
void orc_spline_basis(int nk, int H, double dt, double *B);
void orc_spline_eval(int nk, double T, const double *knots, double t, double *out);
void orc_shift_matrix(int nk, int H, double dt, double *S);
/* The same for a chosen interpolation of the knots (Sec. III-B names the alternatives):
   basis 0 the cubic spline above, 1 straight lines between neighbouring knots, 2 the
   value of the knot at the start of each knot interval held until the next knot, 3
   direct: nk = H values, one per control step (the basis is the identity and the shift
   advances by one step). */
void orc_interp_eval(int basis, int nk, double T, const double *knots, double t, double *out);
void orc_basis_matrix(int basis, int nk, int H, double dt, double *B);
void orc_shift_matrix_b(int basis, int nk, int H, double dt, double *S);

/* Rigid-body terms (no contact). */
void orc_fk(const orc_model *m, const double *q, double *R /*13x9*/, double *pos /*13x3*/, double *com /*13x3*/);
void orc_foot_positions(const orc_model *m, const double *q, double *feet /*4x3*/);
void orc_mass_matrix(const orc_model *m, const double *q, double *M /*18x18*/);
void orc_bias(const orc_model *m, const double *q, const double *v, double *b /*18*/);
double orc_kinetic_energy(const orc_model *m, const double *q, const double *v);
double orc_kinetic_energy_fd(const orc_model *m, const double *q, const double *v, double eps);
double orc_potential_energy(const orc_model *m, const double *q);
void orc_momentum(const orc_model *m, const double *q, const double *v, double *P /*3*/, double *Lo /*3*/);
void orc_retract(const double *q, const double *v, double t, double *qo);
void orc_accel(const orc_model *m, const double *q, const double *v, const double *tau_gen /*18*/, double *vdot);
void orc_rk4(const orc_model *m, double *q, double *v, const double *tau_gen, double dt, int nsteps, int spring,
             const double *kp_target, double kp);

/* One discrete step (linearly implicit velocity update, semi-implicit positions). */
int  orc_step(const orc_model *m, const double *x, const double *u, double kp, double kd, double dt,
              double *xo, double *tau_out);
int  orc_step_system(const orc_model *m, const double *x, const double *u, double kp, double kd, double dt,
                     double *A_out, double *rhs_out);
/* the free box's 6x6 system of the same step, A_b dv_b = rhs_b (scene 3), for diagnostics */
int  orc_step_system_box(const orc_model *m, const double *x, const double *u, double kp, double kd, double dt,
                         double *A_out /*36*/, double *rhs_out /*6*/);
void orc_contact_total(const orc_model *m, const double *x, double *F_robot /*3*/, double *F_box /*3*/, int *n_active);
/* contact geometry and law, exported for their pins (quat is the box orientation, w x y z):
   terrain below a sphere (r > 0) or point (r = 0); sphere against an oriented box (normal
   from the box toward the sphere); point strictly inside an oriented box (shallowest face);
   the penalty law's force and 3x3 damping.  Each returns 1 when in contact. */
int  orc_terrain(const orc_model *m, const double *c, double r, double *delta, double *n);
int  orc_sphere_box(const double *c, double r, const double *p, const double *quat, const double *h, double *delta,
                    double *n);
int  orc_point_box(const double *x, const double *p, const double *quat, const double *h, double *delta, double *n);
int  orc_contact_law(const orc_model *m, double delta, const double *n, const double *vrel, double *F, double *D);

/* Cost, rollout and MPPI (Eqs. 1-2, Algorithm 1). */
double orc_stage_cost(const orc_model *m, const orc_params *p, const double *x, const double *tau);
double orc_rollout(const orc_model *m, const orc_params *p, const double *x0, const double *theta, double *traj);
void orc_rollout_batch(const orc_model *m, const orc_params *p, const double *x0, const double *mu,
                       const double *eps, double *costs, double *traj, int nthreads);
int  orc_weights(int K, double lambda, const double *costs, double *w);
int  orc_update(const orc_params *p, const double *costs, const double *mu, const double *eps,
                double *mu_out, double *w_out);
void orc_shift(const orc_params *p, const double *mu_prime, double *mu_out, double *u0);
int  orc_mppi_step(const orc_model *m, const orc_params *p, uint32_t step, const double *x0, double *mu,
                   double *u0, double *costs, int nthreads);
int  orc_mppi_step_proposal(const orc_model *m, const orc_params *p, uint32_t step, const double *x0, double *mu,
                            const double *center, const double *sd, int Kp, int gate, double *u0, double *costs_p,
                            double *costs, int *accepted, int nthreads);

/* Eq. 3 / Eq. 4 tracking cost with a trotting gait reference (tracking_oracle.c).
   The state error is e = [p - p_ref(t) (3), attitude (3), q - u_ref(t) (12),
   v_w - (v_cmd, 0) (3), omega (3), qd (12)], where p_ref(t) = p_ref0 + (v_cmd t, 0) and the
   attitude error is 2 sgn(qw) (qx, qy, qz) against upright with zero yaw. */
typedef struct orc_tracking {
    double Q[36];                 /* diagonal state weights on e */
    double R[12];                 /* diagonal weights on u - u_ref(t) */
    double p_ref0[3];
    double v_cmd[2];              /* commanded world xy velocity */
    double period, duty;          /* gait period (s) and stance fraction */
    double swing_height;          /* foot lift at mid-swing (m) */
    double stand_height;          /* hip-to-foot-centre height of the reference (m) */
    double raibert_k;             /* gain on (v - v_cmd) in the foothold */
    double box_w;                 /* Q_box of Eq. 4 (free-box scene) */
    double box_goal[2];
    int32_t gait;                 /* 0: standing pose at all times, 1: trot */
    int32_t pad;
} orc_tracking;

/* leg IK: joint angles (abduction, flexion, knee) that put the foot centre at p (3),
   given relative to the hip in the trunk frame; the reach is clamped to the leg's range */
void orc_leg_ik(const orc_model *m, const double *p, double *q);
/* foot target of leg `leg` relative to its hip at gait time t; v_h: the measured base
   velocity in the heading frame (2) */
void orc_gait_foot(const orc_tracking *c, int leg, double t, const double *v_h, const double *cmd_h, double *p);
/* the joint reference u_ref(t) (12), the Raibert feedback taken from the state x0 */
void orc_gait_reference(const orc_model *m, const orc_tracking *c, double t, const double *x0, double *u_ref);
/* one stage term of Eq. 3 (+ Eq. 4): state x at time t_x with joint reference q_ref,
   control u against u_ref */
double orc_tracking_stage(const orc_model *m, const orc_tracking *c, double t_x, const double *x,
                          const double *q_ref, const double *u, const double *u_ref);
/* cost of a rollout trajectory (H+1 states) under controls u (H x 12) at control step
   `step`: sum_k dt [stage(x_{k+1}, u_k)], references at t_k = (step + k) dt */
double orc_tracking_cost(const orc_model *m, const orc_params *p, const orc_tracking *c, uint32_t step,
                         const double *traj, const double *u);
/* rollout of one knot vector with the tracking cost (the dynamics of orc_rollout) */
double orc_rollout_tracking(const orc_model *m, const orc_params *p, const orc_tracking *c, uint32_t step,
                            const double *x0, const double *theta, double *traj);
/* Algorithm 1 with the tracking cost */
int  orc_mppi_step_tracking(const orc_model *m, const orc_params *p, const orc_tracking *c, uint32_t step,
                            const double *x0, double *mu, double *u0, double *costs, int nthreads);

/* Learned proposal network (mlp_oracle.c). */
int  orc_mlp_n_params(void);
void orc_mlp_forward(const double *P, int B, const double *X, double *out, int bf);
void orc_policy_features(const double *x, const double *cmd, const double *origin, const double *in_mean,
                         const double *in_std, double *feat);
void orc_policy_head(const double *out, const double *out_mean, const double *out_std, int nk, double sigma_max,
                     double *center, double *sd);

#endif
