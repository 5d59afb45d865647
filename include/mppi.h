/*
 * mppi.h -- C ABI of the MI355X (gfx950) whole-body MPPI library.
 *
 * The library implements the sampling, rollout and update of model-predictive path
 * integral control (Sec. II-B of the paper: Eq. 1 weights, Eq. 2 mean update,
 * Algorithm 1 loop) over cubic-spline knots tracked by joint PD controllers
 * (Sec. III-B), with a floating-base quadruped simulated by the library's own rigid-body
 * dynamics and penalty contact in place of the MuJoCo simulator (Sec. III-A).
 *
 * Conventions for every call:
 *  - Pointers named d_* are DEVICE pointers owned by the caller; host pointers are named
 *    without the prefix.  The library keeps no caller pointer after a call returns,
 *    except the workspace and stream given to mppi_bind.
 *  - Calls that launch work are asynchronous on the bound HIP stream (passed as void*).
 *    Nothing is returned through host memory except the status code.
 *  - A negative status means nothing was launched; mppi_last_error() describes why.
 *  - All floating-point data is FP32.
 *  - The library never allocates device memory: the caller allocates a workspace of
 *    mppi_workspace_bytes() bytes (256-byte aligned) and binds it.
 *
 * State layout (robot, 37 floats):
 *   [p_world(3), quat wxyz(4), q_joint(12), v_world(3), omega_body(3), qd_joint(12)]
 * joints ordered front-left, front-right, rear-left, rear-right x (abduction, hip
 * flexion, knee).  Scene MPPI_SCENE_FREE_BOX appends the box
 *   [p_world(3), quat wxyz(4), v_world(3), omega_body(3)]  -> 50 floats.
 * Knot layout: joint-major, knots[j * n_knots + i], i-th knot of joint j at time
 *   t_i = i * H * dt / (n_knots - 1).
 */
#ifndef MPPI_H
#define MPPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mppi_status {
    MPPI_OK = 0,
    MPPI_WARN_ALL_NONFINITE = 1,   /* every sample diverged: the nominal was kept (shifted) */
    MPPI_WARN_FALLBACK = 2,        /* the last (gated) proposal step fell back to plain MPPI */
    MPPI_WARN_NONFINITE_INPUT = 3, /* the last step's device start state was not finite: no sample was
                                      rolled out, every cost is +inf and the nominal was kept (shifted) */
    MPPI_EINVAL = -1,              /* bad argument; see mppi_last_error */
    MPPI_ENOMEM = -2,              /* workspace too small */
    MPPI_EHIP = -3,                /* a HIP runtime call failed */
    MPPI_ENONFINITE_INPUT = -4,    /* a host-visible start state is not finite: nothing was launched */
    MPPI_EBUDGET = -5,             /* batched serving: the instance does not fit in the HBM budget */
    MPPI_ESTATE = -6               /* call out of order (e.g. no workspace bound) */
} mppi_status;

enum {
    MPPI_SCENE_FLAT = 0,        /* ground plane z = 0 */
    MPPI_SCENE_HEIGHTFIELD = 1, /* bilinear heightfield */
    MPPI_SCENE_STATIC_BOX = 2,  /* ground plane plus a fixed axis-aligned box (climbing) */
    MPPI_SCENE_FREE_BOX = 3     /* ground plane plus a free box (pushing) */
};

/* Arithmetic of one dynamics step.  The state is FP32 between steps in both modes. */
enum {
    MPPI_ARITH_FP64 = 0,  /* default: step computed in FP64 (FP32-state-limited accuracy) */
    MPPI_ARITH_FP32 = 1,  /* step computed in FP32: faster, per-step error set by the contact conditioning */
    MPPI_ARITH_MIXED = 2  /* kinematics, contact detection and law in FP32; the implicit system (mass matrix,
                             bias, contact damping and forces, leg elimination, 6x6 solves) in FP64.  Lane-split
                             rollout only (MPPI_LANES_SPLIT or DEFAULT); other kernels of the controller (the
                             tracking cost) run in FP32 */
};

#define MPPI_MAX_KNOTS 8
#define MPPI_MAX_HORIZON 256
#define MPPI_MAX_HEIGHTFIELD 14336 /* cells: the grid is staged in LDS with the spline basis */

/* Robot and scene.  The robot is a trunk box with four legs; each leg has abduction
 * (x), hip flexion (y) and knee (y) joints at the hip point (+-hip_x, +-hip_y, 0), a
 * thigh and a calf modelled as uniform rods along -z of their frames, and a massless
 * foot sphere at the calf end.  Contact: normal k*depth - c*v_n while overlapping,
 * friction mu*Fn*tanh(|v_t|/slip_velocity). */
typedef struct mppi_model_desc {
    float trunk_size[3];
    float trunk_mass;
    float hip_x, hip_y;
    float thigh_len, thigh_mass;
    float calf_len, calf_mass;
    float foot_r;
    float gravity;
    float contact_k, contact_c, friction_mu, slip_velocity;
    int32_t scene;
    int32_t hf_nx, hf_ny;       /* heightfield grid (scene 1) */
    float hf_cell, hf_x0, hf_y0;
    const float *heightfield;   /* HOST pointer, hf_ny * hf_nx heights, row = y; copied */
    float sbox_center[3], sbox_half[3]; /* static box (scene 2) */
    float box_half[3], box_mass;        /* free box (scene 3) */
} mppi_model_desc;

/* Controller.  Sample 0 is the noise-free nominal; samples n >= 1 use
 * theta_n = mu + sigma * eps_n.  Running cost per step (dt times)
 *   w_height (z - h_ref)^2 + w_upright (1 - R_zz^2) + w_vel (v_x - v_ref)^2 + w_torque |tau|^2
 * and in scene 3 the velocity term is replaced by
 *   w_reach |p_xy - box_xy|^2 + w_box |box_xy - goal|^2. */
typedef struct mppi_params {
    int32_t K, H, n_knots;
    float dt, sigma, lambda, kp, kd;
    float w_height, h_ref, w_upright, w_vel, v_ref, w_torque, w_reach, w_box;
    float goal[2];
    uint64_t seed;
    uint32_t instance;
    int32_t arith;              /* MPPI_ARITH_FP64 (0, default), MPPI_ARITH_FP32 or MPPI_ARITH_MIXED */
    int32_t basis;              /* knot interpolation, MPPI_BASIS_* (0: cubic, the default) */
    int32_t cost;               /* MPPI_COST_RUNNING (0, default) or MPPI_COST_TRACKING */
    int32_t lanes;              /* lanes per sample of the rollout kernel, MPPI_LANES_* (0: default) */
} mppi_params;

/* Rollout decomposition.  QUAD: one lane per leg, 16 samples per wave.  SPLIT: 16 lanes
 * per sample (four per leg: knot interpolation, trigonometry and the trunk and box
 * corner contacts spread over them), 4 samples per wave, so K = 4096 fills every SIMD of
 * the chip.  Both compute the same step; only summation orders differ.  DEFAULT picks
 * SPLIT when its LDS rows fit (a heightfield above about 11,000 cells in FP64 does not)
 * and QUAD otherwise.  The plant step (mppi_sim_step) and batched serving use QUAD. */
enum { MPPI_LANES_DEFAULT = 0, MPPI_LANES_QUAD = 4, MPPI_LANES_SPLIT = 16 };

/* Interpolation of the knots into per-step joint targets (Sec. III-B uses the cubic
 * spline and names zeroth-order and linear interpolation as the alternatives):
 *   CUBIC  not-a-knot cubic spline through the knots;
 *   LINEAR straight lines between neighbouring knots;
 *   ZERO   each knot's value held from its time until the next knot's.
 * All pass through the knots, so u0 is the first knot; the warm-start shift evaluates
 * the same interpolant one step later. */
enum { MPPI_BASIS_CUBIC = 0, MPPI_BASIS_LINEAR = 1, MPPI_BASIS_ZERO = 2, MPPI_BASIS_DIRECT = 3 };
/* DIRECT samples every control step's targets (the per-timestep representation Sec. III-B
 * compares the spline with): n_knots must equal H (at most MPPI_MAX_HORIZON), knot i is the
 * target of step i, the shift moves every value one step earlier and holds the last.  The
 * noise is drawn inside the rollout's step loop.  Lane-split rollout and running cost only. */

/* The sample cost.  RUNNING: the weights in mppi_params above, summed inside the rollout.
 * TRACKING: Eq. 3 (Sec. IV-B) with the gait reference below, plus Eq. 4's l1 box term
 * (Sec. IV-D) in the free-box scene, evaluated on the rollout trajectories; set its
 * parameters with mppi_set_tracking_cost before the first rollout.  The workspace then
 * holds the K x (H+1) x nx trajectories as well. */
enum { MPPI_COST_RUNNING = 0, MPPI_COST_TRACKING = 1 };

/* Eq. 3 / Eq. 4 cost.  For control step s, rollout step k applies u_k at gait time
 * t_k = (s + k) dt and reaches x_{k+1} at t_{k+1}; the sample cost is
 *   L = sum_{k=0}^{H-1} dt [ e(x_{k+1})^T diag(Q) e(x_{k+1})
 *                            + (u_k - u_ref(t_k))^T diag(R) (u_k - u_ref(t_k))
 *                            + box_weight |box_goal - box_xy(x_{k+1})|_1 ]   (box: free-box scene)
 * with the state error e = [p - p_ref(t) (3), 2 sgn(qw) (qx, qy, qz) (3), q - u_ref(t) (12),
 * v_world - (v_cmd, 0) (3), omega_body (3), qd (12)] and p_ref(t) = p_ref0 + (v_cmd t, 0).
 * u_ref(t): joint targets of a gait.  gait 0 holds every foot stand_height below its hip.
 * gait 1 trots: diagonal leg pairs (front-left with rear-right) half a period apart,
 * stance for the first `duty` of each period.  In the heading frame of the rollout's start
 * state, a foot lands at cmd T_st / 2 + raibert_gain (v - cmd) from its hip (T_st = duty
 * period, v the start state's base velocity), sweeps back by cmd T_st during stance, and
 * returns to the next foothold in swing along (1 - cos(pi s)) / 2 while lifted by
 * swing_height sin(pi s).  Foot targets become joint targets by closed-form leg inverse
 * kinematics (reach clamped to [0.05 (l1 + l2) + |l1 - l2|, 0.999 (l1 + l2)]). */
typedef struct mppi_tracking_cost {
    float Q[36];                 /* diagonal state weights, >= 0 */
    float R[12];                 /* diagonal control weights, >= 0 */
    float p_ref0[3];             /* base position reference at gait time 0 */
    float v_cmd[2];              /* commanded world xy velocity */
    float period, duty;          /* gait period (s, > 0) and stance fraction (0 < duty < 1) */
    float swing_height;          /* foot lift at mid-swing (m, >= 0) */
    float stand_height;          /* hip-to-foot-centre height of the reference (m, > 0) */
    float raibert_gain;          /* foothold gain on the velocity error (s) */
    float box_weight;            /* Q_box of Eq. 4 (free-box scene), >= 0 */
    float box_goal[2];
    int32_t gait;                /* 0: stand, 1: trot */
    int32_t reserved;            /* must be 0 */
} mppi_tracking_cost;

typedef struct mppi_model mppi_model;
typedef struct mppi_ctx mppi_ctx;

/* Copies the description (and the heightfield) into a host-side model.
 * EINVAL on non-positive sizes or masses, an unknown scene, or a heightfield larger
 * than MPPI_MAX_HEIGHTFIELD cells. */
mppi_status mppi_model_create(const mppi_model_desc *desc, mppi_model **out);
void mppi_model_destroy(mppi_model *model);
/* number of floats in a state for this model (37, or 50 with a free box) */
int mppi_model_nx(const mppi_model *model);

/* Creates a controller (Algorithm 1 "Require": samples K, horizon H, temperature
 * lambda, sampling scale sigma).  Builds the spline basis and shift matrix on the host.
 * EINVAL unless 1 <= K, 1 <= H <= MPPI_MAX_HORIZON, 2 <= n_knots <= MPPI_MAX_KNOTS,
 * dt > 0, lambda > 0, sigma >= 0, arith one of MPPI_ARITH_*. */
mppi_status mppi_create(const mppi_model *model, const mppi_params *params, mppi_ctx **out);
void mppi_destroy(mppi_ctx *ctx);
size_t mppi_workspace_bytes(const mppi_ctx *ctx);
/* Host copies of the matrices built at creation (Sec. III-B interpolation, Algorithm 1
 * shift): B_out (HOST, H x n_knots, row k = weights of the knots in step k's joint
 * targets) and S_out (HOST, n_knots x n_knots, the warm-start shift); either may be NULL.
 * Launches nothing; needs no workspace. */
mppi_status mppi_get_basis(const mppi_ctx *ctx, double *B_out, float *S_out);
/* Binds a caller-owned device workspace and stream; uploads model data, spline basis and
 * shift matrix, and sets the nominal to zero.  The step counter is reset to 0.  Also
 * creates the internal stream and two events of the gated proposal step (default
 * priority), released by the next bind or mppi_destroy. */
mppi_status mppi_bind(mppi_ctx *ctx, void *d_workspace, size_t bytes, void *hip_stream);
/* nominal knots mu (12 * n_knots floats, device) in/out */
mppi_status mppi_set_nominal(mppi_ctx *ctx, const float *d_knots);
mppi_status mppi_get_nominal(mppi_ctx *ctx, float *d_knots);
/* control-step counter used as the third Philox counter word (noise of step s) */
mppi_status mppi_set_step(mppi_ctx *ctx, uint32_t step);
uint32_t mppi_get_step(const mppi_ctx *ctx);

/* Gaussian knot noise (Sec. II-B sampling), eps[n * D + d], D = 12 * n_knots:
 * Philox4x32-10 with key (seed_lo, seed_hi) and counter (d / 4, n, step, instance);
 * 24-bit uniforms ((x >> 8) + 1/2) / 2^24 mapped by Box-Muller on word pairs (0,1), (2,3).
 * d_raw (optional) receives the raw words, K x 4*ceil(D/4). */
mppi_status mppi_sample(mppi_ctx *ctx, float *d_eps, uint32_t *d_raw);

/* Rolls out all K samples from d_x0 (Algorithm 1 inner loops): spline targets, PD
 * torques, dynamics step, running cost.  d_eps: K x D noise, or NULL to draw it with
 * Philox for the current step (kept in the workspace for mppi_update).  d_costs: K
 * floats (+inf for a diverged sample).  d_traj: optional K x (H+1) x nx states.  With
 * MPPI_COST_TRACKING the costs are the Eq. 3 / Eq. 4 costs of the trajectories at the
 * current step counter (ESTATE before mppi_set_tracking_cost). */
mppi_status mppi_rollout_batch(mppi_ctx *ctx, const float *d_x0, const float *d_eps, float *d_costs,
                               float *d_traj);

/* Eq. 1 weights from d_costs and Eq. 2 mean update of the knots, using d_eps (or, if
 * NULL, the noise the last Philox rollout kept).  Writes the updated (unshifted) knots
 * to d_knots_out and optionally the weights (K floats).  Does not change the nominal. */
mppi_status mppi_update(mppi_ctx *ctx, const float *d_costs, const float *d_eps, float *d_knots_out,
                        float *d_weights_out);

/* One full control step (Algorithm 1): sample, roll out, weight, update, take the first
 * control u = spline(mu', 0) into d_u0_out (12 floats), shift the nominal by dt, and
 * advance the step counter.  If every sample diverged the shifted old nominal is kept
 * and mppi_sync_status reports MPPI_WARN_ALL_NONFINITE.  The start state is checked for
 * finiteness: when d_x0 is host-visible (managed or mapped host memory) on the host, and
 * the call returns MPPI_ENONFINITE_INPUT without launching; otherwise on the device by
 * the lane-split rollout, which then rolls out nothing and leaves
 * MPPI_WARN_NONFINITE_INPUT for mppi_sync_status. */
mppi_status mppi_step(mppi_ctx *ctx, const float *d_x0, float *d_u0_out);

/* The second half of mppi_step, for callers that time or overlap the two kernels:
 * after mppi_rollout_batch(ctx, d_x0, NULL, d_costs, ...) of the current step, computes
 * the Eq. 1 weights (optionally written to d_weights_out, K floats), the Eq. 2 update,
 * the first control into d_u0_out, shifts the nominal and advances the step counter.
 * mppi_step(ctx, x, u) is exactly rollout_batch(x, NULL, costs) + update_shift(costs, u). */
mppi_status mppi_update_shift(mppi_ctx *ctx, const float *d_costs, float *d_u0_out, float *d_weights_out);

/* Copies the Eq. 3 / Eq. 4 parameters into the controller (host pointer; nothing is
 * launched).  EINVAL on a controller created with cost MPPI_COST_RUNNING, non-finite or
 * negative weights, period <= 0, duty outside (0, 1), stand_height <= 0, an unknown gait
 * or a non-zero reserved field. */
mppi_status mppi_set_tracking_cost(mppi_ctx *ctx, const mppi_tracking_cost *cost);

/* Synchronises the bound stream and returns the status of the last step: MPPI_OK,
 * MPPI_WARN_NONFINITE_INPUT, MPPI_WARN_ALL_NONFINITE or MPPI_WARN_FALLBACK (in that order
 * of precedence). */
mppi_status mppi_sync_status(mppi_ctx *ctx);

/* One dynamics step for n independent states (the plant of a closed loop):
 * x_out = step(x, u) with joint targets d_u (n x 12), PD gains kp, kd, time step dt.
 * d_tau_out (optional) receives the PD torques (n x 12).  d_hf: device heightfield for
 * scene 1 (may be NULL otherwise).  arith: MPPI_ARITH_*; MPPI_ARITH_MIXED steps in FP64. */
mppi_status mppi_sim_step(const mppi_model *model, int arith, int n, const float *d_x, const float *d_u, float kp,
                          float kd, float dt, float *d_x_out, float *d_tau_out, const float *d_hf, void *hip_stream);

/* For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): one plain control step, as mppi_step,
 * of a controller created with mppi_create and NOT bound, with its whole workspace in a
 * static device array of MPPI_STATIC_SCRATCH_BYTES that the library holds per GPU until
 * the process ends.  d_nominal (12 * n_knots floats, device) holds the nominal plan on
 * entry and the shifted plan on return (the scratch keeps nothing the caller needs);
 * d_u0_out receives the first control; the controller's step counter advances.  The
 * spline matrices and heightfield are uploaded from host memory on every call.  Calls on
 * one GPU share its array: calls that overlap in time on one GPU race (serialise them,
 * e.g. on one stream).  Errors: EINVAL when the controller's workspace
 * (mppi_workspace_bytes) exceeds the array, it uses the learned proposal or the tracking
 * cost, or a pointer is null; ESTATE when it is bound; EHIP when the array's address
 * cannot be looked up.  No device memory is allocated or freed. */
#define MPPI_STATIC_SCRATCH_BYTES (16u << 20)
mppi_status mppi_step_static(mppi_ctx *ctx, const float *d_x0, float *d_nominal, float *d_u0_out, void *hip_stream);

const char *mppi_status_str(mppi_status s);
const char *mppi_last_error(const mppi_ctx *ctx);

/* ---------------------------------------------------------------------------------
 * Batched serving: many independent MPPI instances (own model, K, H, knots, state)
 * advanced together, one graph launch per control step.  Each step every live
 * instance samples, rolls out, updates and shifts its nominal exactly as mppi_step
 * does (same Philox counters: step counter per instance, instance id from its params),
 * then advances its own state by one plant step with the new first control and adds
 * dt * running cost to its accumulated cost (closed loop on the GPU).
 *
 * Work is split into tiles of 16 samples popped from a device queue by a persistent
 * kernel; the workgroup finishing an instance's last tile runs its update.  The
 * caller's workspace is the HBM budget: a control region (mppi_batch_control_bytes)
 * followed by a pool from which instances are allocated first-fit.
 * --------------------------------------------------------------------------------- */
#define MPPI_BATCH_MAX_MODELS 8
typedef struct mppi_batch mppi_batch;

/* max_horizon and max_hf_cells size the LDS stage (8 B x max_horizon x 8 knots + 4 B x
 * max_hf_cells <= 64 KiB in FP64 arithmetic).  EINVAL on out-of-range limits. */
mppi_status mppi_batch_create(int max_instances, int max_horizon, int max_hf_cells, int arith, mppi_batch **out);
void mppi_batch_destroy(mppi_batch *b);
size_t mppi_batch_control_bytes(int max_instances, int arith);
/* binds the workspace (256-byte aligned) and stream; forgets all models and instances */
mppi_status mppi_batch_bind(mppi_batch *b, void *d_workspace, size_t bytes, void *hip_stream);
/* registers a model (copies its heightfield into the pool); up to MPPI_BATCH_MAX_MODELS */
mppi_status mppi_batch_add_model(mppi_batch *b, const mppi_model *model, int *slot_out);
/* admits an instance with HOST initial state x0 (nx) and nominal mu (12 * n_knots);
 * MPPI_EBUDGET if it does not fit in the remaining pool or the table is full
 * (nothing is changed then; the caller may queue the request).  K <= 4096,
 * H <= max_horizon; batch instances use the running cost (EINVAL for
 * MPPI_COST_TRACKING). */
mppi_status mppi_batch_admit(mppi_batch *b, int model_slot, const mppi_params *params, const float *x0,
                             const float *mu, int *id_out);
/* releases an instance; its memory is reused only by later stream-ordered admissions */
mppi_status mppi_batch_remove(mppi_batch *b, int id);
/* From the next step on, each control step s of instance id writes row (s mod cap) of
 * d_rec: the state the step started from (nx floats) followed by that step's updated,
 * unshifted knots mu' (12 * n_knots floats).  d_rec is a caller-owned DEVICE buffer of
 * cap * (nx + 12 * n_knots) floats that must stay allocated while recording; NULL stops
 * recording.  (Training data for the learned proposal: pairs of state and weighted plan.) */
mppi_status mppi_batch_record(mppi_batch *b, int id, float *d_rec, int cap);
/* one control step of every live instance: one graph launch on the bound stream */
mppi_status mppi_batch_step(mppi_batch *b);
/* persistent grid = blocks_per_cu x compute units; order 1 = longest horizon first */
mppi_status mppi_batch_set_tuning(mppi_batch *b, int blocks_per_cu, int order);
/* launch shape of the step's graph: mode 0 runs one persistent kernel per scene in use,
 * one after another; mode 1 runs a single persistent kernel over one queue that holds
 * every scene's tiles (each tile branches to its scene's code), so no scene's tail of
 * partly idle compute units is paid separately.  Results are the same in both modes.
 * EINVAL for another mode; takes effect at the next step (the graph is re-captured). */
mppi_status mppi_batch_set_launch_mode(mppi_batch *b, int mode);
/* the current blocks_per_cu, order and launch mode (NULL to skip) */
mppi_status mppi_batch_get_tuning(mppi_batch *b, int *blocks_per_cu, int *order, int *mode);
/* times `steps` control steps (after one untimed step) for each of the 16 candidate
 * tunings, blocks_per_cu in {2, 4, 8, 16} x order x launch mode, on the current instances
 * and keeps the fastest (advances every instance by the 16 (steps + 1) steps it runs);
 * the chosen launch mode is read back with mppi_batch_get_tuning */
mppi_status mppi_batch_autotune(mppi_batch *b, int steps, int *best_blocks_per_cu, int *best_order, float *best_ms);
/* synchronises and copies one instance's state, first control, nominal, accumulated
 * cost and step counter to HOST memory (NULL to skip) */
mppi_status mppi_batch_read(mppi_batch *b, int id, float *x, float *u0, float *mu, float *cost_acc, uint32_t *step);
mppi_status mppi_batch_stats(const mppi_batch *b, int *n_live, int *total_tiles, size_t *bytes_used,
                             size_t *bytes_pool);
const char *mppi_batch_last_error(const mppi_batch *b);

#ifdef __cplusplus
}
#endif
#endif
