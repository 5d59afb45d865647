/*
 * mppi_policy.h -- C ABI of the learned sampling proposal.
 *
 * The paper leaves sampling from richer distributions to future work (Sec. V-B) and
 * cites offline-learned sampling distributions as related work (Sec. II-B).  This
 * library's proposal is a multilayer perceptron
 *     40 -> 512 -> 512 -> 512 -> 512 -> 144, SiLU between layers,
 * mapping (state, command) to a mean and a log standard deviation for each of the
 * 12 joints x 6 knots of the next plan.  It runs on the gfx950 matrix cores with BF16
 * operands and FP32 accumulation; FP32 master weights and Adam moments are kept beside
 * the BF16 copies the products read.
 *
 * Conventions (as in mppi.h):
 *  - d_* pointers are DEVICE pointers owned by the caller; others are host pointers.
 *  - The library never allocates device memory: the caller binds a workspace of
 *    mppi_policy_workspace_bytes() bytes (256-byte aligned).
 *  - Calls that launch work are asynchronous on the bound stream; a negative status
 *    means nothing was launched (mppi_policy_last_error describes why).
 *
 * Input features (40 floats per row, "raw"): the 37-float robot state of mppi.h with the
 * base x, y taken relative to the episode origin, then the command
 * (v_x reference, v_y reference, yaw-rate reference).  The network sees them standardised
 * with the policy's normalisation: (f - in_mean) / in_std.
 * Network output (144 floats per row, standardised): 72 means then 72 log-stds, both
 * joint-major (index j * 6 + k for knot k of joint j).  Training targets (72 floats per
 * row, raw knots) are standardised with (y - out_mean) / out_std; the loss is the
 * Gaussian negative log-likelihood averaged over rows and outputs,
 *     L = mean( (y_std - m)^2 exp(-2 s) / 2 + s ).
 *
 * Parameter layout (flat FP32, 882832 values): per layer l, W_l (fan_in x fan_out,
 * row-major, W[i][o]) then b_l (fan_out).
 */
#ifndef MPPI_POLICY_H
#define MPPI_POLICY_H

#include <stddef.h>
#include <stdint.h>

#include "mppi.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MPPI_POLICY_IN 40
#define MPPI_POLICY_OUT 144
#define MPPI_POLICY_KNOTS 6
#define MPPI_POLICY_TARGET 72

typedef struct mppi_policy mppi_policy;

/* Number of parameters (882832). */
int mppi_policy_n_params(void);

/* Creates a policy able to process up to max_batch rows per call (1..65536).  With
 * ckpt_path NULL the weights are drawn from a seeded uniform(-1/sqrt(fan_in),
 * 1/sqrt(fan_in)) (biases likewise), Adam moments are zero and the normalisation is the
 * identity; otherwise all of these are read from a file written by mppi_policy_save
 * (EINVAL if it is missing or malformed). */
mppi_status mppi_policy_create(const char *ckpt_path, uint64_t seed, int max_batch, mppi_policy **out);
void mppi_policy_destroy(mppi_policy *pol);
size_t mppi_policy_workspace_bytes(const mppi_policy *pol);
/* Binds workspace and stream and uploads weights, moments and normalisation. */
mppi_status mppi_policy_bind(mppi_policy *pol, void *d_workspace, size_t bytes, void *hip_stream);
/* Host arrays in_mean[40], in_std[40], out_mean[72], out_std[72]; stds must be > 0. */
mppi_status mppi_policy_set_normalization(mppi_policy *pol, const float *in_mean, const float *in_std,
                                          const float *out_mean, const float *out_std);
/* Copies the normalisation to host arrays (same order and sizes; NULL to skip one). */
mppi_status mppi_policy_get_normalization(const mppi_policy *pol, float *in_mean, float *in_std, float *out_mean,
                                          float *out_std);
/* FP32 master parameters (n_params floats, device) out / in.  set_params also refreshes
 * the BF16 copies; it leaves the Adam moments and step count unchanged. */
mppi_status mppi_policy_get_params(mppi_policy *pol, float *d_params);
mppi_status mppi_policy_set_params(mppi_policy *pol, const float *d_params);
/* Forward pass of B rows of raw features d_in (B x 40) into d_out (B x 144,
 * standardised network output); 1 <= B <= max_batch. */
mppi_status mppi_policy_forward(mppi_policy *pol, const float *d_in, int B, float *d_out);
/* Loss and gradient over the B rows d_index[0..B) (or rows 0..B-1 if d_index is NULL)
 * of d_in (x 40) and d_target (x 72): d_grad receives n_params floats in the parameter
 * layout, d_loss one float (either may be NULL).  Every index must be a row that d_in
 * and d_target hold: the indices are device data the library does not read on the host,
 * and an index outside the caller's rows makes the kernels read outside those buffers. */
mppi_status mppi_policy_grad(mppi_policy *pol, const float *d_in, const float *d_target, const int *d_index, int B,
                             float *d_grad, float *d_loss);
/* The loss alone (the held-out negative log-likelihood): d_loss receives one float, the
 * loss mppi_policy_grad would report for the same rows, bit for bit (same forward pass,
 * loss kernel and summation order); nothing is trained.  Same index rule as
 * mppi_policy_grad; d_loss must not be NULL. */
mppi_status mppi_policy_nll(mppi_policy *pol, const float *d_in, const float *d_target, const int *d_index, int B,
                            float *d_loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; Kingma and Ba) with
 * the given gradient (n_params floats, device) and learning rate. */
mppi_status mppi_policy_adam(mppi_policy *pol, const float *d_grad, float lr);
/* mppi_policy_grad followed by mppi_policy_adam on its gradient (same index rule). */
mppi_status mppi_policy_train_step(mppi_policy *pol, const float *d_in, const float *d_target, const int *d_index,
                                   int B, float lr, float *d_loss);
/* Adam steps taken so far. */
int mppi_policy_steps(const mppi_policy *pol);
/* Synchronises the stream and writes weights, moments, step count and normalisation
 * to a binary file ("MPPIPOL1" header, then little-endian int32 n_params and step,
 * 224 normalisation floats, and the parameters, first and second moments as FP32). */
mppi_status mppi_policy_save(mppi_policy *pol, const char *path);
/* Proposal of a controller with n_knots knots per joint from one row of network output
 * d_out (144 floats, device): means and log-stds de-standardised, resampled from the 6
 * knots to n_knots knots at the same fractions of the horizon (not-a-knot cubic spline),
 * log-std clamped to [log 0.02, log sigma_max]; d_center and d_sd receive 12 * n_knots
 * floats (joint-major). */
mppi_status mppi_policy_head(mppi_policy *pol, const float *d_out, int n_knots, float sigma_max, float *d_center,
                             float *d_sd);
const char *mppi_policy_last_error(const mppi_policy *pol);

/* ---- training data ----------------------------------------------------------------
 * Training pairs from closed-loop records (the rows mppi_batch_record writes, all of one
 * knot count), on the given stream; needs no policy.  d_records holds n_rec records of
 * steps rows, record r at d_records + r * steps * (37 + 12 * n_knots): the state, then
 * the unshifted knots (joint-major).  A record's pairs are its rows before the first row
 * with a non-finite value or a base height (state index 2) not above fall_z; d_count[r]
 * receives their number.  Row k < d_count[r] of record r gives, at index r * steps + k,
 *   d_feat (x 40): the raw features above -- the state with base x, y taken relative to
 *     the record's origin -- and the command (v, 0, 0);
 *   d_target (x 72): the knots resampled to 6 per joint at the same fractions of the
 *     horizon (the not-a-knot spline through the record's n_knots knots; the identity
 *     for 6), joint-major.
 * Later rows of d_feat and d_target are not written.  d_origin_cmd: n_rec x 3 floats
 * (origin x, origin y, v).  2 <= n_knots <= 8.  Errors: EINVAL (sizes, null buffers, a
 * non-finite fall_z; mppi_policy_last_error(NULL) says which), EHIP. */
mppi_status mppi_policy_pairs(int n_rec, int steps, int n_knots, const float *d_records, const float *d_origin_cmd,
                              float fall_z, float *d_feat, float *d_target, int *d_count, void *hip_stream);

/* ---- controller side -------------------------------------------------------------
 * One control step with an explicit proposal (mean d_center, std d_sd; 12 * n_knots
 * floats each, device): k_prop samples theta_0 = center, theta_1 = the current (shifted)
 * nominal, theta_n = center + sd * eps_n for 2 <= n < k_prop, with eps_n drawn from the
 * same Philox counters as a plain step (Box-Muller evaluated as mppi_sample does).
 * A gated step takes the proposal when its cost under the gate (GATE_COST: the centre's
 * rollout cost; GATE_BEST: the least cost of its samples other than the nominal) is finite
 * and not above the nominal's, and Eq. 1 and Eq. 2 then run over these k_prop samples;
 * otherwise the step is a plain step with K samples around the nominal (the fallback).
 * Then, as in mppi_step, the first control goes to d_u0_out, the nominal is shifted and
 * the step counter advances.  The decision is made on the device, so the call does not
 * synchronise.  With the lane-split rollout the plain K samples are rolled out only on a
 * fallback (after the proposal and the gate, on the bound stream): a step rolls out
 * k_prop samples, or k_prop + K one rollout after the other when it falls back.  With
 * the quad rollout the plain K samples are rolled out beside the proposal's, on an
 * internal stream that mppi_bind creates (side by side only while the process's streams
 * do not outnumber its hardware queues).  With MPPI_PROPOSAL_CONCURRENT added to the gate
 * (either rollout) one rollout launch covers both sets on every step: k_prop + K samples
 * in about one rollout's time, whatever the process's other streams.  That launch is
 * centred on the nominal mu: the plain samples are mu + sigma eps_n (the product rounded
 * once in FP32), so whatever the proposal holds cannot reach the fallback, and the
 * proposal's are mu + ((c - mu) + e_n) (the offset rounded once; theta_1 = mu exactly).
 * The step agrees with the sequential gate within that rounding (the workspace holds
 * both sets).  MPPI_PROPOSAL_GATE_NONE always takes the proposal
 * branch (the nominal still competes as sample 1) and rolls out only the proposal.
 * 2 <= k_prop <= K.  The proposal steps use the running cost (EINVAL for a controller
 * created with MPPI_COST_TRACKING). */
enum {
    MPPI_PROPOSAL_GATE_COST = 0, /* proposal only if its centre's cost is finite and not above the nominal's */
    MPPI_PROPOSAL_GATE_NONE = 1, /* always the proposal's k_prop samples */
    MPPI_PROPOSAL_GATE_BEST = 2, /* proposal only if its best sample other than the nominal is finite and not
                                    above the nominal's cost */
    MPPI_PROPOSAL_CONCURRENT = 4 /* added to GATE_COST or GATE_BEST: the fallback's samples are rolled out with
                                    the proposal's in one launch on every step (latency of one rollout) */
};
mppi_status mppi_step_proposal(mppi_ctx *ctx, const float *d_x0, const float *d_center, const float *d_sd,
                               int k_prop, int gate, float *d_u0_out);
/* Makes every later mppi_step of ctx use the policy: features of the current state and
 * command (host cmd[3]) relative to the host origin_xy[2], a forward pass, the head, and
 * mppi_step_proposal with k_prop samples and the given gate.  The policy's kernels then run on ctx's
 * stream; the policy must not be used on another stream meanwhile.  pol NULL switches
 * the proposal off.  Requires a 37-float state model and the running cost. */
mppi_status mppi_set_proposal(mppi_ctx *ctx, mppi_policy *pol, int k_prop, int gate, const float *cmd,
                              const float *origin_xy);
/* How many proposal steps ran and how many were accepted: device counters (reset by
 * mppi_bind), read back with a synchronisation of the bound stream. */
mppi_status mppi_proposal_stats(mppi_ctx *ctx, int *accepted, int *steps);

/* ---- batched serving side ---------------------------------------------------------
 * Makes instance id of a batch (mppi.h) take its samples from the policy, ungated: each
 * mppi_batch_step then runs, for all such instances together and as the first nodes of
 * the batch's graph, the features of each one's current state, one forward pass over
 * them as a batch, and the head; the instance's K admitted samples are then theta_0 = centre,
 * theta_1 = its shifted nominal, theta_n = centre + sd * eps_n (its own Philox counters,
 * as mppi_step_proposal draws them), and Eq. 1 / Eq. 2 over them give the new nominal,
 * as mppi_step_proposal does with MPPI_PROPOSAL_GATE_NONE.  The admitted sigma is the
 * upper clamp of the proposal's std.  cmd[3] and origin_xy[2] are host arrays copied
 * here.  Every proposal instance of a batch shares one policy, whose max_batch must
 * cover their number; its kernels run on the batch's stream, and it must not be used on
 * another stream while steps are queued.  pol NULL returns the instance to plain
 * sampling.  Requires a 37-float state model and K >= 2.  Launches no kernel; the first
 * call copies the head's resampling table into the batch workspace and synchronises the
 * batch stream. */
mppi_status mppi_batch_set_proposal(mppi_batch *b, int id, mppi_policy *pol, const float *cmd,
                                    const float *origin_xy);

#ifdef __cplusplus
}
#endif
#endif
