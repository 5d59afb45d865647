// Host-side launch interface of the proposal-step helper kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "mppi_launch.h"

namespace prop {
// one learned-proposal instance of a batch: its row of the instance table, its knots per
// joint, the log of its upper std clamp, and its command and origin (cmd[3], origin[2])
struct BatchPropRow {
    int row;
    int nk;
    float log_hi;
    float cmd_origin[5];
};
static_assert(sizeof(BatchPropRow) == 32, "BatchPropRow is 32 bytes");

// e (Kp x D, sample-major) holds standard Gaussian noise on entry; on exit row 0 is 0,
// row 1 is nominal - center and row n >= 2 is sd * e_n
hipError_t launch_proposal_noise(int Kp, int D, float* e, const float* center, const float* sd, const float* nominal,
                                 hipStream_t st);
// the gate of a proposal step from the proposal's Kp costs (best = 0: its centre's cost,
// 1: the least cost of its samples other than the nominal, sample 1) against the
// nominal's: g = {that cost, nominal's}, skip = 1 when the proposal is taken
hipError_t launch_gate(int Kp, const float* costs_p, int best, float* g, int* skip, hipStream_t st);
// the concurrent gated step: E ((K + Kp) x D) as offsets from the nominal, rows 0..K-1
// from the plain step's eps (sigma eps_n, 0 for n = 0; eps copied to eps_out, D x K),
// rows K.. from the proposal's e_prop (Kp x D, offsets from the centre): (c - mu) + e_n
hipError_t launch_pair_noise(int Kp, int K, int D, float sigma, float* E, const float* e_prop, const float* nominal,
                             const float* center, float* eps_out, hipStream_t st);
// state x (37 floats) and cmd_origin = (cmd[3], origin[2]) -> 40 raw features
hipError_t launch_features(const float* x, const float* cmd_origin, float* feat, hipStream_t st);
// raw features (np x 40) of the proposal rows' current states
hipError_t launch_batch_features(int np, const mppi::InstDesc* table, const BatchPropRow* rows, float* feat,
                                 hipStream_t st);
// per proposal row (one workgroup each): the head of its network output row (centre and
// std at its nk knots, resampled with rtab[nk][i][k], rtab is 9 x 8 x 6 floats), then the
// instance's rollout noise, dimension-major e[d K + n]: 0 for n = 0, nominal - centre for
// n = 1, std * Philox Gaussian (the sampler's counters at the instance's step) for n >= 2;
// finally the centre replaces the nominal
hipError_t launch_batch_head_noise(int np, const mppi::InstDesc* table, const BatchPropRow* rows, const float* out,
                                   const float* omean, const float* ostd, const float* rtab, float log_lo,
                                   hipStream_t st);
}  // namespace prop
