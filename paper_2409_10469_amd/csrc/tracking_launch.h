// Host-side launch interface of the Eq. 3 / Eq. 4 tracking-cost kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace track {

// cost parameters as the kernel reads them (mppi_tracking_cost plus the leg lengths)
struct TrackDev {
    float Q[36], R[12];
    float p_ref0[3], v_cmd[2];
    float period, duty, swing_h, stand_h, raibert_k;
    float box_w, box_goal[2];
    float l1, l2;          // thigh and calf lengths (inverse kinematics)
    int gait;
    int box;               // 1: the state carries a free box (Eq. 4 term)
};

struct TrackArgs {
    TrackDev c;
    const float* traj;     // K x (H+1) x nx rollout states (row 0: the start state)
    const double* B;       // knot interpolation H x nk
    const float* mu;       // nominal knots (12 nk)
    const float* eps;      // noise: eps[n * eps_sn + d * eps_sd]
    int eps_sn, eps_sd;
    float sigma;           // theta_n = mu + sigma eps_n for n >= 1, theta_0 = mu
    int K, H, nk, nx;
    float dt;
    uint32_t step;         // control-step counter: rollout step k is at gait time (step + k) dt
    float* costs;          // K sample costs (+inf when not finite)
};

// the gait table from the start state x0 (one workgroup) into `table`
// (tracking_table_bytes(H), 256-byte aligned device memory), then the cost with one 64-lane
// workgroup per sample; arith 0 evaluates in FP64, 1 in FP32
hipError_t launch_tracking_cost(int arith, const TrackArgs& a, const float* x0, void* table, hipStream_t st);
size_t tracking_lds_bytes(int arith, int H, int nk, int nx);
size_t tracking_table_bytes(int H);

}  // namespace track
