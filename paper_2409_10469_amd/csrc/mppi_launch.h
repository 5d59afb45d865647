// Host-side launch interface between the C ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mppi {

template <typename R>
struct ModelT;
using DevModelF = ModelT<float>;
using DevModelD = ModelT<double>;

// per-instance controller parameters as the kernels read them
struct DevParams {
    int K, H, nk, nx;
    float dt, sigma, inv_lambda, kp, kd;
    float w_h, h_ref, w_o, w_v, v_ref, w_tau, w_reach, w_box, goal_x, goal_y;
    uint32_t seed_lo, seed_hi, instance, step;
};

struct RolloutArgs {
    const double* B;       // spline basis H x nk (FP64)
    const float* hf;       // heightfield (scene 1)
    const float* mu;       // nominal knots 12 x nk
    const float* x0;       // initial state
    const float* eps_in;   // explicit noise or null
    int eps_sn, eps_sd;    // strides of eps_in (sample, dimension)
    float* eps_out;        // Philox noise store, D x K (when eps_in is null)
    float* costs;          // K
    float* traj;           // K x (H+1) x nx or null
    int samples_per_block; // samples per workgroup (4 lanes each)
    int direct;            // lane-split rollout: one value per step (nk == H) instead of the basis
    const int* skip;       // lane-split rollout: device flag; when set the launch does nothing
    int* input_status;     // lane-split rollout: set to 1 when x0 is not finite (then nothing is
                           // rolled out and every cost is +inf), to 0 otherwise; or null
};

struct UpdateArgs {
    const float* costs;
    const float* eps;
    int eps_sn, eps_sd;
    const float* mu;
    const float* S;        // shift matrix nk x nk
    float* knots_out;      // unshifted update or null
    float* nominal_out;    // shifted update or null
    float* u0_out;         // first control (12) or null
    float* weights_out;    // K or null
    int* status;           // [0]: 1 if no finite cost; [2]: 1 if a gated proposal step fell back
    // learned-proposal step (prop = 1): when the gate accepts, the update runs over the
    // proposal's Kp samples instead (costs_p, noise eps_p[n * D + d], centre mu_p, unit
    // scale); the gate accepts when gate is null (ungated) or gate[0] (the centre's cost)
    // is finite and not above gate[1] (the nominal's).  pstats, if set, counts
    // [accepted, proposal steps].
    int prop;
    int Kp;
    const float* gate;
    const float* costs_p;
    const float* eps_p;
    const float* mu_p;
    int* pstats;
};

hipError_t launch_sample(const DevParams& P, int D, float* eps, uint32_t* raw, hipStream_t st);
// arith: 0 = FP64 step arithmetic, 1 = FP32
hipError_t launch_rollout(const DevModelF& Mf, const DevModelD& Md, int arith, const DevParams& P,
                          const RolloutArgs& a, hipStream_t st);
// the lane-split rollout (16 lanes per sample); same arguments as launch_rollout, whose
// samples_per_block it ignores.  rollout16_fits: whether its LDS fits for the model.
hipError_t launch_rollout16(const DevModelF& Mf, const DevModelD& Md, int arith, const DevParams& P,
                            const RolloutArgs& a, hipStream_t st);
bool rollout16_fits(int arith, int scene, int hf_cells);
hipError_t launch_update(const DevParams& P, const UpdateArgs& a, hipStream_t st);
hipError_t launch_sim_step(const DevModelF& Mf, const DevModelD& Md, int arith, int n, int nx, const float* x,
                           const float* u, float kp, float kd, float dt, float* xo, float* tau, const float* hf,
                           hipStream_t st);

}  // namespace mppi

namespace mppi {

// ---------------------------------------------------------------------------------
// batched serving: one row of the device instance table
// ---------------------------------------------------------------------------------
constexpr int kTileSamples = 16;  // samples per 64-lane tile (one sample per quad)

struct InstDesc {
    DevParams P;                // K, H, nk, nx, dt, sigma, 1/lambda, gains, cost weights, seed, instance
    int scene, model, ntiles, tile0;
    int hf_cells;
    int explicit_eps;           // 1: eps holds the rollout noise (written before the step), 0: Philox
    const double* B;            // spline basis H x nk
    const float* S;             // shift matrix nk x nk
    const float* hf;            // heightfield of the model (scene 1)
    float* x;                   // current state (nx)
    float* mu;                  // nominal knots (12 nk)
    float* eps;                 // noise, D x K (dimension-major)
    float* costs;               // K
    float* w;                   // K unnormalised weights
    float* u0;                  // last first control (12)
    float* cost_acc;            // running cost of the closed loop
    int* done;                  // finished tiles of the current step
    uint32_t* step;             // control-step counter (Philox counter word)
    float* rec;                 // record rows [x, mu'] (nx + 12 nk floats) or null
    int rec_cap, pad1;          // rows in rec; step s writes row s mod rec_cap
};

template <typename R>
struct BatchArgs {
    const InstDesc* inst;
    const ModelT<R>* models;
    const int* tile_map;        // this scene's tiles -> instance row
    const int* total_tiles;     // number of this scene's tiles
    int* head;                  // this scene's work-queue head
    int* exited;                // blocks that found this scene's queue empty
};

hipError_t launch_batch(int arith, int scene, const void* args /* BatchArgs<R> */, int grid, size_t lds,
                        hipStream_t st);
// one persistent kernel for all scenes; its tile map entries are (row << 8 | tile of the row)
hipError_t launch_batch_all(int arith, const void* args /* BatchArgs<R> */, int grid, size_t lds, hipStream_t st);

}  // namespace mppi
