// Host-side launch interface between the C ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mppi {

template <typename R>
struct ModelT;
using DevModelF = ModelT<float>;
using DevModelD = ModelT<double>;
struct DevParams;

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
    int* status;           // 1 if no finite cost
};

hipError_t launch_sample(const DevParams& P, int D, float* eps, uint32_t* raw, hipStream_t st);
// arith: 0 = FP64 step arithmetic, 1 = FP32
hipError_t launch_rollout(const DevModelF& Mf, const DevModelD& Md, int arith, const DevParams& P,
                          const RolloutArgs& a, hipStream_t st);
hipError_t launch_update(const DevParams& P, const UpdateArgs& a, hipStream_t st);
hipError_t launch_sim_step(const DevModelF& Mf, const DevModelD& Md, int arith, int n, int nx, const float* x,
                           const float* u, float kp, float kd, float dt, float* xo, float* tau, const float* hf,
                           hipStream_t st);

}  // namespace mppi
