// Kernels of the learned-proposal control step that sit beside the rollout:
//   proposal_noise_kernel - effective noise e_n for a rollout of centre c with unit scale,
//                           so that theta_n = c + e_n: e_0 = 0 (the centre), e_1 = mu - c
//                           (the shifted nominal), e_n = sd * eps_n for n >= 2
//   features_kernel       - network input of one state: base xy relative to the origin,
//                           then the command
#include <hip/hip_runtime.h>

#include "proposal_launch.h"

namespace prop {

__global__ __launch_bounds__(256) void proposal_noise_kernel(int Kp, int D, float* __restrict__ e,
                                                             const float* __restrict__ center,
                                                             const float* __restrict__ sd,
                                                             const float* __restrict__ nominal)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= Kp * D) return;
    const int n = i / D, d = i - n * D;
    if (n == 0) e[i] = 0.f;
    else if (n == 1) e[i] = nominal[d] - center[d];
    else e[i] = sd[d] * e[i];
}

hipError_t launch_proposal_noise(int Kp, int D, float* e, const float* center, const float* sd, const float* nominal,
                                 hipStream_t st)
{
    const long n = (long)Kp * D;
    hipLaunchKernelGGL(proposal_noise_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Kp, D, e, center,
                       sd, nominal);
    return hipGetLastError();
}

__global__ void features_kernel(const float* __restrict__ x, const float* __restrict__ co, float* __restrict__ f)
{
    const int t = threadIdx.x;
    if (t < 37) f[t] = x[t] - (t == 0 ? co[3] : t == 1 ? co[4] : 0.f);
    else if (t < 40) f[t] = co[t - 37];
}

hipError_t launch_features(const float* x, const float* cmd_origin, float* feat, hipStream_t st)
{
    hipLaunchKernelGGL(features_kernel, dim3(1), dim3(64), 0, st, x, cmd_origin, feat);
    return hipGetLastError();
}

}  // namespace prop
