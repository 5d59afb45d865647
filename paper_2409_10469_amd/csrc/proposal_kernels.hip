// Kernels of the learned-proposal control step that sit beside the rollout:
//   proposal_noise_kernel - effective noise e_n for a rollout of centre c with unit scale,
//                           so that theta_n = c + e_n: e_0 = 0 (the centre), e_1 = mu - c
//                           (the shifted nominal), e_n = sd * eps_n for n >= 2
//   features_kernel       - network input of one state: base xy relative to the origin,
//                           then the command
//   batch_features_kernel, batch_head_noise_kernel - the same for the learned-proposal
//                           instances of a batch, one row per instance
//   gate_kernel           - the fallback decision of a gated proposal step from the
//                           proposal's costs, before the plain samples are rolled out
//   pair_noise_kernel     - both sample sets as offsets from the nominal, so that one
//                           rollout launch covers them
#include <hip/hip_runtime.h>

#include "mppi_device.h"
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

// One workgroup: g[0] is the proposal's cost under the gate (its centre's, or the least
// over its samples other than the nominal), g[1] the nominal's (sample 1); the proposal
// is taken when g[0] is finite and not above g[1] -- the update kernel reads g and decides
// by the same comparison -- and skip is set then, so the plain rollout returns at once.
__global__ __launch_bounds__(256) void gate_kernel(int Kp, const float* __restrict__ costs_p, int best,
                                                   float* __restrict__ g, int* __restrict__ skip)
{
    __shared__ float sh[4];
    float m = __int_as_float(0x7f800000);
    if (best) {
        for (int n = threadIdx.x; n < Kp; n += 256) {
            const float c = costs_p[n];
            if (n != 1 && fabsf(c) <= 3.0e38f) m = fminf(m, c);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fminf(m, __shfl_xor(m, o, 64));
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
        __syncthreads();
        m = fminf(fminf(sh[0], sh[1]), fminf(sh[2], sh[3]));
    } else {
        m = costs_p[0];
    }
    if (threadIdx.x == 0) {
        const float nom = costs_p[1];
        g[0] = m;
        g[1] = nom;
        skip[0] = (fabsf(m) <= 3.0e38f && m <= nom) ? 1 : 0;
    }
}

hipError_t launch_gate(int Kp, const float* costs_p, int best, float* g, int* skip, hipStream_t st)
{
    hipLaunchKernelGGL(gate_kernel, dim3(1), dim3(256), 0, st, Kp, costs_p, best, g, skip);
    return hipGetLastError();
}

// The two sample sets of the concurrent gated step as offsets from the nominal mu, for one
// rollout launch centred on mu with unit scale: rows 0..K-1 of E hold the plain step's
// eps_n on entry (the sampler's order, E[n D + d]) and sigma eps_n on exit (0 for n = 0,
// the nominal), so the plain samples are mu + sigma eps_n whatever the proposal holds;
// rows K..K+Kp-1 receive the proposal's samples c + e_n as (c - mu) + e_n, each offset
// rounded once (sample 1, e_1 = mu - c, lands on mu exactly).  eps_n is also stored to
// eps_out[d K + n], where the update reads the plain step's noise.
__global__ __launch_bounds__(256) void pair_noise_kernel(int Kp, int K, int D, float sigma, float* __restrict__ E,
                                                         const float* __restrict__ e_prop,
                                                         const float* __restrict__ nominal,
                                                         const float* __restrict__ center,
                                                         float* __restrict__ eps_out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= (K + Kp) * D) return;
    const int n = i / D, d = i - n * D;
    if (n < K) {
        const float eps = E[i];
        E[i] = n == 0 ? 0.f : sigma * eps;
        eps_out[(size_t)d * K + n] = eps;
    } else {
        E[i] = (center[d] - nominal[d]) + e_prop[(size_t)(n - K) * D + d];
    }
}

hipError_t launch_pair_noise(int Kp, int K, int D, float sigma, float* E, const float* e_prop, const float* nominal,
                             const float* center, float* eps_out, hipStream_t st)
{
    const long n = (long)(K + Kp) * D;
    hipLaunchKernelGGL(pair_noise_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Kp, K, D, sigma, E,
                       e_prop, nominal, center, eps_out);
    return hipGetLastError();
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

__global__ __launch_bounds__(256) void batch_features_kernel(int np, const mppi::InstDesc* __restrict__ table,
                                                             const BatchPropRow* __restrict__ rows,
                                                             float* __restrict__ feat)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= np * 40) return;
    const int r = i / 40, t = i - r * 40;
    const BatchPropRow& pr = rows[r];
    const float* x = table[pr.row].x;
    feat[i] = t < 37 ? x[t] - (t == 0 ? pr.cmd_origin[3] : t == 1 ? pr.cmd_origin[4] : 0.f) : pr.cmd_origin[t - 37];
}

hipError_t launch_batch_features(int np, const mppi::InstDesc* table, const BatchPropRow* rows, float* feat,
                                 hipStream_t st)
{
    hipLaunchKernelGGL(batch_features_kernel, dim3((unsigned)((np * 40 + 255) / 256)), dim3(256), 0, st, np, table,
                       rows, feat);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void batch_head_noise_kernel(const mppi::InstDesc* __restrict__ table,
                                                               const BatchPropRow* __restrict__ rows,
                                                               const float* __restrict__ out,
                                                               const float* __restrict__ omean,
                                                               const float* __restrict__ ostd,
                                                               const float* __restrict__ rtab, float log_lo)
{
    __shared__ float sC[12 * 8], sSD[12 * 8];
    const BatchPropRow pr = rows[blockIdx.x];
    const mppi::InstDesc& I = table[pr.row];
    const int nk = pr.nk, D = 12 * nk, K = I.P.K, t = threadIdx.x;
    const float* o = out + (size_t)blockIdx.x * 144;
    if (t < D) {  // head: de-standardised mean and log-std of joint j, resampled to knot i
        const int j = t / nk, i = t - j * nk;
        const float* R = rtab + (size_t)(nk * 8 + i) * 6;
        float m = 0.f, s = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int d = j * 6 + k;
            const float sd = ostd[d];
            m += R[k] * (o[d] * sd + omean[d]);
            s += R[k] * (o[72 + d] + logf(sd));
        }
        s = fminf(fmaxf(s, log_lo), pr.log_hi);
        sC[t] = m;
        sSD[t] = expf(s);
    }
    __syncthreads();
    // noise: counter (d / 4, n, step, instance), Box-Muller on word pairs, as the sampler
    const uint32_t step = I.step[0];
    const int nb = (D + 3) >> 2;
    for (int idx = t; idx < K * nb; idx += 256) {
        const int cb = idx / K, n = idx - cb * K;
        uint32_t w[4] = {(uint32_t)cb, (uint32_t)n, step, I.P.instance};
        mppi::philox4x32_10(w, I.P.seed_lo, I.P.seed_hi);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float r = sqrtf(-2.0f * logf(mppi::u24<float>(w[2 * h])));
            float sn, co;
            sincospif(2.0f * mppi::u24<float>(w[2 * h + 1]), &sn, &co);
            const float g[2] = {r * co, r * sn};
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int d = 4 * cb + 2 * h + q;
                if (d < D) {
                    const float e = n == 0 ? 0.f : n == 1 ? I.mu[d] - sC[d] : sSD[d] * g[q];
                    I.eps[(size_t)d * K + n] = e;
                }
            }
        }
    }
    __syncthreads();  // the nominal has been read (n = 1) before the centre takes its place
    if (t < D) I.mu[t] = sC[t];
}

hipError_t launch_batch_head_noise(int np, const mppi::InstDesc* table, const BatchPropRow* rows, const float* out,
                                   const float* omean, const float* ostd, const float* rtab, float log_lo,
                                   hipStream_t st)
{
    hipLaunchKernelGGL(batch_head_noise_kernel, dim3((unsigned)np), dim3(256), 0, st, table, rows, out, omean, ostd,
                       rtab, log_lo);
    return hipGetLastError();
}

}  // namespace prop
