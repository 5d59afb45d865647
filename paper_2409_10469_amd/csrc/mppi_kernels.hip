// HIP kernels of the whole-body MPPI hot path for gfx950:
//   sample_kernel   - counter-based Gaussian knot noise (Sec. II-B sampling)
//   rollout_kernel  - fused spline + PD + dynamics + running cost over the horizon
//                     (Algorithm 1 inner loops); one sample per quad of lanes
//   update_kernel   - Eq. 1 weights (log-sum-exp shift by the minimum cost) and the
//                     Eq. 2 weighted knot mean, fused with the first-control extraction
//                     and warm-start shift (Algorithm 1 last steps); one block per joint
//   sim_step_kernel - one dynamics step of many states (closed-loop plant)
#include "mppi_device.h"
#include "mppi_launch.h"

namespace mppi {

// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sample_kernel(DevParams P, int D, float* __restrict__ eps,
                                                     uint32_t* __restrict__ raw)
{
    const int nb = (D + 3) >> 2;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= P.K * nb) return;
    const int n = gid / nb, c = gid - n * nb;
    uint32_t w[4] = {(uint32_t)c, (uint32_t)n, P.step, P.instance};
    philox4x32_10(w, P.seed_lo, P.seed_hi);
    if (raw) {
#pragma unroll
        for (int i = 0; i < 4; ++i) raw[(size_t)n * 4 * nb + 4 * c + i] = w[i];
    }
    if (eps) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float r = sqrtf(-2.0f * logf(u24<float>(w[2 * h])));
            float s, co;
            sincospif(2.0f * u24<float>(w[2 * h + 1]), &s, &co);
            const int d0 = 4 * c + 2 * h;
            if (d0 < D) eps[(size_t)n * D + d0] = r * co;
            if (d0 + 1 < D) eps[(size_t)n * D + d0 + 1] = r * s;
        }
    }
}

// ---------------------------------------------------------------------------------
// Rollout of the samples of one workgroup: quad q of the block handles sample
// n = n_base + q.  sB (spline basis, type R) and sHF (heightfield) are in LDS.
// eps addressing: eps_in[n * eps_sn + d * eps_sd] when given; otherwise Philox noise,
// stored to eps_out[d * K + n] (dimension-major for the update's coalesced reads).
// The state is rounded to FP32 after every step; the step itself runs in R.
// ---------------------------------------------------------------------------------
template <int SCENE, typename R>
__device__ __forceinline__ void rollout_samples(const ModelT<R>& M, const DevParams& P, const R* sB, const float* sHF,
                                                R* sTh,
                                                const float* __restrict__ mu, const float* __restrict__ x0,
                                                const float* __restrict__ eps_in, int eps_sn, int eps_sd,
                                                float* __restrict__ eps_out, float* __restrict__ costs,
                                                float* __restrict__ traj, int n_base)
{
    const int tid = threadIdx.x;
    const int leg = tid & 3;
    const int n = n_base + (tid >> 2);
    const bool valid = n < P.K;
    const int ns = valid ? n : P.K - 1;
    const int nk = P.nk;
    const R sigma = P.sigma;

    // knots of this leg's three joints, theta = mu + sigma eps (sample 0 is the nominal),
    // kept in LDS (sTh: 3 * kMaxKnots values per lane) to spare registers
    R* th = sTh + (size_t)tid * 3 * kMaxKnots;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < kMaxKnots; ++i) {
            if (i < nk) {
                const int d = (3 * leg + j) * nk + i;
                R e;
                if (eps_in) {
                    e = eps_in[(size_t)ns * eps_sn + (size_t)d * eps_sd];
                } else {
                    e = gauss_elem<R>(P, (uint32_t)ns, (uint32_t)d);
                    if (valid && eps_out) eps_out[(size_t)d * P.K + n] = (float)e;
                }
                th[j * kMaxKnots + i] = R(mu[d]) + (ns ? sigma * e : R(0));
            }
        }

    Base<R> b;
    Leg<R> lg;
    BoxS<R> bx{};
    load_state(x0, leg, b, lg);
    if constexpr (SCENE == 3) load_box(x0, bx);
    float* tr = (traj && valid) ? traj + (size_t)n * (P.H + 1) * P.nx : nullptr;
    if (tr) {
        store_state(tr, leg, b, lg);
        if (SCENE == 3 && leg == 0) store_box(tr, bx);
    }

    const R dt = P.dt, kp = P.kp, kd = P.kd;
    R L = R(0);
    for (int k = 0; k < P.H; ++k) {
        R u[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            R s = R(0);
#pragma unroll
            for (int i = 0; i < kMaxKnots; ++i)
                if (i < nk) s += sB[k * nk + i] * th[j * kMaxKnots + i];
            u[j] = s;
        }
        R tau2;
        quad_step<SCENE, R>(M, sHF, dt, kp, kd, leg, b, lg, bx, u, tau2);
        round_state(b, lg);
        if constexpr (SCENE == 3) round_box(bx);
        L += dt * stage_cost<SCENE>(P, b, bx, tau2);
        if (tr) {
            store_state(tr + (size_t)(k + 1) * P.nx, leg, b, lg);
            if (SCENE == 3 && leg == 0) store_box(tr + (size_t)(k + 1) * P.nx, bx);
        }
    }
    float Lf = (float)L;
    if (!(fabsf(Lf) <= 3.0e38f)) Lf = __int_as_float(0x7f800000);  // non-finite -> +inf
    if (valid && leg == 0) costs[n] = Lf;
}

template <typename R>
__device__ __forceinline__ void stage_lds(const DevParams& P, int scene, int hf_cells, const double* __restrict__ gB,
                                          const float* __restrict__ ghf, R* sB, float* sHF)
{
    for (int i = threadIdx.x; i < P.H * P.nk; i += blockDim.x) sB[i] = (R)gB[i];
    if (scene == 1)
        for (int i = threadIdx.x; i < hf_cells; i += blockDim.x) sHF[i] = ghf[i];
}

// standalone rollout: block of 4*SPB lanes handles SPB consecutive samples
template <int SCENE, typename R>
__global__ __launch_bounds__(256) void rollout_kernel(ModelT<R> M, DevParams P, const double* __restrict__ gB,
                                                      const float* __restrict__ ghf, const float* __restrict__ mu,
                                                      const float* __restrict__ x0, const float* __restrict__ eps_in,
                                                      int eps_sn, int eps_sd, float* __restrict__ eps_out,
                                                      float* __restrict__ costs, float* __restrict__ traj)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    R* sB = reinterpret_cast<R*>(lds_raw);
    R* sTh = sB + P.H * P.nk;
    float* sHF = reinterpret_cast<float*>(sTh + blockDim.x * 3 * kMaxKnots);
    stage_lds(P, SCENE, M.hf_nx * M.hf_ny, gB, ghf, sB, sHF);
    __syncthreads();
    rollout_samples<SCENE, R>(M, P, sB, sHF, sTh, mu, x0, eps_in, eps_sn, eps_sd, eps_out, costs, traj,
                              blockIdx.x * (blockDim.x >> 2));
}

// ---------------------------------------------------------------------------------
// Update: block j (one per joint, 1024 lanes) recomputes L_min and sum exp over all K
// costs, then the weighted noise sums for its nk knots.  Every reduction is a wave
// butterfly (its result is the same in every lane, since each pairwise sum is
// commutative) followed by the 16 per-wave values added in wave order, so the result is
// deterministic.  The lane count keeps the walks over K short (one pass at K = 1024,
// four at 4096): the kernel is bound by the latency of those passes, not by bandwidth.
// ---------------------------------------------------------------------------------
constexpr int kUpdThreads = 1024;
constexpr int kUpdUnroll = 2;  // samples per thread whose loads are issued together
constexpr int kUpdWaves = kUpdThreads / 64;

__device__ __forceinline__ float wave_reduce(float v, bool is_min)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float u = __shfl_xor(v, o, 64);
        v = is_min ? fminf(v, u) : v + u;
    }
    return v;
}

// all lanes return the block's reduction (sh: kUpdWaves floats)
__device__ __forceinline__ float block_reduce(float v, float* sh, bool is_min)
{
    v = wave_reduce(v, is_min);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = sh[0];
#pragma unroll
    for (int w = 1; w < kUpdWaves; ++w) r = is_min ? fminf(r, sh[w]) : r + sh[w];
    __syncthreads();
    return r;
}

// knots per joint up to kMaxUpdKnots (the direct representation has one per control
// step): the weighted noise sums run over chunks of kMaxKnots knots, one pass over K each
constexpr int kMaxUpdKnots = 256;

__global__ __launch_bounds__(kUpdThreads) void update_kernel(DevParams P, UpdateArgs a)
{
    __shared__ float sh[kUpdWaves];
    __shared__ float acc_w[kMaxKnots][kUpdWaves];
    __shared__ float mup[kMaxUpdKnots];
    const int j = blockIdx.x, t = threadIdx.x, nk = P.nk;
    // a proposal step whose gate accepts updates over the proposal's samples
    const bool prop = a.prop && (!a.gate || (fabsf(a.gate[0]) <= 3.0e38f && a.gate[0] <= a.gate[1]));
    const int K = prop ? a.Kp : P.K;
    const float* __restrict__ costs = prop ? a.costs_p : a.costs;
    const float* __restrict__ eps = prop ? a.eps_p : a.eps;
    const int eps_sn = prop ? 12 * nk : a.eps_sn, eps_sd = prop ? 1 : a.eps_sd;
    const float* mu = prop ? a.mu_p : a.mu;
    const float sigma = prop ? 1.f : P.sigma;
    // the passes over K take kUpdUnroll samples per thread at a time and issue all their
    // loads before using any, so a pass costs one memory round trip per kUpdUnroll
    // samples; each thread still visits its samples in increasing order
    float lmin = __int_as_float(0x7f800000);
    for (int n0 = t; n0 < K; n0 += kUpdUnroll * kUpdThreads) {
        float c[kUpdUnroll];
#pragma unroll
        for (int u = 0; u < kUpdUnroll; ++u) {
            const int n = n0 + u * kUpdThreads;
            c[u] = n < K ? costs[n] : __int_as_float(0x7f800000);
        }
#pragma unroll
        for (int u = 0; u < kUpdUnroll; ++u)
            if (fabsf(c[u]) <= 3.0e38f) lmin = fminf(lmin, c[u]);
    }
    lmin = block_reduce(lmin, sh, true);
    const bool none = !(fabsf(lmin) <= 3.0e38f);
    float s = 0.f;
    for (int c0 = 0; c0 < nk; c0 += kMaxKnots) {
        float acc[kMaxKnots];
#pragma unroll
        for (int i = 0; i < kMaxKnots; ++i) acc[i] = 0.f;
        if (!none) {
            for (int n0 = t; n0 < K; n0 += kUpdUnroll * kUpdThreads) {
                float c[kUpdUnroll], ev[kUpdUnroll][kMaxKnots];
#pragma unroll
                for (int u = 0; u < kUpdUnroll; ++u) {
                    const int n = n0 + u * kUpdThreads;
                    c[u] = n < K ? costs[n] : __int_as_float(0x7f800000);
#pragma unroll
                    for (int i = 0; i < kMaxKnots; ++i)
                        ev[u][i] = (n < K && n > 0 && c0 + i < nk)
                                       ? eps[(size_t)n * eps_sn + (size_t)(j * nk + c0 + i) * eps_sd]
                                       : 0.f;
                }
#pragma unroll
                for (int u = 0; u < kUpdUnroll; ++u) {
                    const int n = n0 + u * kUpdThreads;
                    if (n >= K) continue;
                    const float e = (fabsf(c[u]) <= 3.0e38f) ? expf(-(c[u] - lmin) * P.inv_lambda) : 0.f;
                    if (c0 == 0) s += e;
                    if (n > 0) {
#pragma unroll
                        for (int i = 0; i < kMaxKnots; ++i)
                            if (c0 + i < nk) acc[i] += e * ev[u][i];
                    }
                }
            }
        }
        if (c0 == 0) s = block_reduce(s, sh, false);
#pragma unroll
        for (int i = 0; i < kMaxKnots; ++i) {
            const float r = wave_reduce(acc[i], false);
            if ((t & 63) == 0) acc_w[i][t >> 6] = r;
        }
        __syncthreads();
        if (t < kMaxKnots && c0 + t < nk) {
            float acc_t = acc_w[t][0];
            for (int w = 1; w < kUpdWaves; ++w) acc_t += acc_w[t][w];
            const float m = mu[j * nk + c0 + t];
            mup[c0 + t] = none ? m : m + sigma * (acc_t / s);
        }
        __syncthreads();
    }
    for (int q = t; q < nk; q += kUpdThreads) {
        if (a.knots_out) a.knots_out[j * nk + q] = mup[q];
        if (a.nominal_out) {
            float v = 0.f;
            for (int l = 0; l < nk; ++l) v += a.S[q * nk + l] * mup[l];
            a.nominal_out[j * nk + q] = v;
        }
    }
    if (t == 0 && a.u0_out) a.u0_out[j] = mup[0];
    if (j == 0 && a.weights_out) {
        const float is = none ? 0.f : 1.f / s;
        for (int n0 = t; n0 < K; n0 += kUpdUnroll * kUpdThreads) {
            float c[kUpdUnroll];
#pragma unroll
            for (int u = 0; u < kUpdUnroll; ++u) {
                const int n = n0 + u * kUpdThreads;
                c[u] = n < K ? costs[n] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kUpdUnroll; ++u) {
                const int n = n0 + u * kUpdThreads;
                if (n < K)
                    a.weights_out[n] =
                        (!none && fabsf(c[u]) <= 3.0e38f) ? expf(-(c[u] - lmin) * P.inv_lambda) * is : 0.f;
            }
        }
    }
    if (j == 0 && t == 0) {
        if (a.status) {
            a.status[0] = none ? 1 : 0;
            a.status[2] = (a.prop && !prop) ? 1 : 0;
        }
        if (a.prop && a.pstats) {
            a.pstats[0] += prop ? 1 : 0;
            a.pstats[1] += 1;
        }
    }
}

// ---------------------------------------------------------------------------------
template <int SCENE, typename R>
__global__ __launch_bounds__(256) void sim_step_kernel(ModelT<R> M, int nstate, int nx, const float* __restrict__ x,
                                                       const float* __restrict__ u, float kp, float kd, float dt,
                                                       float* __restrict__ xo, float* __restrict__ tau_out,
                                                       const float* __restrict__ ghf)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float* sHF = reinterpret_cast<float*>(lds_raw);
    const int tid = threadIdx.x;
    if constexpr (SCENE == 1) {
        const int nhf = M.hf_nx * M.hf_ny;
        for (int i = tid; i < nhf; i += blockDim.x) sHF[i] = ghf[i];
    }
    __syncthreads();
    const int leg = tid & 3;
    const int n = blockIdx.x * (blockDim.x >> 2) + (tid >> 2);
    const bool valid = n < nstate;
    const int ns = valid ? n : nstate - 1;
    Base<R> b;
    Leg<R> lg;
    BoxS<R> bx{};
    load_state(x + (size_t)ns * nx, leg, b, lg);
    if constexpr (SCENE == 3) load_box(x + (size_t)ns * nx, bx);
    R uu[3], tauv[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        uu[j] = u[(size_t)ns * 12 + 3 * leg + j];
        tauv[j] = R(kp) * (uu[j] - lg.q[j]) - R(kd) * lg.qd[j];
    }
    R tau2;
    quad_step<SCENE, R>(M, sHF, R(dt), R(kp), R(kd), leg, b, lg, bx, uu, tau2);
    if (!valid) return;
    store_state(xo + (size_t)n * nx, leg, b, lg);
    if (SCENE == 3 && leg == 0) store_box(xo + (size_t)n * nx, bx);
    if (tau_out) {
#pragma unroll
        for (int j = 0; j < 3; ++j) tau_out[(size_t)n * 12 + 3 * leg + j] = (float)tauv[j];
    }
}

// ---------------------------------------------------------------------------------
// Batched serving: a persistent kernel of one-wave workgroups pops (instance, tile)
// items from an atomic queue; a tile is 16 samples of one instance.  The workgroup that
// completes an instance's last tile runs that instance's tail: Eq. 1 weights, the Eq. 2
// update, first control, shift, one plant step of the instance's state with that control
// and its running cost.  No workgroup ever waits on another; the last workgroup to find
// the queue empty resets it for the next launch, so the same graph can be replayed.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

template <int SCENE, typename R>
__device__ __forceinline__ void plant_step(const ModelT<R>& M, const DevParams& P, const float* sHF, float* x,
                                           const float* u0, float* cost_acc)
{
    const int leg = threadIdx.x & 3;
    Base<R> b;
    Leg<R> lg;
    BoxS<R> bx{};
    load_state(x, leg, b, lg);
    if constexpr (SCENE == 3) load_box(x, bx);
    R u[3] = {R(u0[3 * leg]), R(u0[3 * leg + 1]), R(u0[3 * leg + 2])};
    R tau2;
    quad_step<SCENE, R>(M, sHF, R(P.dt), R(P.kp), R(P.kd), leg, b, lg, bx, u, tau2);
    const R l = stage_cost<SCENE>(P, b, bx, tau2);
    __syncthreads();  // every lane has read x
    if (threadIdx.x < 4) {
        store_state(x, leg, b, lg);
        if (SCENE == 3 && leg == 0) store_box(x, bx);
        if (leg == 0) cost_acc[0] += (float)(R(P.dt) * l);
    }
}

template <int SCENE, typename R>
__device__ __forceinline__ void instance_tail(const InstDesc& I, const DevParams& P, const ModelT<R>& M, const float* sHF,
                              float* sMup)
{
    const int t = threadIdx.x, K = P.K, nk = P.nk, D = 12 * nk;
    float lmin = __int_as_float(0x7f800000);
    for (int n = t; n < K; n += 64) {
        const float c = I.costs[n];
        if (fabsf(c) <= 3.0e38f) lmin = fminf(lmin, c);
    }
    lmin = wave_min(lmin);
    const bool none = !(fabsf(lmin) <= 3.0e38f);
    float s = 0.f;
    for (int n = t; n < K; n += 64) {
        const float c = I.costs[n];
        const float e = (!none && fabsf(c) <= 3.0e38f) ? expf(-(c - lmin) * P.inv_lambda) : 0.f;
        I.w[n] = e;
        s += e;
    }
    s = wave_sum(s);
    __syncthreads();  // weights visible to the whole workgroup (one wave)
    for (int d = 0; d < D; ++d) {
        float acc = 0.f;
        for (int n = t; n < K; n += 64)
            if (n > 0) acc += I.w[n] * I.eps[(size_t)d * K + n];
        acc = wave_sum(acc);
        if (t == 0) sMup[d] = none ? I.mu[d] : I.mu[d] + P.sigma * (acc / s);
    }
    __syncthreads();
    if (t < 12) I.u0[t] = sMup[t * nk];
    for (int q = t; q < D; q += 64) {
        const int j = q / nk, i = q - j * nk;
        float v = 0.f;
        for (int l = 0; l < nk; ++l) v += I.S[i * nk + l] * sMup[j * nk + l];
        I.mu[q] = v;
    }
    if (I.rec) {  // the state this step started from and its updated knots
        float* row = I.rec + (size_t)(I.step[0] % (uint32_t)I.rec_cap) * (P.nx + D);
        for (int q = t; q < P.nx; q += 64) row[q] = I.x[q];
        for (int q = t; q < D; q += 64) row[P.nx + q] = sMup[q];
    }
    __syncthreads();
    plant_step<SCENE, R>(M, P, sHF, I.x, I.u0, I.cost_acc);
    if (t == 0) {
        I.step[0] += 1u;
        I.done[0] = 0;
    }
}

// one tile of one instance: stage its basis (and heightfield) in LDS, roll out its 16
// samples; the workgroup that completes the instance's last tile runs its tail
template <int SCENE, typename R>
__device__ __forceinline__ void batch_tile(const InstDesc& I, const ModelT<R>& M, int n_base, unsigned char* lds,
                                           float* sMup, int* s_last)
{
    DevParams P = I.P;
    P.step = I.step[0];
    R* sB = reinterpret_cast<R*>(lds);
    R* sTh = sB + P.H * P.nk;
    float* sHF = reinterpret_cast<float*>(sTh + 64 * 3 * kMaxKnots);
    stage_lds(P, SCENE, I.hf_cells, I.B, I.hf, sB, sHF);
    __syncthreads();
    // Philox noise drawn here and stored for the tail, or the given dimension-major noise
    const float* ein = I.explicit_eps ? I.eps : nullptr;
    rollout_samples<SCENE, R>(M, P, sB, sHF, sTh, I.mu, I.x, ein, 1, P.K, ein ? nullptr : I.eps, I.costs, nullptr,
                              n_base);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *s_last = (atomicAdd(I.done, 1) == I.ntiles - 1);
    __syncthreads();
    if (*s_last) {
        __threadfence();
        instance_tail<SCENE, R>(I, P, M, sHF, sMup);
        __threadfence();
    }
    __syncthreads();
}

// the queue is drained: the last workgroup to find it empty resets it for the next launch
template <typename R>
__device__ __forceinline__ void batch_exit(const BatchArgs<R>& a)
{
    if (threadIdx.x == 0) {
        if (atomicAdd(a.exited, 1) == (int)gridDim.x - 1) {
            *a.head = 0;
            *a.exited = 0;
            __threadfence();
        }
    }
}

// one persistent kernel per scene: its own queue of that scene's tiles
template <int SCENE, typename R>
__global__ __launch_bounds__(64) void batch_kernel(BatchArgs<R> a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int s_tile, s_last;
    __shared__ float sMup[12 * kMaxKnots];
    const int total = *a.total_tiles;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(a.head, 1);
        __syncthreads();
        // wave-uniform from here on: table rows and models are read with scalar loads
        const int t = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (t >= total) break;
        const int i = __builtin_amdgcn_readfirstlane(a.tile_map[t]);
        const InstDesc& I = a.inst[i];
        DevParams P = I.P;
        P.step = I.step[0];
        const ModelT<R>& M = a.models[__builtin_amdgcn_readfirstlane(I.model)];
        R* sB = reinterpret_cast<R*>(lds_raw);
        R* sTh = sB + P.H * P.nk;
        float* sHF = reinterpret_cast<float*>(sTh + 64 * 3 * kMaxKnots);
        stage_lds(P, SCENE, I.hf_cells, I.B, I.hf, sB, sHF);
        __syncthreads();
        const int n_base = (t - I.tile0) * kTileSamples;
        // Philox noise drawn here and stored for the tail, or the given dimension-major noise
        const float* ein = I.explicit_eps ? I.eps : nullptr;
        rollout_samples<SCENE, R>(M, P, sB, sHF, sTh, I.mu, I.x, ein, 1, P.K, ein ? nullptr : I.eps, I.costs, nullptr,
                                  n_base);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) s_last = (atomicAdd(I.done, 1) == I.ntiles - 1);
        __syncthreads();
        if (s_last) {
            __threadfence();
            instance_tail<SCENE, R>(I, P, M, sHF, sMup);
            __threadfence();
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (atomicAdd(a.exited, 1) == (int)gridDim.x - 1) {
            *a.head = 0;
            *a.exited = 0;
            __threadfence();
        }
    }
}

// one persistent kernel for every scene: a single queue whose entries pack the instance
// row and the tile's index inside its instance (row << 8 | tile); each tile branches to
// its scene's code (uniform over the workgroup).  In FP32 the four scenes' code together
// needs a few registers more than half the file; it is held to two waves per SIMD (the
// per-scene FP32 kernels' occupancy), in FP64 to one.
template <typename R>
__global__ __launch_bounds__(64, sizeof(R) == 4 ? 2 : 1) void batch_kernel_all(BatchArgs<R> a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int s_tile, s_last;
    __shared__ float sMup[12 * kMaxKnots];
    const int total = *a.total_tiles;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(a.head, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (t >= total) break;
        const int packed = __builtin_amdgcn_readfirstlane(a.tile_map[t]);
        const InstDesc& I = a.inst[packed >> 8];
        const ModelT<R>& M = a.models[__builtin_amdgcn_readfirstlane(I.model)];
        const int n_base = (packed & 255) * kTileSamples;
        switch (__builtin_amdgcn_readfirstlane(I.scene)) {
        case 0: batch_tile<0, R>(I, M, n_base, lds_raw, sMup, &s_last); break;
        case 1: batch_tile<1, R>(I, M, n_base, lds_raw, sMup, &s_last); break;
        case 2: batch_tile<2, R>(I, M, n_base, lds_raw, sMup, &s_last); break;
        default: batch_tile<3, R>(I, M, n_base, lds_raw, sMup, &s_last); break;
        }
    }
    batch_exit(a);
}

// ---------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------
hipError_t launch_sample(const DevParams& P, int D, float* eps, uint32_t* raw, hipStream_t st)
{
    const int nb = (D + 3) / 4;
    const long total = (long)P.K * nb;
    const int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(sample_kernel, dim3(blocks), dim3(256), 0, st, P, D, eps, raw);
    return hipGetLastError();
}

template <typename R>
static size_t rollout_lds_bytes(const ModelT<R>& M, const DevParams& P, int threads)
{
    size_t b = sizeof(R) * ((size_t)P.H * P.nk + (size_t)threads * 3 * kMaxKnots);
    if (M.scene == 1) b += sizeof(float) * (size_t)M.hf_nx * M.hf_ny;
    return b;
}

template <typename R>
static hipError_t launch_rollout_t(const ModelT<R>& M, const DevParams& P, const RolloutArgs& a, hipStream_t st)
{
    const int threads = a.samples_per_block * 4;
    const int blocks = (P.K + a.samples_per_block - 1) / a.samples_per_block;
    const size_t lds = rollout_lds_bytes(M, P, threads);
    if (lds > 65536) return hipErrorInvalidValue;
#define MPPI_LAUNCH_ROLLOUT(S)                                                                                    \
    hipLaunchKernelGGL((rollout_kernel<S, R>), dim3(blocks), dim3(threads), lds, st, M, P, a.B, a.hf, a.mu, a.x0,  \
                       a.eps_in, a.eps_sn, a.eps_sd, a.eps_out, a.costs, a.traj)
    switch (M.scene) {
    case 0: MPPI_LAUNCH_ROLLOUT(0); break;
    case 1: MPPI_LAUNCH_ROLLOUT(1); break;
    case 2: MPPI_LAUNCH_ROLLOUT(2); break;
    case 3: MPPI_LAUNCH_ROLLOUT(3); break;
    default: return hipErrorInvalidValue;
    }
#undef MPPI_LAUNCH_ROLLOUT
    return hipGetLastError();
}

hipError_t launch_rollout(const DevModelF& Mf, const DevModelD& Md, int arith, const DevParams& P,
                          const RolloutArgs& a, hipStream_t st)
{
    return arith == 1 ? launch_rollout_t(Mf, P, a, st) : launch_rollout_t(Md, P, a, st);
}

hipError_t launch_update(const DevParams& P, const UpdateArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(update_kernel, dim3(12), dim3(kUpdThreads), 0, st, P, a);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_sim_step_t(const ModelT<R>& M, int n, int nx, const float* x, const float* u, float kp,
                                    float kd, float dt, float* xo, float* tau, const float* hf, hipStream_t st)
{
    const int spb = 16;
    const int blocks = (n + spb - 1) / spb;
    const size_t lds = (M.scene == 1) ? (size_t)M.hf_nx * M.hf_ny * sizeof(float) : 0;
#define MPPI_LAUNCH_SIM(S)                                                                                      \
    hipLaunchKernelGGL((sim_step_kernel<S, R>), dim3(blocks), dim3(4 * spb), lds, st, M, n, nx, x, u, kp, kd, dt, \
                       xo, tau, hf)
    switch (M.scene) {
    case 0: MPPI_LAUNCH_SIM(0); break;
    case 1: MPPI_LAUNCH_SIM(1); break;
    case 2: MPPI_LAUNCH_SIM(2); break;
    case 3: MPPI_LAUNCH_SIM(3); break;
    default: return hipErrorInvalidValue;
    }
#undef MPPI_LAUNCH_SIM
    return hipGetLastError();
}

hipError_t launch_sim_step(const DevModelF& Mf, const DevModelD& Md, int arith, int n, int nx, const float* x,
                           const float* u, float kp, float kd, float dt, float* xo, float* tau, const float* hf,
                           hipStream_t st)
{
    return arith == 1 ? launch_sim_step_t(Mf, n, nx, x, u, kp, kd, dt, xo, tau, hf, st)
                      : launch_sim_step_t(Md, n, nx, x, u, kp, kd, dt, xo, tau, hf, st);
}

template <typename R>
static hipError_t launch_batch_t(int scene, const BatchArgs<R>& a, int grid, size_t lds, hipStream_t st)
{
    switch (scene) {
    case 0: hipLaunchKernelGGL((batch_kernel<0, R>), dim3(grid), dim3(64), lds, st, a); break;
    case 1: hipLaunchKernelGGL((batch_kernel<1, R>), dim3(grid), dim3(64), lds, st, a); break;
    case 2: hipLaunchKernelGGL((batch_kernel<2, R>), dim3(grid), dim3(64), lds, st, a); break;
    case 3: hipLaunchKernelGGL((batch_kernel<3, R>), dim3(grid), dim3(64), lds, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_all(int arith, const void* args, int grid, size_t lds, hipStream_t st)
{
    if (arith == 1)
        hipLaunchKernelGGL(batch_kernel_all<float>, dim3(grid), dim3(64), lds, st,
                           *static_cast<const BatchArgs<float>*>(args));
    else
        hipLaunchKernelGGL(batch_kernel_all<double>, dim3(grid), dim3(64), lds, st,
                           *static_cast<const BatchArgs<double>*>(args));
    return hipGetLastError();
}

hipError_t launch_batch(int arith, int scene, const void* args, int grid, size_t lds, hipStream_t st)
{
    if (arith == 1) return launch_batch_t(scene, *static_cast<const BatchArgs<float>*>(args), grid, lds, st);
    return launch_batch_t(scene, *static_cast<const BatchArgs<double>*>(args), grid, lds, st);
}

}  // namespace mppi
