// Kernels of the learned sampling proposal: a 40 -> 512 x 4 -> 144 SiLU network with
// BF16 operands and FP32 accumulation on the gfx950 matrix cores.
//
// Every product of the forward and backward passes is written in one form,
// C = A B^T with both operands stored k-contiguous, so one LDS-tiled MFMA kernel serves
// all of them; the producers write the transposed copies the next product needs:
//   forward     Z_l   = H_{l-1} W_l            A = H_{l-1} [B x fi],  B = W_l^T [fo x fi]
//   input grad  dA    = dZ_l W_l^T             A = dZ_l    [B x fo],  B = W_l   [fi x fo]
//   weight grad dW_l  = H_{l-1}^T dZ_l         A = H^T     [fi x B],  B = dZ^T  [fo x B]
// The weight gradient reduces over the batch and is split along it; the split partials
// and the per-tile bias-gradient column sums are reduced in a fixed order, so a training
// step is deterministic.
#include <hip/hip_runtime.h>

#include "mlp_launch.h"

namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BK = kGemmBK;
constexpr int LDK = BK + 8;  // LDS row pitch in bf16: 144 B keeps the 16-byte fragment reads conflict-free

__device__ __forceinline__ float sigm(float z) { return 1.f / (1.f + expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z)
{
    const float s = sigm(z);
    return s * (1.f + z * (1.f - s));
}

// ---------------------------------------------------------------------------------
// GEMM: 256 threads = 4 waves in a 2 x 2 grid, each wave a (BM/2) x (BN/2) block of
// 16 x 16 accumulator tiles fed by v_mfma_f32_16x16x32_bf16.  Operand fragments: lane l
// holds row (l mod 16) and the 8 k-values 8 (l / 16) .. +7 of the 32-wide k step (both
// operands use the same k assignment); the accumulator holds column (l mod 16), rows
// 4 (l / 16) .. +3.  Tiles of A and B pass through LDS, the next tile's global loads
// overlapping the current tile's products.
// ---------------------------------------------------------------------------------
template <int BM, int BN, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g)
{
    constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
    constexpr int CA = BM * BK / (8 * 256), CB = BN * BK / (8 * 256);
    __shared__ __align__(16) __bf16 sA[BM * LDK];
    __shared__ __align__(16) __bf16 sB[BN * LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const size_t kb = (size_t)blockIdx.z * g.K;
    const __bf16* A = g.A + (size_t)m0 * g.lda + kb;
    const __bf16* B = g.B + (size_t)n0 * g.ldb + kb;

    u32x4 ra[CA], rb[CB];
#define MLP_GLOAD(k0)                                                                                      \
    do {                                                                                                   \
        _Pragma("unroll") for (int c = 0; c < CA; ++c)                                                     \
        {                                                                                                  \
            const int idx = tid + 256 * c, row = idx >> 3, col = (idx & 7) * 8;                            \
            ra[c] = *reinterpret_cast<const u32x4*>(A + (size_t)row * g.lda + (k0) + col);                 \
        }                                                                                                  \
        _Pragma("unroll") for (int c = 0; c < CB; ++c)                                                     \
        {                                                                                                  \
            const int idx = tid + 256 * c, row = idx >> 3, col = (idx & 7) * 8;                            \
            rb[c] = *reinterpret_cast<const u32x4*>(B + (size_t)row * g.ldb + (k0) + col);                 \
        }                                                                                                  \
    } while (0)

    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    MLP_GLOAD(0);
    for (int k0 = 0; k0 < g.K; k0 += BK) {
        __syncthreads();
#pragma unroll
        for (int c = 0; c < CA; ++c) {
            const int idx = tid + 256 * c, row = idx >> 3, col = (idx & 7) * 8;
            *reinterpret_cast<u32x4*>(sA + row * LDK + col) = ra[c];
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int idx = tid + 256 * c, row = idx >> 3, col = (idx & 7) * 8;
            *reinterpret_cast<u32x4*>(sB + row * LDK + col) = rb[c];
        }
        __syncthreads();
        if (k0 + BK < g.K) MLP_GLOAD(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 32) {
            bf16x8 a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                a[i] = *reinterpret_cast<const bf16x8*>(sA + (wm * WM + i * 16 + (lane & 15)) * LDK + kk +
                                                        (lane >> 4) * 8);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(sB + (wn * WN + j * 16 + (lane & 15)) * LDK + kk +
                                                        (lane >> 4) * 8);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }

#undef MLP_GLOAD

    // ---- epilogues -------------------------------------------------------------
    if constexpr (EPI == EPI_SPLITK) {
        float* C = g.C + (size_t)blockIdx.z * g.c_split_stride;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int n = n0 + wn * WN + j * 16 + (lane & 15);
                const int mb = m0 + wm * WM + i * 16 + (lane >> 4) * 4;
#pragma unroll
                for (int r = 0; r < 4; ++r) C[(size_t)(mb + r) * g.ldc + n] = acc[i][j][r];
            }
    } else if constexpr (EPI == EPI_OUT) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int n = n0 + wn * WN + j * 16 + (lane & 15);
                const int mb = m0 + wm * WM + i * 16 + (lane >> 4) * 4;
                if (n < g.n_store) {
                    const float bv = g.bias[n];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (mb + r < g.m_store) g.C[(size_t)(mb + r) * g.ldc + n] = acc[i][j][r] + bv;
                }
            }
    } else if constexpr (EPI == EPI_HIDDEN) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int n = n0 + wn * WN + j * 16 + (lane & 15);
                const int mb = m0 + wm * WM + i * 16 + (lane >> 4) * 4;
                const float bv = g.bias[n];
                bf16x4 hv;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float z = acc[i][j][r] + bv;
                    if (g.C) g.C[(size_t)(mb + r) * g.ldc + n] = z;
                    hv[r] = (__bf16)silu(z);
                    g.H[(size_t)(mb + r) * g.ldh + n] = hv[r];
                }
                if (g.Ht) *reinterpret_cast<bf16x4*>(g.Ht + (size_t)n * g.ldht + mb) = hv;
            }
    } else {  // EPI_DACT
        float cs[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) cs[j] = 0.f;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int n = n0 + wn * WN + j * 16 + (lane & 15);
                const int mb = m0 + wm * WM + i * 16 + (lane >> 4) * 4;
                bf16x4 hv;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float dz = acc[i][j][r] * dsilu(g.Zp[(size_t)(mb + r) * g.ldz + n]);
                    hv[r] = (__bf16)dz;
                    g.H[(size_t)(mb + r) * g.ldh + n] = hv[r];
                    cs[j] += dz;
                }
                *reinterpret_cast<bf16x4*>(g.Ht + (size_t)n * g.ldht + mb) = hv;
            }
        // column sums: the four row groups of the wave, then the two waves sharing columns
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            cs[j] += __shfl_xor(cs[j], 16, 64);
            cs[j] += __shfl_xor(cs[j], 32, 64);
        }
        __syncthreads();  // all waves are done reading sA
        float* red = reinterpret_cast<float*>(sA);  // [2][BN]
        if (lane < 16)
#pragma unroll
            for (int j = 0; j < TN; ++j) red[wm * BN + wn * WN + j * 16 + lane] = cs[j];
        __syncthreads();
        for (int c = tid; c < BN; c += 256) g.colpart[(size_t)blockIdx.y * g.N + n0 + c] = red[c] + red[BN + c];
    }
}

int gemm_tile_m(int M, int N, int splits)
{
    if (M <= 0 || N <= 0 || M % 64 || N % 64) return 0;
    const long big = (long)(M / 128) * (N / 128) * splits;
    if (M % 128 == 0 && N % 128 == 0 && big >= 240) return 128;
    const long mid = (long)(M / 128) * (N / 64) * splits;
    if (M % 128 == 0 && mid >= 240) return 128;
    return 64;
}

template <int BM, int BN>
static void launch_tile(int epi, const GemmArgs& g, int splits, hipStream_t st)
{
    const dim3 grid(g.N / BN, g.M / BM, splits);
    switch (epi) {
    case EPI_HIDDEN: hipLaunchKernelGGL((gemm_kernel<BM, BN, EPI_HIDDEN>), grid, dim3(256), 0, st, g); break;
    case EPI_OUT: hipLaunchKernelGGL((gemm_kernel<BM, BN, EPI_OUT>), grid, dim3(256), 0, st, g); break;
    case EPI_DACT: hipLaunchKernelGGL((gemm_kernel<BM, BN, EPI_DACT>), grid, dim3(256), 0, st, g); break;
    default: hipLaunchKernelGGL((gemm_kernel<BM, BN, EPI_SPLITK>), grid, dim3(256), 0, st, g); break;
    }
}

hipError_t launch_gemm(int epi, const GemmArgs& g, int splits, hipStream_t st)
{
    const int bm = gemm_tile_m(g.M, g.N, splits);
    if (!bm || g.K <= 0 || g.K % BK || splits < 1) return hipErrorInvalidValue;
    const bool wide = bm == 128 && g.N % 128 == 0 && (long)(g.M / 128) * (g.N / 128) * splits >= 240;
    if (bm == 128 && wide) launch_tile<128, 128>(epi, g, splits, st);
    else if (bm == 128) launch_tile<128, 64>(epi, g, splits, st);
    else launch_tile<64, 64>(epi, g, splits, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void prep_kernel(PrepArgs a)
{
    const int gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= a.Bp * kInPad) return;
    const int r = gid / kInPad, c = gid - r * kInPad;
    float v = 0.f;
    if (r < a.B && c < kIn) {
        const int row = a.idx ? a.idx[r] : r;
        v = (a.X[(size_t)row * kIn + c] - a.mean[c]) / a.std[c];
    }
    const __bf16 b = (__bf16)v;
    a.X0[(size_t)r * kInPad + c] = b;
    a.X0t[(size_t)c * a.Bp + r] = b;
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t st)
{
    const int n = a.Bp * kInPad;
    hipLaunchKernelGGL(prep_kernel, dim3((n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

// One block per kLossRows rows.  Phase 1: every (row, output pair d) element is
// independent; thread t takes elements t, t + 256, ... (9 each), writes the row-major dz
// and keeps both errors in an LDS tile.  Phase 2: the tile gives the transposed dz rows
// (16-byte stores), the per-column sums of the block (fixed order) and the loss sum.
constexpr int kLossRows = 32;
__global__ __launch_bounds__(256) void loss_kernel(LossArgs a)
{
    __shared__ float sD[kOut][kLossRows + 1];
    __shared__ float red[256];
    const int t = threadIdx.x, r0 = blockIdx.x * kLossRows;
    const float inv = 1.f / ((float)a.B * 72.f);
    float lsum = 0.f;
#pragma unroll
    for (int j = 0; j < kLossRows * 72 / 256; ++j) {
        const int e = t + 256 * j, rr = e / 72, d = e - rr * 72, r = r0 + rr;
        float dm = 0.f, dsv = 0.f;
        if (r < a.B) {
            const int row = a.idx ? a.idx[r] : r;
            const float y = (a.Y[(size_t)row * 72 + d] - a.omean[d]) / a.ostd[d];
            const float m = a.out[(size_t)r * kOut + d], s = a.out[(size_t)r * kOut + 72 + d];
            const float err = y - m, w = expf(-2.f * s), q = err * err * w;
            lsum += 0.5f * q + s;
            dm = -err * w * inv;
            dsv = (1.f - q) * inv;
        }
        sD[d][rr] = dm;
        sD[72 + d][rr] = dsv;
        a.dZ[(size_t)r * kOutPad + d] = (__bf16)dm;
        a.dZ[(size_t)r * kOutPad + 72 + d] = (__bf16)dsv;
    }
    // zero padding columns of the row-major copy: 48 per row
    for (int e = t; e < kLossRows * (kOutPad - kOut); e += 256) {
        const int rr = e / (kOutPad - kOut), c = kOut + (e - rr * (kOutPad - kOut));
        a.dZ[(size_t)(r0 + rr) * kOutPad + c] = (__bf16)0.f;
    }
    red[t] = lsum;
    __syncthreads();
    // transposed rows: kOutPad columns x kLossRows rows in 8-element chunks
    for (int e = t; e < kOutPad * (kLossRows / 8); e += 256) {
        const int c = e / (kLossRows / 8), k8 = (e - c * (kLossRows / 8)) * 8;
        bf16x8 v;
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = (__bf16)(c < kOut ? sD[c][k8 + u] : 0.f);
        *reinterpret_cast<bf16x8*>(a.dZt + (size_t)c * a.Bp + r0 + k8) = v;
    }
    if (t < kOutPad) {
        float cs = 0.f;
        if (t < kOut)
            for (int rr = 0; rr < kLossRows; ++rr) cs += sD[t][rr];
        a.dbpart[(size_t)blockIdx.x * kOutPad + t] = cs;
    }
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) red[t] += red[t + st];
        __syncthreads();
    }
    if (t == 0) a.lpart[blockIdx.x] = red[0];
}

hipError_t launch_loss(const LossArgs& a, hipStream_t st)
{
    if (a.Bp % kLossRows) return hipErrorInvalidValue;
    hipLaunchKernelGGL(loss_kernel, dim3(a.Bp / kLossRows), dim3(256), 0, st, a);
    return hipGetLastError();
}

int loss_rows_per_block() { return kLossRows; }

// ---------------------------------------------------------------------------------
__device__ __forceinline__ int find_layer(const LayerGeom& g, int p)
{
    int l = 0;
#pragma unroll
    for (int k = 1; k < kLayers; ++k)
        if (p >= g.off[k]) l = k;
    return l;
}

__device__ __forceinline__ float reduced_grad(const ReduceArgs& a, int p);

__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p == 0 && a.loss) {
        float s = 0.f;
        for (int i = 0; i < a.nl; ++i) s += a.lpart[i];
        a.loss[0] = s * a.lscale;
    }
    if (p >= a.g.off[kLayers]) return;
    a.G[p] = reduced_grad(a, p);
}

// gradient of parameter p from the fixed-order partial sums
__device__ __forceinline__ float reduced_grad(const ReduceArgs& a, int p)
{
    const int l = find_layer(a.g, p);
    const int q = p - a.g.off[l], fi = a.g.fi[l], fo = a.g.fo[l], fop = a.g.fop[l];
    float s = 0.f;
    if (q < fi * fo) {
        const int i = q / fo, o = q - i * fo;
        const size_t stride = (size_t)a.g.fip[l] * fop;
        const float* w = a.wpart[l] + (size_t)i * fop + o;
        for (int k = 0; k < a.S[l]; ++k) s += w[k * stride];
    } else {
        const int o = q - fi * fo;
        const float* b = a.bpart[l] + o;
        for (int k = 0; k < a.T[l]; ++k) s += b[(size_t)k * fop];
    }
    return s;
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st)
{
    const int n = a.g.off[kLayers];
    hipLaunchKernelGGL(reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Adam (Kingma and Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// p <- p - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps); then the bf16 shadows
__device__ __forceinline__ void adam_update(const AdamArgs& a, int p, float gr)
{
    float w = a.P[p];
    if (a.update) {
        const float m = a.b1 * a.m[p] + a.omb1 * gr;
        const float v = a.b2 * a.v[p] + a.omb2 * gr * gr;
        a.m[p] = m;
        a.v[p] = v;
        w -= a.lr * (m * a.inv_c1) / (sqrtf(v * a.inv_c2) + a.eps);
        a.P[p] = w;
    }
    const int l = find_layer(a.g, p);
    const int q = p - a.g.off[l], fo = a.g.fo[l];
    if (q < a.g.fi[l] * fo) {
        const int i = q / fo, o = q - i * fo;
        a.Wt[l][(size_t)o * a.g.fip[l] + i] = (__bf16)w;
        if (a.Wn[l]) a.Wn[l][(size_t)i * a.g.fop[l] + o] = (__bf16)w;
    }
}

__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= a.g.off[kLayers]) return;
    adam_update(a, p, a.update ? a.G[p] : 0.f);
}

// training step tail: fixed-order gradient reduction and Adam in one pass (the gradient
// is not stored)
__global__ __launch_bounds__(256) void reduce_adam_kernel(ReduceArgs r, AdamArgs a)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p == 0 && r.loss) {
        float s = 0.f;
        for (int i = 0; i < r.nl; ++i) s += r.lpart[i];
        r.loss[0] = s * r.lscale;
    }
    if (p >= r.g.off[kLayers]) return;
    adam_update(a, p, reduced_grad(r, p));
}

hipError_t launch_reduce_adam(const ReduceArgs& r, const AdamArgs& a, hipStream_t st)
{
    const int n = r.g.off[kLayers];
    hipLaunchKernelGGL(reduce_adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, r, a);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t st)
{
    const int n = a.g.off[kLayers];
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
__global__ void head_kernel(HeadArgs a)
{
    const int t = threadIdx.x;
    if (t >= 12 * a.nk) return;
    const int j = t / a.nk, i = t - j * a.nk;
    float m = 0.f, s = 0.f;
#pragma unroll
    for (int k = 0; k < kKnots; ++k) {
        const int d = j * kKnots + k;
        const float sd = a.ostd[d];
        m += a.R[i][k] * (a.out[d] * sd + a.omean[d]);
        s += a.R[i][k] * (a.out[72 + d] + logf(sd));
    }
    s = fminf(fmaxf(s, a.log_lo), a.log_hi);
    a.center[t] = m;
    a.sd[t] = expf(s);
}

hipError_t launch_head(const HeadArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(head_kernel, dim3(1), dim3(128), 0, st, a);
    return hipGetLastError();
}

}  // namespace mlp
