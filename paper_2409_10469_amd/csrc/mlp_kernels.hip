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
constexpr int kPF = 3;       // k-tiles of global loads in flight

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
// 4 (l / 16) .. +3.  Tiles of A and B pass through LDS; the global loads of the next kPF
// k-tiles are in flight (in registers) while the current tile's products run.
// ---------------------------------------------------------------------------------
template <int BM, int BN, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g)
{
    constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
    constexpr int CA = BM * BK / (8 * 256), CB = BN * BK / (8 * 256);
    // LDS: the operand tiles during the k loop, then the fp32 output tile for the epilogue
    constexpr int LDC = BN + 4;  // output tile row pitch in floats (16-byte aligned rows)
    constexpr int kAB = (BM + BN) * LDK * 2, kC = BM * LDC * 4;
    __shared__ __align__(16) unsigned char smem[kAB > kC ? kAB : kC];
    __shared__ float red[4][BN];
    __bf16* sA = reinterpret_cast<__bf16*>(smem);
    __bf16* sB = sA + BM * LDK;
    float* sC = reinterpret_cast<float*>(smem);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    // M-tiles vary fastest: workgroups go round-robin to the 8 XCDs, so the N-tiles of one
    // row panel of A share an XCD and its L2 (A is the large operand; B is re-read per XCD)
    const int mt = blockIdx.x, m0 = mt * BM, n0 = blockIdx.y * BN;
    const size_t kb = (size_t)blockIdx.z * g.K;
    const __bf16* A = g.A + (size_t)m0 * g.lda + kb;
    const __bf16* B = g.B + (size_t)n0 * g.ldb + kb;

    // register-staged prefetch kPF k-tiles deep: stage s of the ring holds k-tile
    // (k / BK) with (k / BK) mod kPF = s; each k-tile is stored to LDS, consumed, and its
    // stage refilled with the k-tile kPF ahead
    u32x4 ra[kPF][CA], rb[kPF][CB];
#define MLP_GLOAD(s, k0)                                                                                   \
    do {                                                                                                   \
        _Pragma("unroll") for (int c = 0; c < CA; ++c)                                                     \
        {                                                                                                  \
            const int idx = tid + 256 * c, row = idx >> 3, col = (idx & 7) * 8;                            \
            ra[s][c] = *reinterpret_cast<const u32x4*>(A + (size_t)row * g.lda + (k0) + col);              \
        }                                                                                                  \
        _Pragma("unroll") for (int c = 0; c < CB; ++c)                                                     \
        {                                                                                                  \
            const int idx = tid + 256 * c, row = idx >> 3, col = (idx & 7) * 8;                            \
            rb[s][c] = *reinterpret_cast<const u32x4*>(B + (size_t)row * g.ldb + (k0) + col);              \
        }                                                                                                  \
    } while (0)

    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
    for (int s = 0; s < kPF; ++s)
        if (s * BK < g.K) MLP_GLOAD(s, s * BK);
    for (int kt = 0; kt < g.K; kt += kPF * BK) {
#pragma unroll
        for (int s = 0; s < kPF; ++s) {
            const int k0 = kt + s * BK;
            if (k0 >= g.K) break;
            __syncthreads();
#pragma unroll
            for (int c = 0; c < CA; ++c) {
                const int idx = tid + 256 * c, row = idx >> 3, col = (idx & 7) * 8;
                *reinterpret_cast<u32x4*>(sA + row * LDK + col) = ra[s][c];
            }
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int idx = tid + 256 * c, row = idx >> 3, col = (idx & 7) * 8;
                *reinterpret_cast<u32x4*>(sB + row * LDK + col) = rb[s][c];
            }
            __syncthreads();
            if (k0 + kPF * BK < g.K) MLP_GLOAD(s, k0 + kPF * BK);
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
    }

#undef MLP_GLOAD

    // ---- epilogues: the accumulators (plus the bias where one is added) go to the LDS
    // tile sC [BM x LDC]; every output then leaves in 16-byte pieces of its rows
    __syncthreads();  // all waves are done with sA / sB
    {
        float bv[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int n = n0 + wn * WN + j * 16 + (lane & 15);
            bv[j] = 0.f;
            if constexpr (EPI == EPI_HIDDEN) bv[j] = g.bias[n];
            if constexpr (EPI == EPI_OUT) bv[j] = n < g.n_store ? g.bias[n] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int nl = wn * WN + j * 16 + (lane & 15);
                const int ml = wm * WM + i * 16 + (lane >> 4) * 4;
#pragma unroll
                for (int r = 0; r < 4; ++r) sC[(ml + r) * LDC + nl] = acc[i][j][r] + bv[j];
            }
    }
    __syncthreads();
    constexpr int RC = BN / 8, MC = BM / 8;  // 8-wide pieces per tile row / per tile column
    if constexpr (EPI == EPI_SPLITK) {
        float* C = g.C + (size_t)blockIdx.z * g.c_split_stride;
#pragma unroll
        for (int e = tid; e < BM * RC; e += 256) {
            const int row = e / RC, c8 = (e - row * RC) * 8;
            float* dst = C + (size_t)(m0 + row) * g.ldc + n0 + c8;
            *reinterpret_cast<f32x4*>(dst) = *reinterpret_cast<const f32x4*>(sC + row * LDC + c8);
            *reinterpret_cast<f32x4*>(dst + 4) = *reinterpret_cast<const f32x4*>(sC + row * LDC + c8 + 4);
        }
    } else if constexpr (EPI == EPI_OUT) {  // caller's buffer: element stores, rows in order
        for (int e = tid; e < BM * BN; e += 256) {
            const int row = e / BN, col = e - row * BN;
            if (m0 + row < g.m_store && n0 + col < g.n_store)
                g.C[(size_t)(m0 + row) * g.ldc + n0 + col] = sC[row * LDC + col];
        }
    } else if constexpr (EPI == EPI_HIDDEN) {
#pragma unroll
        for (int e = tid; e < BM * RC; e += 256) {
            const int row = e / RC, c8 = (e - row * RC) * 8;
            float* zt = sC + row * LDC + c8;
            const f32x4 z0 = *reinterpret_cast<const f32x4*>(zt), z1 = *reinterpret_cast<const f32x4*>(zt + 4);
            if (g.C) {
                float* dst = g.C + (size_t)(m0 + row) * g.ldc + n0 + c8;
                *reinterpret_cast<f32x4*>(dst) = z0;
                *reinterpret_cast<f32x4*>(dst + 4) = z1;
            }
            bf16x8 hv;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                hv[u] = (__bf16)silu(z0[u]);
                hv[4 + u] = (__bf16)silu(z1[u]);
            }
            *reinterpret_cast<bf16x8*>(g.H + (size_t)(m0 + row) * g.ldh + n0 + c8) = hv;
            if (g.Ht) {  // keep the rounded activations for the transposed copy
#pragma unroll
                for (int u = 0; u < 8; ++u) zt[u] = (float)hv[u];
            }
        }
        if (g.Ht) {
            __syncthreads();
#pragma unroll
            for (int e = tid; e < BN * MC; e += 256) {
                const int col = e / MC, m8 = (e - col * MC) * 8;
                bf16x8 v;
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = (__bf16)sC[(m8 + u) * LDC + col];
                *reinterpret_cast<bf16x8*>(g.Ht + (size_t)(n0 + col) * g.ldht + m0 + m8) = v;
            }
        }
    } else {  // EPI_DACT: dz = (dL/dh) * silu'(z) with the stored pre-activation z
#pragma unroll
        for (int e = tid; e < BM * RC; e += 256) {
            const int row = e / RC, c8 = (e - row * RC) * 8;
            float* at = sC + row * LDC + c8;
            const float* zp = g.Zp + (size_t)(m0 + row) * g.ldz + n0 + c8;
            const f32x4 z0 = *reinterpret_cast<const f32x4*>(zp), z1 = *reinterpret_cast<const f32x4*>(zp + 4);
            bf16x8 hv;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float dz = at[u] * dsilu(u < 4 ? z0[u] : z1[u - 4]);
                at[u] = dz;
                hv[u] = (__bf16)dz;
            }
            *reinterpret_cast<bf16x8*>(g.H + (size_t)(m0 + row) * g.ldh + n0 + c8) = hv;
        }
        __syncthreads();
#pragma unroll
        for (int e = tid; e < BN * MC; e += 256) {
            const int col = e / MC, m8 = (e - col * MC) * 8;
            bf16x8 v;
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = (__bf16)sC[(m8 + u) * LDC + col];
            *reinterpret_cast<bf16x8*>(g.Ht + (size_t)(n0 + col) * g.ldht + m0 + m8) = v;
        }
        // column sums of dz over the tile's rows: four quarters in row order, then in order
        for (int e = tid; e < 4 * BN; e += 256) {
            const int q = e / BN, col = e - q * BN;
            float cs = 0.f;
            for (int row = q * (BM / 4); row < (q + 1) * (BM / 4); ++row) cs += sC[row * LDC + col];
            red[q][col] = cs;
        }
        __syncthreads();
        for (int c = tid; c < BN; c += 256)
            g.colpart[(size_t)mt * g.N + n0 + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    }
}

template <int BM, int BN>
static void launch_tile(int epi, const GemmArgs& g, int splits, hipStream_t st)
{
    const dim3 grid(g.M / BM, g.N / BN, splits);
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
    if (bm == 128 && use_wide(g.M, g.N, splits)) launch_tile<128, 128>(epi, g, splits, st);
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
// Parameter pass: the fixed-order gradient reduction, Adam, and the BF16 shadows, in one
// kernel with three modes over the same work split.  Every layer's fan-out is a multiple
// of 4 and its parameter offset too, so threads own groups of 4 consecutive columns and
// move them as 16-byte vectors.
//   Weight tiles, kTileI x kTileO of one layer's W (rows i, columns o): thread t owns
//   columns o0 + 4 (t mod 16) .. +3 of rows i0 + t/16 and i0 + t/16 + 16.  The split-K
//   partials, P, m, v and the row-major shadow W are accessed along o; the transposed
//   shadow W^T goes through an LDS tile and leaves as 16-byte pieces of its rows.
//   Bias blocks, 64 columns of one layer's b: 16 row groups sum contiguous slices of the
//   per-tile column partials, then the 16 sums are added in a fixed order.
// The reduction order is the same in every mode, so the fused step equals reduce + Adam
// bit for bit; the first bias block also sums the loss partials.
// ---------------------------------------------------------------------------------
constexpr int kTileI = 32, kTileO = 64;
enum { PASS_REDUCE = 0, PASS_ADAM = 1, PASS_REDUCE_ADAM = 2 };

__device__ __forceinline__ int weight_tiles(const LayerGeom& g, int l)
{
    return ((g.fi[l] + kTileI - 1) / kTileI) * ((g.fo[l] + kTileO - 1) / kTileO);
}

static int pass_blocks(const LayerGeom& g)
{
    int n = 0;
    for (int l = 0; l < kLayers; ++l)
        n += ((g.fi[l] + kTileI - 1) / kTileI) * ((g.fo[l] + kTileO - 1) / kTileO) + (g.fo[l] + 63) / 64;
    return n;
}

// Adam (Kingma and Ba) on 4 consecutive parameters from p (16-byte aligned):
// m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2, p <- p - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps);
// returns the (new) weights
__device__ __forceinline__ f32x4 adam4(const AdamArgs& a, int p, f32x4 gr)
{
    f32x4 w = *reinterpret_cast<const f32x4*>(a.P + p);
    if (a.update) {
        f32x4 m = *reinterpret_cast<const f32x4*>(a.m + p), v = *reinterpret_cast<const f32x4*>(a.v + p);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            m[u] = a.b1 * m[u] + a.omb1 * gr[u];
            v[u] = a.b2 * v[u] + a.omb2 * gr[u] * gr[u];
            w[u] -= a.lr * (m[u] * a.inv_c1) / (sqrtf(v[u] * a.inv_c2) + a.eps);
        }
        *reinterpret_cast<f32x4*>(a.m + p) = m;
        *reinterpret_cast<f32x4*>(a.v + p) = v;
        *reinterpret_cast<f32x4*>(a.P + p) = w;
    }
    return w;
}

template <int MODE>
__global__ __launch_bounds__(256) void param_pass_kernel(ReduceArgs r, AdamArgs a)
{
    __shared__ __align__(16) __bf16 sT[kTileO][kTileI + 8];
    __shared__ __align__(16) float sS[16][64];
    const LayerGeom& g = (MODE == PASS_ADAM) ? a.g : r.g;
    const int t = threadIdx.x, oq = t & 15, rg = t >> 4;
    int rem = blockIdx.x, l = 0;
    while (l < kLayers && rem >= weight_tiles(g, l)) rem -= weight_tiles(g, l++);
    if (l < kLayers) {  // ---- weight tile
        const int fi = g.fi[l], fo = g.fo[l], fip = g.fip[l], fop = g.fop[l];
        const int nto = (fo + kTileO - 1) / kTileO;
        const int i0 = (rem / nto) * kTileI, o0 = (rem % nto) * kTileO, o = o0 + 4 * oq;
        const bool ocol = o < fo;  // all four columns (fo is a multiple of 4)
        f32x4 gr[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
        if constexpr (MODE != PASS_ADAM) {
            // all partial loads issued together: rows and columns of the tile stay inside
            // the fip x fop planes, and planes past the last split re-read the last one
            const int S = r.S[l];
            const size_t stride = (size_t)fip * fop;
            f32x4 v[2][kMaxSplits];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float* wp = r.wpart[l] + (size_t)(i0 + rg + 16 * h) * fop + o;
#pragma unroll
                for (int k = 0; k < kMaxSplits; ++k)
                    v[h][k] = *reinterpret_cast<const f32x4*>(wp + (size_t)min(k, S - 1) * stride);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int k = 0; k < kMaxSplits; ++k)
                    if (k < S) gr[h] += v[h][k];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int il = rg + 16 * h, i = i0 + il;
            f32x4 w = f32x4{0.f, 0.f, 0.f, 0.f};
            if (ocol && i < fi) {
                const int p = g.off[l] + i * fo + o;
                if constexpr (MODE == PASS_REDUCE) {
                    *reinterpret_cast<f32x4*>(r.G + p) = gr[h];
                } else {
                    if constexpr (MODE == PASS_ADAM)
                        gr[h] = a.update ? *reinterpret_cast<const f32x4*>(a.G + p) : f32x4{0.f, 0.f, 0.f, 0.f};
                    w = adam4(a, p, gr[h]);
                    if (a.Wn[l]) {
                        bf16x4 wb;
#pragma unroll
                        for (int u = 0; u < 4; ++u) wb[u] = (__bf16)w[u];
                        *reinterpret_cast<bf16x4*>(a.Wn[l] + (size_t)i * fop + o) = wb;
                    }
                }
            }
            if constexpr (MODE != PASS_REDUCE) {
#pragma unroll
                for (int u = 0; u < 4; ++u) sT[4 * oq + u][il] = (__bf16)w[u];
            }
        }
        if constexpr (MODE != PASS_REDUCE) {
            __syncthreads();
            const int row = t >> 2, c = t & 3;  // 64 rows of W^T, 4 pieces of 8 each
            *reinterpret_cast<bf16x8*>(a.Wt[l] + (size_t)(o0 + row) * fip + i0 + 8 * c) =
                *reinterpret_cast<const bf16x8*>(&sT[row][8 * c]);
        }
        return;
    }
    // ---- bias block
    int lb = 0;
    while (lb < kLayers && rem >= (g.fo[lb] + 63) / 64) rem -= (g.fo[lb++] + 63) / 64;
    const int fi = g.fi[lb], fo = g.fo[lb], fop = g.fop[lb];
    const int o = rem * 64 + 4 * oq;
    const bool ocol = o < fo;
    if constexpr (MODE != PASS_ADAM) {
        const int T = r.T[lb], q = (T + 15) / 16, k0 = rg * q, k1 = min(T, k0 + q);
        f32x4 s = f32x4{0.f, 0.f, 0.f, 0.f};
        if (ocol)
#pragma unroll 8
            for (int k = k0; k < k1; ++k) s += *reinterpret_cast<const f32x4*>(r.bpart[lb] + (size_t)k * fop + o);
        *reinterpret_cast<f32x4*>(&sS[rg][4 * oq]) = s;
        __syncthreads();
    }
    if (t < 16 && ocol) {
        const int p = g.off[lb] + fi * fo + o;
        f32x4 gr = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (MODE != PASS_ADAM) {
            gr = *reinterpret_cast<const f32x4*>(&sS[0][4 * oq]);
#pragma unroll
            for (int k = 1; k < 16; ++k) gr += *reinterpret_cast<const f32x4*>(&sS[k][4 * oq]);
        }
        if constexpr (MODE == PASS_REDUCE) {
            *reinterpret_cast<f32x4*>(r.G + p) = gr;
        } else {
            if constexpr (MODE == PASS_ADAM)
                gr = a.update ? *reinterpret_cast<const f32x4*>(a.G + p) : f32x4{0.f, 0.f, 0.f, 0.f};
            adam4(a, p, gr);
        }
    }
    if constexpr (MODE != PASS_ADAM) {
        if (lb == 0 && rem == 0 && r.loss) {  // loss: lane sums, then the lanes in order
            __syncthreads();
            float* sl = &sS[0][0];
            if (t < 64) {
                float s = 0.f;
                for (int k = t; k < r.nl; k += 64) s += r.lpart[k];
                sl[t] = s;
            }
            __syncthreads();
            if (t == 0) {
                float s = 0.f;
                for (int k = 0; k < 64; ++k) s += sl[k];
                r.loss[0] = s * r.lscale;
            }
        }
    }
}

template <int MODE>
static hipError_t launch_pass(const ReduceArgs& r, const AdamArgs& a, hipStream_t st)
{
    const LayerGeom& g = MODE == PASS_ADAM ? a.g : r.g;
    hipLaunchKernelGGL(param_pass_kernel<MODE>, dim3(pass_blocks(g)), dim3(256), 0, st, r, a);
    return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& r, hipStream_t st) { return launch_pass<PASS_REDUCE>(r, AdamArgs{}, st); }

hipError_t launch_reduce_adam(const ReduceArgs& r, const AdamArgs& a, hipStream_t st)
{
    return launch_pass<PASS_REDUCE_ADAM>(r, a, st);
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t st) { return launch_pass<PASS_ADAM>(ReduceArgs{}, a, st); }

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

// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void loss_sum_kernel(const float* __restrict__ lpart, int nl, float lscale,
                                                      float* __restrict__ loss)
{
    __shared__ float sl[64];
    const int t = threadIdx.x;
    float s = 0.f;
    for (int k = t; k < nl; k += 64) s += lpart[k];
    sl[t] = s;
    __syncthreads();
    if (t == 0) {
        float tot = 0.f;
        for (int k = 0; k < 64; ++k) tot += sl[k];
        loss[0] = tot * lscale;
    }
}

hipError_t launch_loss_sum(const float* lpart, int nl, float lscale, float* loss, hipStream_t st)
{
    hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(64), 0, st, lpart, nl, lscale, loss);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Training pairs of one closed-loop record per workgroup.  A row is usable while every
// value of it is finite and the base is above the fall height: the first row that is not
// ends the record (the smallest such index, found with an LDS minimum).  Rows before it
// give the features -- the state with the base x, y taken relative to the origin, then the
// command (v, 0, 0) -- and the targets, each joint's knots resampled to 6 with R.
__global__ __launch_bounds__(256) void pairs_kernel(PairsArgs a)
{
    __shared__ int first_bad;
    const int t = threadIdx.x, r = blockIdx.x;
    const int W = 37 + 12 * a.nk;
    const float* rec = a.rec + (size_t)r * a.steps * W;
    if (t == 0) first_bad = a.steps;
    __syncthreads();
    for (int k = t; k < a.steps; k += 256) {
        const float* row = rec + (size_t)k * W;
        bool ok = row[2] > a.fall_z;  // false for a NaN height too
        for (int c = 0; c < W; ++c) ok = ok && isfinite(row[c]);
        if (!ok) atomicMin(&first_bad, k);
    }
    __syncthreads();
    const int n = first_bad;
    if (t == 0) a.count[r] = n;
    const float ox = a.oc[3 * r], oy = a.oc[3 * r + 1], v = a.oc[3 * r + 2];
    float* feat = a.feat + (size_t)r * a.steps * 40;
    for (int e = t; e < n * 40; e += 256) {
        const int k = e / 40, c = e - k * 40;
        float x = 0.f;
        if (c < 37) x = rec[(size_t)k * W + c] - (c == 0 ? ox : c == 1 ? oy : 0.f);
        else if (c == 37) x = v;
        feat[e] = x;
    }
    float* tgt = a.tgt + (size_t)r * a.steps * 72;
    for (int e = t; e < n * 72; e += 256) {
        const int k = e / 72, d = e - k * 72, j = d / kKnots, i = d - j * kKnots;
        const float* kn = rec + (size_t)k * W + 37 + j * a.nk;
        float y = 0.f;
        for (int q = 0; q < a.nk; ++q) y += a.R[i][q] * kn[q];
        tgt[e] = y;
    }
}

hipError_t launch_pairs(const PairsArgs& a, hipStream_t st)
{
    if (a.n_rec < 1 || a.steps < 1 || a.nk < 2 || a.nk > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pairs_kernel, dim3(a.n_rec), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace mlp
