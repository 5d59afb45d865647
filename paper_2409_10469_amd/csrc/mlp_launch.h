// Host-side launch interface of the proposal-network kernels (BF16 MFMA GEMMs with
// fused epilogues, loss, gradient reduction, Adam, feature and head kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlp {

constexpr int kLayers = 5;
constexpr int kIn = 40, kInPad = 64, kHidden = 512, kOut = 144, kOutPad = 192, kKnots = 6;
constexpr int kGemmBK = 64;  // reduction tile; every K handed to a GEMM is a multiple of it
constexpr int kMaxSplits = 8;  // most batch splits of a weight-gradient product

enum Epilogue {
    EPI_HIDDEN = 0,  // z = acc + b -> Z (fp32, optional), silu(z) -> H (bf16) and H^T (bf16, optional)
    EPI_OUT = 1,     // acc + b -> C (fp32) for rows < m_store, columns < n_store
    EPI_DACT = 2,    // dz = acc * silu'(Zp) -> H (bf16), H^T (bf16); per-M-tile column sums of dz
    EPI_SPLITK = 3   // acc -> C + blockIdx.z * c_split_stride (fp32 partial of a split reduction)
};

// C[m][n] = sum_k A[m][k] B[n][k] over k in [z K, (z+1) K) for split z; A and B bf16,
// row strides lda, ldb (elements).  M, N multiples of the tile; K a multiple of 64.
struct GemmArgs {
    const __bf16* A;
    const __bf16* B;
    int lda, ldb;
    int M, N, K;
    float* C;
    int ldc;
    long c_split_stride;
    const float* bias;
    __bf16* H;
    int ldh;
    __bf16* Ht;
    int ldht;
    const float* Zp;
    int ldz;
    float* colpart;  // [M / BM][N]
    int m_store, n_store;
};

// Tile choice: the largest tile that still gives at least 1024 workgroups (4 per CU).
// One 256-thread workgroup per CU leaves a single wave per SIMD and too few memory
// requests in flight for the epilogue's output stream; at batch 4096 every product here
// takes 64 x 64 tiles (measured: 164 us per training step against 186 us with 128 x 64).
constexpr long kMinBlocks = 1024;
inline bool use_wide(int M, int N, int splits)
{
    return M % 128 == 0 && N % 128 == 0 && (long)(M / 128) * (N / 128) * splits >= kMinBlocks;
}
// the M-tile height used (for the column-sum partial count), or 0 on a shape error
inline int gemm_tile_m(int M, int N, int splits)
{
    if (M <= 0 || N <= 0 || M % 64 || N % 64) return 0;
    if (use_wide(M, N, splits)) return 128;
    if (M % 128 == 0 && (long)(M / 128) * (N / 64) * splits >= kMinBlocks) return 128;
    return 64;
}
hipError_t launch_gemm(int epi, const GemmArgs& g, int splits, hipStream_t st);

// raw features (rows idx[r] of X, stride 40) -> standardised bf16 X0 [Bp x 64] and X0^T [64 x Bp]
struct PrepArgs {
    const float* X;
    const int* idx;
    int B, Bp;
    const float* mean;
    const float* std;
    __bf16* X0;
    __bf16* X0t;
};
hipError_t launch_prep(const PrepArgs& a, hipStream_t st);

// Gaussian NLL of out [Bp x 144] against standardised targets; dz of the last layer
struct LossArgs {
    const float* out;
    const float* Y;
    const int* idx;
    int B, Bp;
    const float* omean;
    const float* ostd;
    __bf16* dZ;     // [Bp x 192]
    __bf16* dZt;    // [192 x Bp]
    float* dbpart;  // [Bp / loss_rows_per_block()][192]
    float* lpart;   // [Bp / loss_rows_per_block()]
};
hipError_t launch_loss(const LossArgs& a, hipStream_t st);
int loss_rows_per_block();  // rows of one loss workgroup (Bp must be a multiple); partial rows = Bp / this

struct LayerGeom {
    int off[kLayers + 1];  // flat parameter offsets (W then b per layer)
    int fi[kLayers], fo[kLayers], fip[kLayers], fop[kLayers];
};

// G = split-K and per-tile partial sums reduced in a fixed order; loss = sum(lpart) * scale
struct ReduceArgs {
    LayerGeom g;
    const float* wpart[kLayers];  // [S][fip][fop]
    const float* bpart[kLayers];  // [T][fop]
    int S[kLayers], T[kLayers];  // S <= kMaxSplits
    float* G;
    const float* lpart;
    int nl;
    float lscale;
    float* loss;
};
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st);

// Adam (update = 1) or shadow refresh only (update = 0); bf16 shadows W^T [fop x fip] and
// W [fip x fop] (layers >= 1) rewritten from the FP32 master weights
struct AdamArgs {
    LayerGeom g;
    float* P;
    float* m;
    float* v;
    const float* G;
    float lr, b1, b2, omb1, omb2, eps, inv_c1, inv_c2;  // omb = 1 - beta, rounded once from double
    __bf16* Wt[kLayers];
    __bf16* Wn[kLayers];
    int update;
};
hipError_t launch_adam(const AdamArgs& a, hipStream_t st);
// the reduction of launch_reduce and the update of launch_adam in one pass (G not stored)
hipError_t launch_reduce_adam(const ReduceArgs& r, const AdamArgs& a, hipStream_t st);

// network output (standardised) -> proposal centre and std for nk knots per joint
struct HeadArgs {
    const float* out;
    const float* omean;
    const float* ostd;
    int nk;
    float R[8][kKnots];  // resampling matrix, nk x 6
    float log_lo, log_hi;
    float* center;
    float* sd;
};
hipError_t launch_head(const HeadArgs& a, hipStream_t st);

// the mean loss from the loss kernel's partials, summed in the order of the parameter
// pass (lane t adds partials t, t + 64, ...; then the 64 lane sums in order), so it equals
// the loss a gradient or training step reports for the same rows
hipError_t launch_loss_sum(const float* lpart, int nl, float lscale, float* loss, hipStream_t st);

// closed-loop records -> training pairs (one workgroup per record)
struct PairsArgs {
    const float* rec;   // n_rec x steps x (37 + 12 nk): state, then the unshifted knots
    const float* oc;    // n_rec x 3: origin x, origin y, commanded forward velocity
    int n_rec, steps, nk;
    float fall_z;       // a row whose base height is not above this ends the record's pairs
    float R[kKnots][8]; // target knot i from record knot k, 6 x nk
    float* feat;        // n_rec x steps x 40
    float* tgt;         // n_rec x steps x 72
    int* count;         // n_rec: pairs of each record
};
hipError_t launch_pairs(const PairsArgs& a, hipStream_t st);

}  // namespace mlp
