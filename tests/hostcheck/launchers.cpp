// Stand-ins of the kernel launchers for the host range check: each checks, against the
// buffers the driver registered, every address range its kernel reads or writes, derived
// from the launch arguments the way the kernel derives them.  The batch launcher records
// its arguments so that a graph launch re-checks the per-tile accesses on the current
// instance table.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "hip/hip_runtime.h"
#include "mlp_launch.h"
#include "mppi_device.h"
#include "mppi_launch.h"
#include "proposal_launch.h"
#include "tracking_launch.h"

struct Region {
    const char* base;
    size_t bytes;
};
static std::vector<Region> g_regions;
int g_bad = 0;
int g_batch_tiles = 0, g_prop_rows = 0;

void range_register(const void* p, size_t bytes) { g_regions.push_back({(const char*)p, bytes}); }

bool range_check(const void* p, size_t bytes, const char* what)
{
    for (const Region& r : g_regions)
        if ((const char*)p >= r.base && (const char*)p + bytes <= r.base + r.bytes) return true;
    std::printf("  OUT OF RANGE %s: %p + %zu\n", what, p, bytes);
    ++g_bad;
    return false;
}
#define CHK(p, n, what) \
    do {                \
        if (p) range_check(p, n, what); \
    } while (0)

static void fail(const char* what)
{
    std::printf("  INCONSISTENT %s\n", what);
    ++g_bad;
}

// elements e[n * sn + d * sd] for n < K, d < D
static size_t strided_span(int K, int D, int sn, int sd) { return (size_t)(K - 1) * sn + (size_t)(D - 1) * sd + 1; }

namespace mppi {
hipError_t launch_sample(const DevParams& P, int D, float* eps, uint32_t* raw, hipStream_t)
{
    CHK(eps, 4ull * P.K * D, "sample noise");
    CHK(raw, 4ull * P.K * 4 * ((D + 3) / 4), "sample words");
    return hipSuccess;
}

template <typename R>
static void check_model_hf(const ModelT<R>& M, const float* hf, const char* what)
{
    if (M.scene == 1) range_check(hf, 4ull * M.hf_nx * M.hf_ny, what);
}

hipError_t launch_rollout(const DevModelF& Mf, const DevModelD& Md, int arith, const DevParams& P, const RolloutArgs& a,
                          hipStream_t)
{
    const int D = 12 * P.nk;
    if (P.K < 1 || P.H < 1 || P.nk < 2 || P.nk > kMaxKnots) fail("rollout shape");
    range_check(a.B, 8ull * P.H * P.nk, "rollout basis");
    range_check(a.mu, 4ull * D, "rollout nominal");
    range_check(a.x0, 4ull * P.nx, "rollout state");
    range_check(a.costs, 4ull * P.K, "rollout costs");
    if (a.eps_in) range_check(a.eps_in, 4 * strided_span(P.K, D, a.eps_sn, a.eps_sd), "rollout given noise");
    CHK(a.eps_out, 4ull * D * P.K, "rollout noise out");
    CHK(a.traj, 4ull * P.K * (P.H + 1) * P.nx, "rollout trajectories");
    if (arith == 1) check_model_hf(Mf, a.hf, "rollout heightfield");
    else check_model_hf(Md, a.hf, "rollout heightfield");
    return hipSuccess;
}

hipError_t launch_rollout16(const DevModelF& Mf, const DevModelD& Md, int arith, const DevParams& P,
                            const RolloutArgs& a, hipStream_t st)
{
    if (!rollout16_fits(arith, arith == 1 ? Mf.scene : Md.scene, arith == 1 ? Mf.hf_nx * Mf.hf_ny : Md.hf_nx * Md.hf_ny))
        fail("rollout16 LDS");
    CHK(a.skip, 4, "rollout skip flag");
    CHK(a.input_status, 4, "rollout start-state flag");
    if (!a.direct) return launch_rollout(Mf, Md, arith, P, a, st);  // same ranges as the quad kernel
    const int D = 12 * P.nk;  // direct: one value per step
    if (P.K < 1 || P.H < 1 || P.nk != P.H) fail("rollout16 direct shape");
    range_check(a.mu, 4ull * D, "rollout nominal");
    range_check(a.x0, 4ull * P.nx, "rollout state");
    range_check(a.costs, 4ull * P.K, "rollout costs");
    if (a.eps_in) range_check(a.eps_in, 4 * strided_span(P.K, D, a.eps_sn, a.eps_sd), "rollout given noise");
    CHK(a.eps_out, 4ull * D * P.K, "rollout noise out");
    CHK(a.traj, 4ull * P.K * (P.H + 1) * P.nx, "rollout trajectories");
    return hipSuccess;
}

bool rollout16_fits(int arith, int scene, int hf_cells)
{
    const size_t rows = (4 * (scene == 3 ? 55 : 28) * 20 + 4 * 64) * (arith == 1 ? 4 : 8);
    return rows + (scene == 1 ? 4ull * hf_cells : 0) <= 65536;
}

hipError_t launch_update(const DevParams& P, const UpdateArgs& a, hipStream_t)
{
    const int D = 12 * P.nk;
    range_check(a.costs, 4ull * P.K, "update costs");
    range_check(a.mu, 4ull * D, "update nominal");
    range_check(a.S, 4ull * P.nk * P.nk, "update shift");
    range_check(a.eps, 4 * strided_span(P.K, D, a.eps_sn, a.eps_sd), "update noise");
    CHK(a.knots_out, 4ull * D, "update knots");
    CHK(a.nominal_out, 4ull * D, "update shifted nominal");
    CHK(a.u0_out, 48, "update first control");
    CHK(a.weights_out, 4ull * P.K, "update weights");
    range_check(a.status, 12, "update status");
    if (a.prop) {
        if (a.Kp < 2 || a.Kp > P.K) fail("proposal sample count");
        range_check(a.costs_p, 4ull * a.Kp, "update proposal costs");
        range_check(a.eps_p, 4ull * a.Kp * D, "update proposal noise");
        range_check(a.mu_p, 4ull * D, "update proposal centre");
        CHK(a.gate, 8, "update gate costs");
        CHK(a.pstats, 8, "update proposal counters");
    }
    return hipSuccess;
}

hipError_t launch_sim_step(const DevModelF& Mf, const DevModelD& Md, int arith, int n, int nx, const float* x,
                           const float* u, float, float, float, float* xo, float* tau, const float* hf, hipStream_t)
{
    range_check(x, 4ull * n * nx, "plant state");
    range_check(u, 48ull * n, "plant targets");
    range_check(xo, 4ull * n * nx, "plant next state");
    CHK(tau, 48ull * n, "plant torques");
    if (arith == 1) check_model_hf(Mf, hf, "plant heightfield");
    else check_model_hf(Md, hf, "plant heightfield");
    return hipSuccess;
}

// what one persistent batch kernel touches for each tile of its scene's queue
// (scene -1: the single-launch queue, whose entries are row << 8 | tile of the row)
static void check_batch(int scene, const BatchArgs<double>& a)
{
    const int total = *a.total_tiles;
    std::vector<std::vector<int>> seen;
    for (int t = 0; t < total; ++t) {
        range_check(a.tile_map + t, 4, "tile map");
        const int row = scene < 0 ? a.tile_map[t] >> 8 : a.tile_map[t];
        if (row < 0) fail("negative table row");
        range_check(a.inst + row, sizeof(InstDesc), "instance row");
        const InstDesc& I = a.inst[row];
        const int K = I.P.K, D = 12 * I.P.nk, nx = I.P.nx;
        if (scene >= 0 && I.scene != scene) fail("tile of another scene");
        if (I.scene < 0 || I.scene > 3) fail("scene out of range");
        const int k = scene < 0 ? (a.tile_map[t] & 255) : t - I.tile0;
        if (k < 0 || k >= I.ntiles) fail("tile index outside its instance");
        // every tile of a row exactly once, so the row's tile counter reaches ntiles once
        if ((int)seen.size() <= row) seen.resize(row + 1);
        if (seen[row].empty()) seen[row].assign(I.ntiles, 0);
        if (seen[row][k]++) fail("tile queued twice");
        const int n0 = k * kTileSamples, n1 = std::min(K, n0 + kTileSamples);
        if (n0 < 0 || n0 >= K) fail("tile outside its instance");
        range_check(I.B, 8ull * I.P.H * I.P.nk, "batch basis");
        range_check(I.S, 4ull * I.P.nk * I.P.nk, "batch shift");
        range_check(I.x, 4ull * nx, "batch state");
        range_check(I.mu, 4ull * D, "batch nominal");
        for (int d = 0; d < D; ++d) range_check(I.eps + (size_t)d * K + n0, 4ull * (n1 - n0), "batch noise tile");
        range_check(I.costs + n0, 4ull * (n1 - n0), "batch costs tile");
        range_check(I.w, 4ull * K, "batch weights");
        range_check(I.u0, 48, "batch first control");
        range_check(I.cost_acc, 4, "batch running cost");
        range_check(I.done, 4, "batch tile counter");
        range_check(I.step, 4, "batch step counter");
        CHK(I.rec, 4ull * I.rec_cap * (nx + D), "batch record rows");
        if (I.hf_cells) range_check(I.hf, 4ull * I.hf_cells, "batch heightfield");
        if (I.explicit_eps && I.P.sigma != 1.f) fail("given-noise row without unit scale");
        ++g_batch_tiles;
    }
    for (const auto& r : seen)
        for (int c : r)
            if (c != 1) fail("a tile of a queued row is missing");
}

struct Captured {
    int scene;
    BatchArgs<double> a;
};
static std::vector<Captured> g_captured;

hipError_t launch_batch(int, int scene, const void* args, int grid, size_t lds, hipStream_t)
{
    if (grid < 1 || lds > 65536) fail("batch launch shape");
    g_captured.push_back({scene, *static_cast<const BatchArgs<double>*>(args)});  // same layout for both types
    return hipSuccess;
}

hipError_t launch_batch_all(int, const void* args, int grid, size_t lds, hipStream_t)
{
    if (grid < 1 || lds > 65536) fail("batch launch shape");
    g_captured.push_back({-1, *static_cast<const BatchArgs<double>*>(args)});
    return hipSuccess;
}
}  // namespace mppi

namespace prop {
struct CapturedFeatures;
struct CapturedHead;
void clear_captured();
void replay_captured();
}  // namespace prop

void capture_begin()
{
    mppi::g_captured.clear();
    prop::clear_captured();
}
void capture_replay()
{
    prop::replay_captured();
    for (const auto& c : mppi::g_captured) mppi::check_batch(c.scene, c.a);
}

namespace prop {
hipError_t launch_proposal_noise(int Kp, int D, float* e, const float* center, const float* sd, const float* nominal,
                                 hipStream_t)
{
    range_check(e, 4ull * Kp * D, "proposal noise");
    range_check(center, 4ull * D, "proposal centre");
    range_check(sd, 4ull * D, "proposal std");
    range_check(nominal, 4ull * D, "proposal nominal");
    return hipSuccess;
}

hipError_t launch_gate(int Kp, const float* costs_p, int best, float* g, int* skip, hipStream_t)
{
    if (Kp < 2 || (best != 0 && best != 1)) fail("gate shape");
    range_check(costs_p, 4ull * Kp, "gate proposal costs");
    range_check(g, 8, "gate costs");
    range_check(skip, 4, "gate skip flag");
    return hipSuccess;
}

hipError_t launch_pair_noise(int Kp, int K, int D, float sigma, float* E, const float* e_prop, const float* nominal,
                             const float* center, float* eps_out, hipStream_t)
{
    if (Kp < 2 || K < 1 || D < 1 || !(sigma >= 0.f)) fail("pair noise shape");
    range_check(E, 4ull * (K + Kp) * D, "pair offsets");
    range_check(e_prop, 4ull * Kp * D, "pair proposal noise");
    range_check(nominal, 4ull * D, "pair nominal");
    range_check(center, 4ull * D, "pair centre");
    range_check(eps_out, 4ull * K * D, "pair eps out");
    return hipSuccess;
}

hipError_t launch_features(const float* x, const float* co, float* f, hipStream_t)
{
    range_check(x, 4 * 37, "features state");
    range_check(co, 4 * 5, "features command");
    range_check(f, 4 * 40, "features");
    return hipSuccess;
}

// the batched proposal's launches are captured into the batch graph: each is checked when
// issued and again at every graph launch (capture_replay), against the live table
struct CapturedFeatures {
    int np;
    const mppi::InstDesc* table;
    const BatchPropRow* rows;
    float* feat;
};
struct CapturedHead {
    int np;
    const mppi::InstDesc* table;
    const BatchPropRow* rows;
    const float *out, *omean, *ostd, *rtab;
    float log_lo;
};
std::vector<CapturedFeatures> g_cap_features;
std::vector<CapturedHead> g_cap_head;

hipError_t check_batch_features(int np, const mppi::InstDesc* table, const BatchPropRow* rows, float* feat)
{
    range_check(rows, sizeof(BatchPropRow) * np, "proposal rows");
    range_check(feat, 160ull * np, "batch features");
    for (int r = 0; r < np; ++r) {
        range_check(table + rows[r].row, sizeof(mppi::InstDesc), "proposal table row");
        range_check(table[rows[r].row].x, 4 * 37, "proposal state");
        if (table[rows[r].row].P.nx != 37) fail("proposal state of another size");
    }
    g_prop_rows += np;
    return hipSuccess;
}

hipError_t launch_batch_features(int np, const mppi::InstDesc* table, const BatchPropRow* rows, float* feat,
                                 hipStream_t)
{
    g_cap_features.push_back({np, table, rows, feat});
    return check_batch_features(np, table, rows, feat);
}

hipError_t check_batch_head_noise(int np, const mppi::InstDesc* table, const BatchPropRow* rows, const float* out,
                                  const float* omean, const float* ostd, const float* rtab)
{
    range_check(out, 576ull * np, "proposal network outputs");
    range_check(omean, 4 * 72, "output mean");
    range_check(ostd, 4 * 72, "output std");
    for (int r = 0; r < np; ++r) {
        const BatchPropRow& pr = rows[r];
        const mppi::InstDesc& I = table[pr.row];
        const int nk = pr.nk, D = 12 * nk, K = I.P.K;
        if (nk != I.P.nk || nk < 2 || nk > 8) fail("proposal knots");
        for (int i = 0; i < nk; ++i) range_check(rtab + (size_t)(nk * 8 + i) * 6, 24, "resampling row");
        range_check(I.step, 4, "proposal step counter");
        for (int cb = 0; cb < (D + 3) / 4; ++cb)
            for (int q = 0; q < 4; ++q) {
                const int d = 4 * cb + q;
                if (d < D) range_check(I.eps + (size_t)d * K, 4ull * K, "proposal noise row");
            }
        range_check(I.mu, 4ull * D, "proposal nominal");
        if (!I.explicit_eps || I.P.sigma != 1.f) fail("proposal row flags");
        if (!std::isfinite(pr.log_hi)) fail("proposal std clamp");
    }
    return hipSuccess;
}

hipError_t launch_batch_head_noise(int np, const mppi::InstDesc* table, const BatchPropRow* rows, const float* out,
                                   const float* omean, const float* ostd, const float* rtab, float log_lo,
                                   hipStream_t)
{
    g_cap_head.push_back({np, table, rows, out, omean, ostd, rtab, log_lo});
    return check_batch_head_noise(np, table, rows, out, omean, ostd, rtab);
}

void clear_captured()
{
    g_cap_features.clear();
    g_cap_head.clear();
}
void replay_captured()
{
    for (const auto& c : g_cap_features) check_batch_features(c.np, c.table, c.rows, c.feat);
    for (const auto& c : g_cap_head) check_batch_head_noise(c.np, c.table, c.rows, c.out, c.omean, c.ostd, c.rtab);
}
}  // namespace prop

namespace track {
hipError_t launch_tracking_cost(int arith, const TrackArgs& a, const float* x0, void* table, hipStream_t)
{
    const int D = 12 * a.nk;
    if (a.K < 1 || a.H < 1 || a.nk < 2 || a.nk > 8 || (a.nx != 37 && a.nx != 50) || (arith != 0 && arith != 1))
        fail("tracking shape");
    if (a.c.box != (a.nx == 50)) fail("tracking box flag");
    range_check(x0, 4ull * a.nx, "tracking start state");
    range_check(table, tracking_table_bytes(a.H), "tracking gait table");
    if (((uintptr_t)table & 7) != 0) fail("tracking table alignment");
    range_check(a.traj, 4ull * a.K * (a.H + 1) * a.nx, "tracking trajectories");
    range_check(a.B, 8ull * a.H * a.nk, "tracking basis");
    range_check(a.mu, 4ull * D, "tracking nominal");
    range_check(a.eps, 4 * strided_span(a.K, D, a.eps_sn, a.eps_sd), "tracking noise");
    range_check(a.costs, 4ull * a.K, "tracking costs");
    if (tracking_lds_bytes(arith, a.H, a.nk, a.nx) > 65536) fail("tracking LDS");
    return hipSuccess;
}
size_t tracking_lds_bytes(int arith, int H, int nk, int nx)
{
    (void)H; (void)nk; (void)nx;
    return (arith == 0 ? sizeof(double) : sizeof(float)) * 8 * 12;
}
size_t tracking_table_bytes(int H) { return sizeof(double) * (size_t)(H + 1) * 12; }
}  // namespace track

namespace mlp {
static size_t span(long rows, long ld, long cols, size_t esz) { return ((rows - 1) * ld + cols) * esz; }

hipError_t launch_gemm(int epi, const GemmArgs& g, int splits, hipStream_t)
{
    const int bm = gemm_tile_m(g.M, g.N, splits);
    if (!bm || g.K % kGemmBK || splits < 1) {
        fail("gemm shape");
        return hipErrorInvalidValue;
    }
    range_check(g.A, span(g.M, g.lda, (long)g.K * splits, 2), "gemm A");
    range_check(g.B, span(g.N, g.ldb, (long)g.K * splits, 2), "gemm B");
    if (epi == EPI_SPLITK)
        range_check(g.C, (size_t)(splits - 1) * g.c_split_stride * 4 + span(g.M, g.ldc, g.N, 4), "gemm partials");
    if (epi == EPI_OUT) {
        range_check(g.C, span(g.m_store, g.ldc, g.n_store, 4), "gemm output");
        range_check(g.bias, 4ull * g.n_store, "gemm bias");
    }
    if (epi == EPI_HIDDEN) {
        CHK(g.C, span(g.M, g.ldc, g.N, 4), "gemm pre-activation");
        range_check(g.H, span(g.M, g.ldh, g.N, 2), "gemm activation");
        CHK(g.Ht, span(g.N, g.ldht, g.M, 2), "gemm transposed activation");
        range_check(g.bias, 4ull * g.N, "gemm bias");
    }
    if (epi == EPI_DACT) {
        range_check(g.Zp, span(g.M, g.ldz, g.N, 4), "gemm stored pre-activation");
        range_check(g.H, span(g.M, g.ldh, g.N, 2), "gemm error");
        range_check(g.Ht, span(g.N, g.ldht, g.M, 2), "gemm transposed error");
        range_check(g.colpart, (size_t)(g.M / bm) * g.N * 4, "gemm column partials");
    }
    return hipSuccess;
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t)
{
    if (!a.idx) range_check(a.X, 160ull * a.B, "input rows");
    range_check(a.X0, 2ull * a.Bp * kInPad, "padded input");
    range_check(a.X0t, 2ull * a.Bp * kInPad, "transposed input");
    range_check(a.mean, 160, "input mean");
    range_check(a.std, 160, "input std");
    return hipSuccess;
}

int loss_rows_per_block() { return 32; }

hipError_t launch_loss(const LossArgs& a, hipStream_t)
{
    if (a.Bp % 32) fail("loss rows");
    range_check(a.out, 4ull * a.B * kOut, "loss outputs");
    if (!a.idx) range_check(a.Y, 288ull * a.B, "loss targets");
    range_check(a.dZ, 2ull * a.Bp * kOutPad, "loss error");
    range_check(a.dZt, 2ull * kOutPad * a.Bp, "loss transposed error");
    range_check(a.dbpart, 4ull * (a.Bp / 32) * kOutPad, "loss column partials");
    range_check(a.lpart, 4ull * (a.Bp / 32), "loss partials");
    return hipSuccess;
}

hipError_t launch_loss_sum(const float* lpart, int nl, float, float* loss, hipStream_t)
{
    if (nl < 1) fail("loss partial count");
    range_check(lpart, 4ull * nl, "loss partials");
    range_check(loss, 4, "loss");
    return hipSuccess;
}

hipError_t launch_pairs(const PairsArgs& a, hipStream_t)
{
    if (a.n_rec < 1 || a.steps < 1 || a.nk < 2 || a.nk > 8) fail("pairs shape");
    const size_t rows = (size_t)a.n_rec * a.steps;
    range_check(a.rec, 4 * rows * (37 + 12 * a.nk), "pairs records");
    range_check(a.oc, 12ull * a.n_rec, "pairs origins and commands");
    range_check(a.feat, 160 * rows, "pairs features");
    range_check(a.tgt, 288 * rows, "pairs targets");
    range_check(a.count, 4ull * a.n_rec, "pairs counts");
    return hipSuccess;
}

static void check_reduce(const ReduceArgs& a)
{
    for (int l = 0; l < kLayers; ++l) {
        if (a.S[l] < 1 || a.S[l] > kMaxSplits) fail("split count");
        range_check(a.wpart[l], 4ull * a.S[l] * a.g.fip[l] * a.g.fop[l], "weight partials");
        range_check(a.bpart[l], 4ull * a.T[l] * a.g.fop[l], "bias partials");
    }
    range_check(a.lpart, 4ull * a.nl, "loss partials");
    CHK(a.loss, 4, "loss");
}

static void check_adam(const AdamArgs& a, bool reads_gradient)
{
    const size_t n = a.g.off[kLayers];
    range_check(a.P, 4 * n, "parameters");
    if (a.update) {
        range_check(a.m, 4 * n, "first moments");
        range_check(a.v, 4 * n, "second moments");
        if (reads_gradient) range_check(a.G, 4 * n, "gradient");
    }
    for (int l = 0; l < kLayers; ++l) {
        range_check(a.Wt[l], 2ull * a.g.fop[l] * a.g.fip[l], "transposed weight copy");
        CHK(a.Wn[l], 2ull * a.g.fip[l] * a.g.fop[l], "weight copy");
    }
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t)
{
    check_reduce(a);
    range_check(a.G, 4ull * a.g.off[kLayers], "gradient");
    return hipSuccess;
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t)
{
    check_adam(a, true);
    return hipSuccess;
}

hipError_t launch_reduce_adam(const ReduceArgs& r, const AdamArgs& a, hipStream_t)
{
    check_reduce(r);
    check_adam(a, false);
    return hipSuccess;
}

hipError_t launch_head(const HeadArgs& a, hipStream_t)
{
    range_check(a.out, 4 * kOut, "head outputs");
    range_check(a.omean, 4 * 72, "head mean");
    range_check(a.ostd, 4 * 72, "head std");
    range_check(a.center, 48ull * a.nk, "head centre");
    range_check(a.sd, 48ull * a.nk, "head std out");
    return hipSuccess;
}
}  // namespace mlp
