// Batched serving runtime: many independent MPPI instances advanced by one graph
// launch per control step.
//
// The caller's workspace is the HBM budget.  A first-fit allocator carves per-instance
// buffers (state, nominal, noise, costs, weights, spline matrices) out of it; an
// instance that does not fit is refused with MPPI_EBUDGET and the caller queues it.
// The device instance table, tile map and tile count live at the front of the
// workspace and are re-uploaded (stream-ordered) when the set of instances changes, so
// the captured graph stays valid: the persistent kernel reads everything from the table.
//
// Instances may take their samples from the learned proposal (ungated: every step uses
// the proposal's K samples, the shifted nominal kept as sample 1).  Before the graph, one
// features launch, one network forward over all such instances as a batch, and one
// head-and-noise launch write each one's centre into its nominal slot and its rollout
// noise; the persistent kernel then reads that noise instead of drawing Philox noise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "mppi.h"
#include "mppi_device.h"
#include "mppi_launch.h"
#include "mppi_policy.h"
#include "policy_internal.h"
#include "proposal_launch.h"

// defined in mppi_api.cpp
extern "C++" {
namespace mppi_host {
bool model_info(const mppi_model* m, int* scene, int* nx, const float** hf, int* hf_cells, const void** dev_f,
                const void** dev_d);
void spline_matrices(int nk, int H, double dt, int basis, std::vector<double>& B, std::vector<float>& S);
}  // namespace mppi_host
}

namespace {

constexpr size_t kAlign = 256;
constexpr int kQueues = 5;  // four scene queues and the combined one
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// first-fit allocator over [base, base + size)
struct Arena {
    std::map<size_t, size_t> free_;  // offset -> size
    size_t used = 0;
    void reset(size_t base, size_t size)
    {
        free_.clear();
        if (size) free_[base] = size;
        used = 0;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, o = it->first + bytes;
                free_.erase(it);
                if (rest) free_[o] = rest;
                used += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes);
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct ModelSlot {
    int scene, nx, hf_cells;
    size_t hf_off;
};

struct Instance {
    bool live = false;
    int model = 0;
    mppi_params p{};
    size_t off = 0, bytes = 0;
    float* rec = nullptr;  // caller's record buffer
    int rec_cap = 0;
    bool prop = false;     // samples from the batch's proposal network
    float cmd_origin[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    // offsets inside the allocation
    size_t o_B, o_S, o_x, o_mu, o_eps, o_costs, o_w, o_u0, o_acc, o_done, o_step;
};

}  // namespace

struct mppi_batch {
    int max_inst, max_H, max_hf, arith;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // used only to capture the graph
    size_t o_table, o_models, o_pool;
    size_t o_prows, o_feat, o_pout, o_rtab;  // proposal rows, features, network outputs, resampling
    // one work queue per scene, then the combined queue of the single-launch mode
    size_t o_tiles[kQueues], o_total[kQueues], o_head[kQueues], o_exited[kQueues];
    int scene_tiles[4] = {0, 0, 0, 0};
    bool scene_used[4] = {false, false, false, false};
    Arena arena;
    std::vector<ModelSlot> models;
    std::vector<char> model_blob;  // ModelT<R> per slot (host copy)
    std::vector<Instance> inst;
    mppi::InstDesc* h_table = nullptr;  // pinned mirrors
    int* h_tiles = nullptr;
    hipEvent_t upload_done = nullptr;
    bool dirty = true, upload_pending = false;
    int total_tiles = 0, n_live = 0;
    int grid = 0, blocks_per_cu = 4, order = 1;
    int mode = 0;  // 0: one persistent kernel per scene in use; 1: one kernel for every scene
    mppi_policy* policy = nullptr;  // shared by every proposal instance
    prop::BatchPropRow* h_prows = nullptr;
    int n_prop = 0;
    bool rtab_ready = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // what the graph's proposal launches were captured with: their row count and the
    // policy's workspace (a change of either makes the graph stale)
    int cap_n_prop = 0;
    const mppi_policy* cap_policy = nullptr;
    const void* cap_policy_ws = nullptr;
    std::string err;
};

namespace {

thread_local std::string g_berr;

mppi_status bfail(mppi_batch* b, mppi_status s, const std::string& m)
{
    if (b) b->err = m;
    g_berr = m;
    return s;
}
mppi_status bhip(mppi_batch* b, hipError_t e, const char* what)
{
    if (e == hipSuccess) return MPPI_OK;
    return bfail(b, MPPI_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}
char* wsp(mppi_batch* b, size_t off) { return (char*)b->ws + off; }
size_t model_size(int arith) { return arith == 1 ? sizeof(mppi::ModelT<float>) : sizeof(mppi::ModelT<double>); }
// proposal rows, feature rows (40 floats), network output rows (144 floats), resampling table
size_t prop_bytes(int max_inst)
{
    return align_up(sizeof(prop::BatchPropRow) * max_inst) + align_up(sizeof(float) * 40 * max_inst) +
           align_up(sizeof(float) * 144 * max_inst) + align_up(sizeof(float) * 9 * 8 * 6);
}

// teardown: errors here have no caller to report to and do not change what is released
void drop_graph(mppi_batch* b)
{
    // an executable graph may still be running on the caller's stream (the null stream
    // included): let it finish
    if (b->exec) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->cap_n_prop = 0;
    b->cap_policy = nullptr;
    b->cap_policy_ws = nullptr;
}

size_t batch_lds(const mppi_batch* b)
{
    const size_t rb = b->arith == 1 ? sizeof(float) : sizeof(double);
    return rb * ((size_t)b->max_H * MPPI_MAX_KNOTS + 64 * 3 * MPPI_MAX_KNOTS) + sizeof(float) * (size_t)b->max_hf;
}

// rebuild the table and the per-scene tile maps in the pinned mirrors; queue the upload
mppi_status upload_table(mppi_batch* b)
{
    mppi_status s;
    if (b->upload_pending && (s = bhip(b, hipEventSynchronize(b->upload_done), "wait upload"))) return s;
    const int tiles_per_scene = b->max_inst * (4096 / mppi::kTileSamples);
    int row = 0, all_tiles = 0, np = 0;
    std::vector<int> row_inst;  // admission index of each table row
    for (int sc = 0; sc < 4; ++sc) {
        std::vector<int> ids;
        for (int i = 0; i < b->max_inst; ++i)
            if (b->inst[i].live && b->models[b->inst[i].model].scene == sc) ids.push_back(i);
        if (b->order == 1)  // longest horizon first: long tiles start early, short ones fill the tail
            std::stable_sort(ids.begin(), ids.end(), [&](int x, int y) { return b->inst[x].p.H > b->inst[y].p.H; });
        int* map = b->h_tiles + sc * (tiles_per_scene + 1);
        int tile = 0;
        for (int i : ids) {
            const Instance& in = b->inst[i];
            const mppi_params& p = in.p;
            mppi::InstDesc& d = b->h_table[row];
            d = mppi::InstDesc{};
            d.P.K = p.K; d.P.H = p.H; d.P.nk = p.n_knots; d.P.nx = b->models[in.model].nx;
            d.P.dt = p.dt; d.P.sigma = p.sigma; d.P.inv_lambda = 1.f / p.lambda; d.P.kp = p.kp; d.P.kd = p.kd;
            d.P.w_h = p.w_height; d.P.h_ref = p.h_ref; d.P.w_o = p.w_upright; d.P.w_v = p.w_vel;
            d.P.v_ref = p.v_ref; d.P.w_tau = p.w_torque; d.P.w_reach = p.w_reach; d.P.w_box = p.w_box;
            d.P.goal_x = p.goal[0]; d.P.goal_y = p.goal[1];
            d.P.seed_lo = (uint32_t)(p.seed & 0xffffffffu); d.P.seed_hi = (uint32_t)(p.seed >> 32);
            d.P.instance = p.instance;
            d.scene = sc;
            d.model = in.model;
            d.ntiles = (p.K + mppi::kTileSamples - 1) / mppi::kTileSamples;
            d.tile0 = tile;
            d.hf_cells = b->models[in.model].hf_cells;
            d.hf = d.hf_cells ? (const float*)wsp(b, b->models[in.model].hf_off) : nullptr;
            char* base = wsp(b, in.off);
            d.B = (const double*)(base + in.o_B);
            d.S = (const float*)(base + in.o_S);
            d.x = (float*)(base + in.o_x);
            d.mu = (float*)(base + in.o_mu);
            d.eps = (float*)(base + in.o_eps);
            d.costs = (float*)(base + in.o_costs);
            d.w = (float*)(base + in.o_w);
            d.u0 = (float*)(base + in.o_u0);
            d.cost_acc = (float*)(base + in.o_acc);
            d.done = (int*)(base + in.o_done);
            d.step = (uint32_t*)(base + in.o_step);
            d.rec = in.rec;
            d.rec_cap = in.rec_cap;
            if (in.prop) {  // unit scale around the centre; the admitted sigma is the std clamp
                d.explicit_eps = 1;
                d.P.sigma = 1.f;
                prop::BatchPropRow& pr = b->h_prows[np++];
                pr.row = row;
                pr.nk = p.n_knots;
                pr.log_hi = std::log(p.sigma);
                for (int q = 0; q < 5; ++q) pr.cmd_origin[q] = in.cmd_origin[q];
            }
            for (int k = 0; k < d.ntiles; ++k) map[tile + k] = row;
            tile += d.ntiles;
            row_inst.push_back(i);
            ++row;
        }
        map[tiles_per_scene] = tile;  // the count, staged after the map
        b->scene_tiles[sc] = tile;
        all_tiles += tile;
    }
    // the combined queue: every tile of every row as (row << 8 | tile of the row), rows in
    // admission order or longest horizon first over all scenes (K <= 4096 keeps the tile
    // index below 256)
    int* all_map = b->h_tiles + 4 * (tiles_per_scene + 1);
    {
        std::vector<int> rows(row);
        for (int r = 0; r < row; ++r) rows[r] = r;
        std::sort(rows.begin(), rows.end(), [&](int x, int y) {
            if (b->order == 1 && b->h_table[x].P.H != b->h_table[y].P.H) return b->h_table[x].P.H > b->h_table[y].P.H;
            return row_inst[x] < row_inst[y];
        });
        int tile = 0;
        for (int r : rows)
            for (int k = 0; k < b->h_table[r].ntiles; ++k) all_map[tile++] = (r << 8) | k;
        all_map[tiles_per_scene] = tile;
    }
    b->total_tiles = all_tiles;
    b->n_live = row;
    b->n_prop = np;
    hipStream_t st = b->stream;
    if ((s = bhip(b, hipMemcpyAsync(wsp(b, b->o_table), b->h_table, sizeof(mppi::InstDesc) * std::max(row, 1),
                                    hipMemcpyHostToDevice, st), "upload table")))
        return s;
    for (int q = 0; q < kQueues; ++q) {
        const int* map = b->h_tiles + q * (tiles_per_scene + 1);
        const int n = q < 4 ? b->scene_tiles[q] : all_tiles;
        if (n && (s = bhip(b, hipMemcpyAsync(wsp(b, b->o_tiles[q]), map, sizeof(int) * n, hipMemcpyHostToDevice, st),
                           "upload tiles")))
            return s;
        if ((s = bhip(b, hipMemcpyAsync(wsp(b, b->o_total[q]), map + tiles_per_scene, sizeof(int),
                                        hipMemcpyHostToDevice, st), "upload tile count")))
            return s;
    }
    if (np && (s = bhip(b, hipMemcpyAsync(wsp(b, b->o_prows), b->h_prows, sizeof(prop::BatchPropRow) * np,
                                          hipMemcpyHostToDevice, st), "upload proposal rows")))
        return s;
    if ((s = bhip(b, hipEventRecord(b->upload_done, st), "record upload"))) return s;
    b->upload_pending = true;
    b->dirty = false;
    return MPPI_OK;
}

// learned-proposal instances: features, one forward over all of them, head and noise
mppi_status proposal_prestep(mppi_batch* b, hipStream_t st)
{
    mppi_status s;
    const auto* table = (const mppi::InstDesc*)wsp(b, b->o_table);
    const auto* rows = (const prop::BatchPropRow*)wsp(b, b->o_prows);
    float* feat = (float*)wsp(b, b->o_feat);
    float* out = (float*)wsp(b, b->o_pout);
    if ((s = bhip(b, prop::launch_batch_features(b->n_prop, table, rows, feat, st), "proposal features launch")))
        return s;
    if (mppi_host::policy_forward_rows(b->policy, feat, b->n_prop, out, st) != MPPI_OK)
        return bfail(b, MPPI_EINVAL, std::string("proposal forward: ") + mppi_host::policy_error(b->policy));
    const float *omean, *ostd;
    if (mppi_host::policy_out_norm(b->policy, &omean, &ostd) != MPPI_OK)
        return bfail(b, MPPI_ESTATE, std::string("proposal: ") + mppi_host::policy_error(b->policy));
    return bhip(b, prop::launch_batch_head_noise(b->n_prop, table, rows, out, omean, ostd,
                                                 (const float*)wsp(b, b->o_rtab), std::log(0.02f), st),
                "proposal head launch");
}


// one persistent kernel per scene in use, in one graph
mppi_status capture(mppi_batch* b)
{
    drop_graph(b);
    int dev = 0, cus = 0;
    mppi_status s;
    if ((s = bhip(b, hipGetDevice(&dev), "get device"))) return s;
    if ((s = bhip(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "cu count"))) return s;
    b->grid = std::max(1, cus * b->blocks_per_cu);
    const size_t lds = batch_lds(b);
    // capture on the library's own stream (the caller's may be the legacy null stream,
    // which cannot be captured); the graph is then launched on the caller's stream
    if (!b->cap_stream && (s = bhip(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "stream")))
        return s;
    hipStream_t st = b->cap_stream;
    if ((s = bhip(b, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture"))) return s;
    // the learned-proposal instances' features, network pass and head come first; then the
    // scenes' kernels run one after another, or one kernel takes the combined queue of
    // every scene's tiles
    const mppi_status ps = b->n_prop ? proposal_prestep(b, st) : MPPI_OK;
    hipError_t le = hipSuccess;
    if (b->mode == 1 && !ps) {
        const int q = 4;
        if (b->arith == 1) {
            mppi::BatchArgs<float> a{(const mppi::InstDesc*)wsp(b, b->o_table),
                                     (const mppi::ModelT<float>*)wsp(b, b->o_models),
                                     (const int*)wsp(b, b->o_tiles[q]), (const int*)wsp(b, b->o_total[q]),
                                     (int*)wsp(b, b->o_head[q]), (int*)wsp(b, b->o_exited[q])};
            le = mppi::launch_batch_all(1, &a, b->grid, lds, st);
        } else {
            mppi::BatchArgs<double> a{(const mppi::InstDesc*)wsp(b, b->o_table),
                                      (const mppi::ModelT<double>*)wsp(b, b->o_models),
                                      (const int*)wsp(b, b->o_tiles[q]), (const int*)wsp(b, b->o_total[q]),
                                      (int*)wsp(b, b->o_head[q]), (int*)wsp(b, b->o_exited[q])};
            le = mppi::launch_batch_all(0, &a, b->grid, lds, st);
        }
    }
    for (int sc = 0; sc < 4 && !ps && le == hipSuccess && b->mode == 0; ++sc) {
        if (!b->scene_used[sc]) continue;
        hipStream_t ss = st;
        if (b->arith == 1) {
            mppi::BatchArgs<float> a{(const mppi::InstDesc*)wsp(b, b->o_table),
                                     (const mppi::ModelT<float>*)wsp(b, b->o_models),
                                     (const int*)wsp(b, b->o_tiles[sc]), (const int*)wsp(b, b->o_total[sc]),
                                     (int*)wsp(b, b->o_head[sc]), (int*)wsp(b, b->o_exited[sc])};
            le = mppi::launch_batch(1, sc, &a, b->grid, lds, ss);
        } else {
            mppi::BatchArgs<double> a{(const mppi::InstDesc*)wsp(b, b->o_table),
                                      (const mppi::ModelT<double>*)wsp(b, b->o_models),
                                      (const int*)wsp(b, b->o_tiles[sc]), (const int*)wsp(b, b->o_total[sc]),
                                      (int*)wsp(b, b->o_head[sc]), (int*)wsp(b, b->o_exited[sc])};
            le = mppi::launch_batch(0, sc, &a, b->grid, lds, ss);
        }
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(st, &g);
    if (ps || le != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (ps) return ps;
        if ((s = bhip(b, le, "batch launch"))) return s;
        return bhip(b, ee, "end capture");
    }
    b->graph = g;
    if ((s = bhip(b, hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "instantiate graph"))) return s;
    b->cap_n_prop = b->n_prop;
    b->cap_policy = b->n_prop ? b->policy : nullptr;
    b->cap_policy_ws = b->n_prop ? mppi_host::policy_workspace(b->policy) : nullptr;
    return MPPI_OK;
}

}  // namespace

extern "C" {

mppi_status mppi_batch_create(int max_instances, int max_horizon, int max_hf_cells, int arith, mppi_batch** out)
{
    if (!out) return bfail(nullptr, MPPI_EINVAL, "null output");
    *out = nullptr;
    if (max_instances < 1 || max_instances > 4096) return bfail(nullptr, MPPI_EINVAL, "max_instances in [1, 4096]");
    if (max_horizon < 1 || max_horizon > MPPI_MAX_HORIZON) return bfail(nullptr, MPPI_EINVAL, "bad max_horizon");
    if (max_hf_cells < 0 || max_hf_cells > MPPI_MAX_HEIGHTFIELD) return bfail(nullptr, MPPI_EINVAL, "bad max_hf_cells");
    if (arith != MPPI_ARITH_FP64 && arith != MPPI_ARITH_FP32) return bfail(nullptr, MPPI_EINVAL, "bad arith");
    mppi_batch* b = new (std::nothrow) mppi_batch();
    if (!b) return bfail(nullptr, MPPI_ENOMEM, "host allocation failed");
    b->max_inst = max_instances;
    b->max_H = max_horizon;
    b->max_hf = max_hf_cells;
    b->arith = arith;
    if (batch_lds(b) > 65536) {
        delete b;
        return bfail(nullptr, MPPI_EINVAL, "max_horizon and max_hf_cells exceed the 64 KiB LDS stage");
    }
    b->inst.resize(max_instances);
    const int max_tiles = max_instances * (4096 / mppi::kTileSamples);
    if (hipHostMalloc((void**)&b->h_table, sizeof(mppi::InstDesc) * max_instances, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&b->h_tiles, sizeof(int) * kQueues * (max_tiles + 1), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->h_prows, sizeof(prop::BatchPropRow) * max_instances, hipHostMallocDefault) !=
            hipSuccess ||
        hipEventCreateWithFlags(&b->upload_done, hipEventDisableTiming) != hipSuccess) {
        mppi_batch_destroy(b);
        return bfail(nullptr, MPPI_EHIP, "pinned host allocation failed");
    }
    *out = b;
    return MPPI_OK;
}

void mppi_batch_destroy(mppi_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->upload_done) (void)hipEventDestroy(b->upload_done);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->h_table) (void)hipHostFree(b->h_table);
    if (b->h_tiles) (void)hipHostFree(b->h_tiles);
    if (b->h_prows) (void)hipHostFree(b->h_prows);
    delete b;
}

size_t mppi_batch_control_bytes(int max_instances, int arith)
{
    const int max_tiles = max_instances * (4096 / mppi::kTileSamples);
    return align_up(sizeof(mppi::InstDesc) * max_instances) +
           kQueues * (align_up(sizeof(int) * max_tiles) + 3 * kAlign) +
           align_up(model_size(arith) * MPPI_BATCH_MAX_MODELS) + prop_bytes(max_instances);
}

mppi_status mppi_batch_bind(mppi_batch* b, void* ws, size_t bytes, void* stream)
{
    if (!b || !ws) return bfail(b, MPPI_EINVAL, "null batch or workspace");
    if (((uintptr_t)ws & (kAlign - 1)) != 0) return bfail(b, MPPI_EINVAL, "workspace must be 256-byte aligned");
    const size_t ctrl = mppi_batch_control_bytes(b->max_inst, b->arith);
    if (bytes < ctrl) return bfail(b, MPPI_ENOMEM, "workspace smaller than the control region");
    drop_graph(b);
    b->ws = ws;
    b->ws_bytes = bytes;
    b->stream = (hipStream_t)stream;
    size_t o = 0;
    b->o_table = o; o += align_up(sizeof(mppi::InstDesc) * b->max_inst);
    const size_t queues = o;
    for (int q = 0; q < kQueues; ++q) {
        b->o_total[q] = o; o += kAlign;
        b->o_head[q] = o; o += kAlign;
        b->o_exited[q] = o; o += kAlign;
    }
    for (int q = 0; q < kQueues; ++q) {
        b->o_tiles[q] = o;
        o += align_up(sizeof(int) * b->max_inst * (4096 / mppi::kTileSamples));
    }
    b->o_models = o; o += align_up(model_size(b->arith) * MPPI_BATCH_MAX_MODELS);
    b->o_prows = o; o += align_up(sizeof(prop::BatchPropRow) * b->max_inst);
    b->o_feat = o; o += align_up(sizeof(float) * 40 * b->max_inst);
    b->o_pout = o; o += align_up(sizeof(float) * 144 * b->max_inst);
    b->o_rtab = o; o += align_up(sizeof(float) * 9 * 8 * 6);
    b->o_pool = o;
    b->arena.reset(o, bytes - o);
    b->models.clear();
    b->model_blob.assign(model_size(b->arith) * MPPI_BATCH_MAX_MODELS, 0);
    for (auto& in : b->inst) in = Instance{};
    for (int sc = 0; sc < 4; ++sc) b->scene_used[sc] = false;
    b->policy = nullptr;
    b->n_prop = 0;
    b->rtab_ready = false;
    b->dirty = true;
    hipStream_t st = b->stream;
    mppi_status s;
    // zero the queue heads, exit counters and tile counts (plain fill before any capture)
    if ((s = bhip(b, hipMemsetAsync(wsp(b, queues), 0, kQueues * 3 * kAlign, st), "clear queues"))) return s;
    return bhip(b, hipStreamSynchronize(st), "bind synchronise");
}

mppi_status mppi_batch_add_model(mppi_batch* b, const mppi_model* m, int* slot_out)
{
    if (!b || !m || !slot_out) return bfail(b, MPPI_EINVAL, "null argument");
    if (!b->ws) return bfail(b, MPPI_ESTATE, "no workspace bound");
    if ((int)b->models.size() >= MPPI_BATCH_MAX_MODELS) return bfail(b, MPPI_EINVAL, "too many models");
    int scene, nx, cells;
    const float* hf;
    const void *df, *dd;
    mppi_host::model_info(m, &scene, &nx, &hf, &cells, &df, &dd);
    if (scene == MPPI_SCENE_HEIGHTFIELD && cells > b->max_hf)
        return bfail(b, MPPI_EINVAL, "heightfield larger than max_hf_cells");
    ModelSlot ms{scene, nx, scene == MPPI_SCENE_HEIGHTFIELD ? cells : 0, 0};
    mppi_status s;
    if (ms.hf_cells) {
        if (!b->arena.alloc(sizeof(float) * ms.hf_cells, &ms.hf_off))
            return bfail(b, MPPI_EBUDGET, "no room for the heightfield in the workspace");
        if ((s = bhip(b, hipMemcpy(wsp(b, ms.hf_off), hf, sizeof(float) * ms.hf_cells, hipMemcpyHostToDevice),
                      "upload heightfield")))
            return s;
    }
    const int slot = (int)b->models.size();
    b->models.push_back(ms);
    if (!b->scene_used[scene]) {
        b->scene_used[scene] = true;
        drop_graph(b);  // a new scene adds a kernel to the graph
    }
    const size_t sz = model_size(b->arith);
    std::memcpy(&b->model_blob[sz * slot], b->arith == 1 ? df : dd, sz);
    if ((s = bhip(b, hipMemcpy(wsp(b, b->o_models + sz * slot), &b->model_blob[sz * slot], sz,
                               hipMemcpyHostToDevice), "upload model")))
        return s;
    *slot_out = slot;
    return MPPI_OK;
}

mppi_status mppi_batch_admit(mppi_batch* b, int slot, const mppi_params* p, const float* x0, const float* mu,
                             int* id_out)
{
    if (!b || !p || !x0 || !mu || !id_out) return bfail(b, MPPI_EINVAL, "null argument");
    if (!b->ws) return bfail(b, MPPI_ESTATE, "no workspace bound");
    if (slot < 0 || slot >= (int)b->models.size()) return bfail(b, MPPI_EINVAL, "unknown model slot");
    if (p->K < 1 || p->K > 4096) return bfail(b, MPPI_EINVAL, "K must be in [1, 4096] for batched serving");
    if (p->H < 1 || p->H > b->max_H) return bfail(b, MPPI_EINVAL, "H outside [1, max_horizon]");
    if (p->n_knots < 2 || p->n_knots > MPPI_MAX_KNOTS) return bfail(b, MPPI_EINVAL, "n_knots must be in [2, 8]");
    if (!(p->dt > 0.f) || !(p->lambda > 0.f) || !(p->sigma >= 0.f)) return bfail(b, MPPI_EINVAL, "bad dt/lambda/sigma");
    if (p->basis < MPPI_BASIS_CUBIC || p->basis > MPPI_BASIS_ZERO) return bfail(b, MPPI_EINVAL, "unknown basis");
    if (p->cost != MPPI_COST_RUNNING) return bfail(b, MPPI_EINVAL, "batch instances use the running cost");
    int id = -1;
    for (int i = 0; i < b->max_inst; ++i)
        if (!b->inst[i].live) {
            id = i;
            break;
        }
    if (id < 0) return bfail(b, MPPI_EBUDGET, "instance table full");
    Instance in{};
    in.model = slot;
    in.p = *p;
    const int nx = b->models[slot].nx, D = 12 * p->n_knots;
    size_t o = 0;
    in.o_B = o; o = align_up(o + sizeof(double) * p->H * p->n_knots);
    in.o_S = o; o = align_up(o + sizeof(float) * p->n_knots * p->n_knots);
    in.o_x = o; o = align_up(o + sizeof(float) * nx);
    in.o_mu = o; o = align_up(o + sizeof(float) * D);
    in.o_eps = o; o = align_up(o + sizeof(float) * (size_t)D * p->K);
    in.o_costs = o; o = align_up(o + sizeof(float) * p->K);
    in.o_w = o; o = align_up(o + sizeof(float) * p->K);
    in.o_u0 = o; o = align_up(o + sizeof(float) * 12);
    in.o_acc = o; o = align_up(o + sizeof(float));
    in.o_done = o; o = align_up(o + sizeof(int));
    in.o_step = o; o = align_up(o + sizeof(uint32_t));
    in.bytes = o;
    if (!b->arena.alloc(in.bytes, &in.off)) return bfail(b, MPPI_EBUDGET, "instance does not fit in the HBM budget");
    // initial contents, written in stream order behind any running step
    std::vector<char> init(in.bytes, 0);
    std::vector<double> Bm;
    std::vector<float> Sm;
    mppi_host::spline_matrices(p->n_knots, p->H, p->dt, p->basis, Bm, Sm);
    std::memcpy(&init[in.o_B], Bm.data(), sizeof(double) * Bm.size());
    std::memcpy(&init[in.o_S], Sm.data(), sizeof(float) * Sm.size());
    std::memcpy(&init[in.o_x], x0, sizeof(float) * nx);
    std::memcpy(&init[in.o_mu], mu, sizeof(float) * D);
    mppi_status s;
    if ((s = bhip(b, hipMemcpyAsync(wsp(b, in.off), init.data(), in.bytes, hipMemcpyHostToDevice, b->stream),
                  "upload instance")) ||
        (s = bhip(b, hipStreamSynchronize(b->stream), "admit synchronise"))) {
        b->arena.release(in.off, in.bytes);
        return s;
    }
    in.live = true;
    b->inst[id] = in;
    b->dirty = true;
    *id_out = id;
    return MPPI_OK;
}

mppi_status mppi_batch_remove(mppi_batch* b, int id)
{
    if (!b || id < 0 || id >= b->max_inst || !b->inst[id].live) return bfail(b, MPPI_EINVAL, "unknown instance");
    // later admissions reuse the memory only through stream-ordered copies
    b->arena.release(b->inst[id].off, b->inst[id].bytes);
    b->inst[id].live = false;
    b->dirty = true;
    return MPPI_OK;
}

mppi_status mppi_batch_record(mppi_batch* b, int id, float* d_rec, int cap)
{
    if (!b || id < 0 || id >= b->max_inst || !b->inst[id].live) return bfail(b, MPPI_EINVAL, "unknown instance");
    if (d_rec && cap < 1) return bfail(b, MPPI_EINVAL, "record capacity must be >= 1");
    b->inst[id].rec = d_rec;
    b->inst[id].rec_cap = d_rec ? cap : 0;
    b->dirty = true;
    return MPPI_OK;
}

mppi_status mppi_batch_set_proposal(mppi_batch* b, int id, mppi_policy* pol, const float* cmd, const float* origin_xy)
{
    if (!b || id < 0 || id >= b->max_inst || !b->inst[id].live) return bfail(b, MPPI_EINVAL, "unknown instance");
    Instance& in = b->inst[id];
    if (!pol) {
        if (in.prop) b->dirty = true;
        in.prop = false;
        return MPPI_OK;
    }
    if (b->models[in.model].nx != 37) return bfail(b, MPPI_EINVAL, "the proposal needs a 37-float state model");
    if (!cmd || !origin_xy) return bfail(b, MPPI_EINVAL, "null command or origin");
    if (in.p.K < 2) return bfail(b, MPPI_EINVAL, "the proposal needs K >= 2 samples");
    if (!(in.p.sigma > 0.f)) return bfail(b, MPPI_EINVAL, "the proposal needs sigma > 0 (upper std clamp)");
    if (b->policy && b->policy != pol)
        for (const auto& o : b->inst)
            if (o.live && o.prop && &o != &in)
                return bfail(b, MPPI_EINVAL, "every proposal instance of a batch uses the same policy");
    const float *om, *os;
    if (mppi_host::policy_out_norm(pol, &om, &os) != MPPI_OK)
        return bfail(b, MPPI_ESTATE, std::string("proposal: ") + mppi_host::policy_error(pol));
    mppi_status s;
    if (!b->rtab_ready) {
        float rtab[9 * 8 * 6];
        mppi_host::policy_resample_table(rtab);
        if ((s = bhip(b, hipMemcpyAsync(wsp(b, b->o_rtab), rtab, sizeof(rtab), hipMemcpyHostToDevice, b->stream),
                      "upload resampling table")) ||
            (s = bhip(b, hipStreamSynchronize(b->stream), "synchronise")))
            return s;
        b->rtab_ready = true;
    }
    b->policy = pol;
    for (int q = 0; q < 3; ++q) in.cmd_origin[q] = cmd[q];
    in.cmd_origin[3] = origin_xy[0];
    in.cmd_origin[4] = origin_xy[1];
    in.prop = true;
    b->dirty = true;
    return MPPI_OK;
}

mppi_status mppi_batch_step(mppi_batch* b)
{
    if (!b) return bfail(nullptr, MPPI_EINVAL, "null batch");
    if (!b->ws) return bfail(b, MPPI_ESTATE, "no workspace bound");
    mppi_status s;
    if (b->dirty && (s = upload_table(b))) return s;
    if (b->total_tiles == 0) return MPPI_OK;
    // the graph holds the proposal launches for the row count and policy workspace it was
    // captured with
    if (b->exec && (b->n_prop != b->cap_n_prop ||
                    (b->n_prop && (b->policy != b->cap_policy ||
                                   mppi_host::policy_workspace(b->policy) != b->cap_policy_ws))))
        drop_graph(b);
    if (!b->exec && (s = capture(b))) return s;
    return bhip(b, hipGraphLaunch(b->exec, b->stream), "graph launch");
}

mppi_status mppi_batch_set_tuning(mppi_batch* b, int blocks_per_cu, int order)
{
    if (!b || blocks_per_cu < 1 || blocks_per_cu > 32 || (order != 0 && order != 1))
        return bfail(b, MPPI_EINVAL, "blocks_per_cu in [1, 32], order 0 (admission) or 1 (longest horizon first)");
    if (blocks_per_cu != b->blocks_per_cu) drop_graph(b);
    b->blocks_per_cu = blocks_per_cu;
    if (order != b->order) b->dirty = true;
    b->order = order;
    return MPPI_OK;
}

mppi_status mppi_batch_set_launch_mode(mppi_batch* b, int mode)
{
    if (!b || (mode != 0 && mode != 1))
        return bfail(b, MPPI_EINVAL, "launch mode 0 (one kernel per scene) or 1 (one kernel for every scene)");
    if (mode != b->mode) drop_graph(b);
    b->mode = mode;
    return MPPI_OK;
}

mppi_status mppi_batch_get_tuning(mppi_batch* b, int* blocks_per_cu, int* order, int* mode)
{
    if (!b) return bfail(nullptr, MPPI_EINVAL, "null batch");
    if (blocks_per_cu) *blocks_per_cu = b->blocks_per_cu;
    if (order) *order = b->order;
    if (mode) *mode = b->mode;
    return MPPI_OK;
}

mppi_status mppi_batch_autotune(mppi_batch* b, int steps, int* best_blocks_per_cu, int* best_order,
                                float* best_ms)
{
    if (!b || steps < 1) return bfail(b, MPPI_EINVAL, "null batch or steps < 1");
    if (!b->ws) return bfail(b, MPPI_ESTATE, "no workspace bound");
    const int cand_blocks[] = {2, 4, 8, 16};
    float best = 1e30f;
    int bb = b->blocks_per_cu, bo = b->order, bm = b->mode;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return bfail(b, MPPI_EHIP, "event create");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bfail(b, MPPI_EHIP, "event create");
    }
    mppi_status s = MPPI_OK;
    for (int c = 0; c < 16 && !s; ++c) {
        const int mode = c >> 3, order = (c >> 2) & 1, cb = cand_blocks[c & 3];
        if ((s = mppi_batch_set_launch_mode(b, mode)) || (s = mppi_batch_set_tuning(b, cb, order))) break;
        if ((s = mppi_batch_step(b))) break;  // warm-up and capture
        if ((s = bhip(b, hipEventRecord(e0, b->stream), "autotune event"))) break;
        for (int i = 0; i < steps && !s; ++i) s = mppi_batch_step(b);
        if (s || (s = bhip(b, hipEventRecord(e1, b->stream), "autotune event"))) break;
        float ms = 0.f;
        if ((s = bhip(b, hipEventSynchronize(e1), "autotune wait")) ||
            (s = bhip(b, hipEventElapsedTime(&ms, e0, e1), "autotune timing")))
            break;
        ms /= steps;
        if (ms < best) {
            best = ms;
            bb = cb;
            bo = order;
            bm = mode;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) return s;
    if ((s = mppi_batch_set_launch_mode(b, bm)) || (s = mppi_batch_set_tuning(b, bb, bo))) return s;
    if (best_blocks_per_cu) *best_blocks_per_cu = bb;
    if (best_order) *best_order = bo;
    if (best_ms) *best_ms = best;
    return MPPI_OK;
}

mppi_status mppi_batch_read(mppi_batch* b, int id, float* x, float* u0, float* mu, float* cost_acc, uint32_t* step)
{
    if (!b || id < 0 || id >= b->max_inst || !b->inst[id].live) return bfail(b, MPPI_EINVAL, "unknown instance");
    const Instance& in = b->inst[id];
    mppi_status s;
    if ((s = bhip(b, hipStreamSynchronize(b->stream), "synchronise"))) return s;
    char* base = wsp(b, in.off);
    const int nx = b->models[in.model].nx, D = 12 * in.p.n_knots;
    if (x && (s = bhip(b, hipMemcpy(x, base + in.o_x, sizeof(float) * nx, hipMemcpyDeviceToHost), "read x")))
        return s;
    if (u0 && (s = bhip(b, hipMemcpy(u0, base + in.o_u0, sizeof(float) * 12, hipMemcpyDeviceToHost), "read u0")))
        return s;
    if (mu && (s = bhip(b, hipMemcpy(mu, base + in.o_mu, sizeof(float) * D, hipMemcpyDeviceToHost), "read mu")))
        return s;
    if (cost_acc &&
        (s = bhip(b, hipMemcpy(cost_acc, base + in.o_acc, sizeof(float), hipMemcpyDeviceToHost), "read cost")))
        return s;
    if (step &&
        (s = bhip(b, hipMemcpy(step, base + in.o_step, sizeof(uint32_t), hipMemcpyDeviceToHost), "read step")))
        return s;
    return MPPI_OK;
}

mppi_status mppi_batch_stats(const mppi_batch* b, int* n_live, int* total_tiles, size_t* bytes_used,
                             size_t* bytes_pool)
{
    if (!b) return bfail(nullptr, MPPI_EINVAL, "null batch");
    int live = 0;
    for (const auto& in : b->inst) live += in.live;
    if (n_live) *n_live = live;
    if (total_tiles) *total_tiles = b->total_tiles;
    if (bytes_used) *bytes_used = b->arena.used;
    if (bytes_pool) *bytes_pool = b->ws ? b->ws_bytes - b->o_pool : 0;
    return MPPI_OK;
}

const char* mppi_batch_last_error(const mppi_batch* b) { return b ? b->err.c_str() : g_berr.c_str(); }

}  // extern "C"
