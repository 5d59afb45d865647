// C ABI of the learned sampling proposal: parameter storage, workspace layout, seeded
// initialisation, checkpoints, and the launch sequences of the forward pass, the
// gradient (forward, loss, backward, fixed-order reduction) and Adam.
#include "mppi_policy.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mlp_launch.h"
#include "policy_internal.h"
#include "proposal_launch.h"

using namespace mlp;

struct mppi_policy {
    int max_batch = 0, bp_max = 0;
    std::vector<float> hP, hm, hv;  // host copies (initial values or a loaded checkpoint)
    float norm[224];                // in_mean 40, in_std 40, out_mean 72, out_std 72
    int steps = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    LayerGeom geom{};
    size_t o_P, o_m, o_v, o_G, o_Wt[kLayers], o_Wn[kLayers], o_norm, o_X0, o_X0t;
    size_t o_Z[kLayers - 1], o_H[kLayers - 1], o_Ht[kLayers - 1];
    size_t o_out, o_dZ[2], o_dZt[2], o_wpart[kLayers], o_bpart[kLayers], o_lpart, o_loss, o_feat, o_out1;
    size_t shadow_begin, shadow_end, total;
    std::string err;
};

namespace {

thread_local std::string g_perr;

const int kFi[kLayers] = {kIn, kHidden, kHidden, kHidden, kHidden};
const int kFo[kLayers] = {kHidden, kHidden, kHidden, kHidden, kOut};
const int kFip[kLayers] = {kInPad, kHidden, kHidden, kHidden, kHidden};
const int kFop[kLayers] = {kHidden, kHidden, kHidden, kHidden, kOutPad};

mppi_status pfail(mppi_policy* p, mppi_status s, const std::string& msg)
{
    if (p) p->err = msg;
    g_perr = msg;
    return s;
}

mppi_status phip(mppi_policy* p, hipError_t e, const char* what)
{
    if (e == hipSuccess) return MPPI_OK;
    return pfail(p, MPPI_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename T>
T* at(mppi_policy* p, size_t off)
{
    return reinterpret_cast<T*>(static_cast<char*>(p->ws) + off);
}

int pad64(int b) { return (b + 63) / 64 * 64; }

// splits of the batch reduction of the weight gradients: K per split a multiple of 64
int batch_splits(int bp)
{
    int s = kMaxSplits;
    while (s > 1 && bp % (64 * s)) s >>= 1;
    return s;
}

uint64_t splitmix(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void layout(mppi_policy* p)
{
    const int n = p->geom.off[kLayers];
    const int bp = p->bp_max;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = a256(o + bytes);
        return r;
    };
    p->o_P = take(4ull * n);
    p->o_m = take(4ull * n);
    p->o_v = take(4ull * n);
    p->o_G = take(4ull * n);
    p->shadow_begin = o;
    for (int l = 0; l < kLayers; ++l) p->o_Wt[l] = take(2ull * kFop[l] * kFip[l]);
    for (int l = 0; l < kLayers; ++l) p->o_Wn[l] = l ? take(2ull * kFip[l] * kFop[l]) : 0;
    p->shadow_end = o;
    p->o_norm = take(4ull * 224);
    p->o_X0 = take(2ull * bp * kInPad);
    p->o_X0t = take(2ull * bp * kInPad);
    for (int l = 0; l < kLayers - 1; ++l) {
        p->o_Z[l] = take(4ull * bp * kHidden);
        p->o_H[l] = take(2ull * bp * kHidden);
        p->o_Ht[l] = take(2ull * bp * kHidden);
    }
    p->o_out = take(4ull * bp * kOut);
    for (int i = 0; i < 2; ++i) {
        p->o_dZ[i] = take(2ull * bp * kHidden);
        p->o_dZt[i] = take(2ull * bp * kHidden);
    }
    for (int l = 0; l < kLayers; ++l) p->o_wpart[l] = take(4ull * kMaxSplits * kFip[l] * kFop[l]);
    // column-sum partials: at most one row per 32 batch rows (loss workgroups; the
    // input-gradient GEMM tiles are 64 or 128 rows)
    for (int l = 0; l < kLayers; ++l) p->o_bpart[l] = take(4ull * (bp / 32) * kFop[l]);
    p->o_lpart = take(4ull * (bp / 32));
    p->o_loss = take(4ull * 4);
    p->o_feat = take(4ull * kIn);
    p->o_out1 = take(4ull * kOut);
    p->total = o;
}

mppi_status need_bound(mppi_policy* p)
{
    if (!p) return pfail(nullptr, MPPI_EINVAL, "null policy");
    if (!p->ws) return pfail(p, MPPI_ESTATE, "no workspace bound (call mppi_policy_bind)");
    return MPPI_OK;
}

mppi_status refresh_shadows(mppi_policy* p, hipStream_t st)
{
    AdamArgs a{};
    a.g = p->geom;
    a.P = at<float>(p, p->o_P);
    for (int l = 0; l < kLayers; ++l) {
        a.Wt[l] = at<__bf16>(p, p->o_Wt[l]);
        a.Wn[l] = l ? at<__bf16>(p, p->o_Wn[l]) : nullptr;
    }
    a.update = 0;
    return phip(p, launch_adam(a, st), "shadow refresh launch");
}

// forward over rows of d_in (idx or identity): fills Z, H, H^T of the hidden layers and
// the output (d_out rows < B, stride 144, or the internal output buffer)
mppi_status forward(mppi_policy* p, const float* d_in, const int* d_idx, int B, float* d_out, bool keep,
                    hipStream_t st)
{
    const int bp = pad64(B);
    PrepArgs pa{d_in, d_idx, B, bp, at<float>(p, p->o_norm), at<float>(p, p->o_norm) + 40,
                at<__bf16>(p, p->o_X0), at<__bf16>(p, p->o_X0t)};
    mppi_status s;
    if ((s = phip(p, launch_prep(pa, st), "input launch"))) return s;
    const float* P = at<float>(p, p->o_P);
    for (int l = 0; l < kLayers; ++l) {
        GemmArgs g{};
        g.A = l ? at<__bf16>(p, p->o_H[l - 1]) : at<__bf16>(p, p->o_X0);
        g.lda = kFip[l];
        g.B = at<__bf16>(p, p->o_Wt[l]);
        g.ldb = kFip[l];
        g.M = bp;
        g.N = kFop[l];
        g.K = kFip[l];
        g.bias = P + p->geom.off[l] + kFi[l] * kFo[l];
        if (l < kLayers - 1) {
            g.C = keep ? at<float>(p, p->o_Z[l]) : nullptr;
            g.ldc = kHidden;
            g.H = at<__bf16>(p, p->o_H[l]);
            g.ldh = kHidden;
            g.Ht = keep ? at<__bf16>(p, p->o_Ht[l]) : nullptr;
            g.ldht = bp;
            if ((s = phip(p, launch_gemm(EPI_HIDDEN, g, 1, st), "forward launch"))) return s;
        } else {
            g.C = d_out;
            g.ldc = kOut;
            g.m_store = B;
            g.n_store = kOut;
            if ((s = phip(p, launch_gemm(EPI_OUT, g, 1, st), "output launch"))) return s;
        }
    }
    return MPPI_OK;
}

// forward, loss and backward products; ra receives the partial-sum layout of the gradient
mppi_status backward(mppi_policy* p, const float* d_in, const float* d_target, const int* d_idx, int B,
                     ReduceArgs& ra, hipStream_t st)
{
    const int bp = pad64(B);
    mppi_status s;
    float* out = at<float>(p, p->o_out);
    if ((s = forward(p, d_in, d_idx, B, out, true, st))) return s;
    const float* nrm = at<float>(p, p->o_norm);
    LossArgs la{out, d_target, d_idx, B, bp, nrm + 80, nrm + 152, at<__bf16>(p, p->o_dZ[0]),
                at<__bf16>(p, p->o_dZt[0]), at<float>(p, p->o_bpart[kLayers - 1]), at<float>(p, p->o_lpart)};
    if ((s = phip(p, launch_loss(la, st), "loss launch"))) return s;
    ra = ReduceArgs{};
    ra.g = p->geom;
    ra.T[kLayers - 1] = bp / loss_rows_per_block();
    const int S = batch_splits(bp);
    int cur = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        GemmArgs w{};
        w.A = l ? at<__bf16>(p, p->o_Ht[l - 1]) : at<__bf16>(p, p->o_X0t);
        w.lda = bp;
        w.B = at<__bf16>(p, p->o_dZt[cur]);
        w.ldb = bp;
        w.M = kFip[l];
        w.N = kFop[l];
        w.K = bp / S;
        w.C = at<float>(p, p->o_wpart[l]);
        w.ldc = kFop[l];
        w.c_split_stride = (long)kFip[l] * kFop[l];
        if ((s = phip(p, launch_gemm(EPI_SPLITK, w, S, st), "weight-gradient launch"))) return s;
        ra.wpart[l] = w.C;
        ra.S[l] = S;
        ra.bpart[l] = at<float>(p, p->o_bpart[l]);
        if (l == 0) break;
        GemmArgs d{};
        d.A = at<__bf16>(p, p->o_dZ[cur]);
        d.lda = kFop[l];
        d.B = at<__bf16>(p, p->o_Wn[l]);
        d.ldb = kFop[l];
        d.M = bp;
        d.N = kFip[l];
        d.K = kFop[l];
        d.Zp = at<float>(p, p->o_Z[l - 1]);
        d.ldz = kHidden;
        d.H = at<__bf16>(p, p->o_dZ[cur ^ 1]);
        d.ldh = kHidden;
        d.Ht = at<__bf16>(p, p->o_dZt[cur ^ 1]);
        d.ldht = bp;
        d.colpart = at<float>(p, p->o_bpart[l - 1]);
        const int bm = gemm_tile_m(d.M, d.N, 1);
        if (!bm) return pfail(p, MPPI_EINVAL, "bad backward shape");
        ra.T[l - 1] = bp / bm;
        if ((s = phip(p, launch_gemm(EPI_DACT, d, 1, st), "input-gradient launch"))) return s;
        cur ^= 1;
    }
    ra.lpart = at<float>(p, p->o_lpart);
    ra.nl = bp / loss_rows_per_block();
    ra.lscale = (float)(1.0 / ((double)B * 72.0));
    return MPPI_OK;
}

mppi_status grad(mppi_policy* p, const float* d_in, const float* d_target, const int* d_idx, int B, float* d_grad,
                 float* d_loss, hipStream_t st)
{
    ReduceArgs ra;
    mppi_status s;
    if ((s = backward(p, d_in, d_target, d_idx, B, ra, st))) return s;
    ra.G = d_grad;
    ra.loss = d_loss;
    return phip(p, launch_reduce(ra, st), "reduce launch");
}

AdamArgs adam_args(mppi_policy* p, const float* d_grad, float lr)
{
    const int t = p->steps + 1;
    AdamArgs a{};
    a.g = p->geom;
    a.P = at<float>(p, p->o_P);
    a.m = at<float>(p, p->o_m);
    a.v = at<float>(p, p->o_v);
    a.G = d_grad;
    a.lr = lr;
    a.b1 = 0.9f;
    a.b2 = 0.999f;
    a.omb1 = (float)(1.0 - 0.9);
    a.omb2 = (float)(1.0 - 0.999);
    a.eps = 1e-8f;
    a.inv_c1 = (float)(1.0 / (1.0 - std::pow(0.9, t)));
    a.inv_c2 = (float)(1.0 / (1.0 - std::pow(0.999, t)));
    for (int l = 0; l < kLayers; ++l) {
        a.Wt[l] = at<__bf16>(p, p->o_Wt[l]);
        a.Wn[l] = l ? at<__bf16>(p, p->o_Wn[l]) : nullptr;
    }
    a.update = 1;
    return a;
}

mppi_status adam(mppi_policy* p, const float* d_grad, float lr, hipStream_t st)
{
    mppi_status s = phip(p, launch_adam(adam_args(p, d_grad, lr), st), "adam launch");
    if (!s) p->steps += 1;
    return s;
}

mppi_status check_batch(mppi_policy* p, int B)
{
    if (B < 1 || B > p->max_batch) return pfail(p, MPPI_EINVAL, "batch must be in [1, max_batch]");
    return MPPI_OK;
}

// resampling of the 6-knot spline at nk knots spaced over the same horizon
void resample_matrix(int nk, float R[8][kKnots])
{
    std::vector<double> B, Sd;
    std::memset(R, 0, sizeof(float) * 8 * kKnots);
    if (nk == kKnots) {
        for (int i = 0; i < kKnots; ++i) R[i][i] = 1.f;
        return;
    }
    // basis of the 6-knot not-a-knot spline on [0, 1] evaluated at i / (nk - 1)
    for (int k = 0; k < kKnots; ++k)
        for (int i = 0; i < nk; ++i) R[i][k] = (float)mppi_host::spline_basis_at(kKnots, 1.0, k, (double)i / (nk - 1));
}

}  // namespace

namespace mppi_host {
mppi_status policy_infer(mppi_policy* p, const float* d_x, const float* d_cmd_origin, int nk, float sigma_max,
                         float* d_center, float* d_sd, hipStream_t st)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    float* feat = at<float>(p, p->o_feat);
    float* out = at<float>(p, p->o_out1);
    if ((s = phip(p, prop::launch_features(d_x, d_cmd_origin, feat, st), "features launch"))) return s;
    if ((s = forward(p, feat, nullptr, 1, out, false, st))) return s;
    HeadArgs h{};
    h.out = out;
    h.omean = at<float>(p, p->o_norm) + 80;
    h.ostd = at<float>(p, p->o_norm) + 152;
    h.nk = nk;
    resample_matrix(nk, h.R);
    h.log_lo = std::log(0.02f);
    h.log_hi = std::log(sigma_max);
    h.center = d_center;
    h.sd = d_sd;
    return phip(p, launch_head(h, st), "head launch");
}
const char* policy_error(const mppi_policy* p) { return p ? p->err.c_str() : g_perr.c_str(); }

// network output rows (B x 144) of raw feature rows (B x 40) on stream st
mppi_status policy_forward_rows(mppi_policy* p, const float* d_in, int B, float* d_out, hipStream_t st)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    if ((s = check_batch(p, B))) return s;
    return forward(p, d_in, nullptr, B, d_out, false, st);
}

const void* policy_workspace(const mppi_policy* p) { return p ? p->ws : nullptr; }

// device pointers of the output standardisation (mean and std of the 72 means)
mppi_status policy_out_norm(mppi_policy* p, const float** omean, const float** ostd)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    *omean = at<float>(p, p->o_norm) + 80;
    *ostd = at<float>(p, p->o_norm) + 152;
    return MPPI_OK;
}

// the head's resampling matrices for every knot count: rtab[nk][i][k], 9 x 8 x 6 floats
void policy_resample_table(float* rtab)
{
    std::memset(rtab, 0, sizeof(float) * 9 * 8 * kKnots);
    for (int nk = 2; nk <= 8; ++nk) resample_matrix(nk, reinterpret_cast<float(*)[kKnots]>(rtab + nk * 8 * kKnots));
}
}  // namespace mppi_host

extern "C" {

int mppi_policy_n_params(void)
{
    int n = 0;
    for (int l = 0; l < kLayers; ++l) n += kFi[l] * kFo[l] + kFo[l];
    return n;
}

mppi_status mppi_policy_create(const char* ckpt, uint64_t seed, int max_batch, mppi_policy** out)
{
    if (!out) return pfail(nullptr, MPPI_EINVAL, "null output");
    *out = nullptr;
    if (max_batch < 1 || max_batch > 65536) return pfail(nullptr, MPPI_EINVAL, "max_batch must be in [1, 65536]");
    mppi_policy* p = new (std::nothrow) mppi_policy();
    if (!p) return pfail(nullptr, MPPI_ENOMEM, "host allocation failed");
    int o = 0;
    for (int l = 0; l < kLayers; ++l) {
        p->geom.off[l] = o;
        p->geom.fi[l] = kFi[l];
        p->geom.fo[l] = kFo[l];
        p->geom.fip[l] = kFip[l];
        p->geom.fop[l] = kFop[l];
        o += kFi[l] * kFo[l] + kFo[l];
    }
    p->geom.off[kLayers] = o;
    p->max_batch = max_batch;
    p->bp_max = pad64(max_batch);
    p->hP.assign(o, 0.f);
    p->hm.assign(o, 0.f);
    p->hv.assign(o, 0.f);
    for (int i = 0; i < 40; ++i) p->norm[i] = 0.f, p->norm[40 + i] = 1.f;
    for (int i = 0; i < 72; ++i) p->norm[80 + i] = 0.f, p->norm[152 + i] = 1.f;
    if (!ckpt) {
        uint64_t st = seed;
        for (int l = 0; l < kLayers; ++l) {
            const double bound = 1.0 / std::sqrt((double)kFi[l]);
            const int nl = kFi[l] * kFo[l] + kFo[l];
            for (int i = 0; i < nl; ++i) {
                const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
                p->hP[p->geom.off[l] + i] = (float)((2.0 * u - 1.0) * bound);
            }
        }
    } else {
        FILE* f = std::fopen(ckpt, "rb");
        if (!f) {
            delete p;
            return pfail(nullptr, MPPI_EINVAL, std::string("cannot open checkpoint ") + ckpt);
        }
        char magic[8];
        int32_t hdr[2];
        bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "MPPIPOL1", 8) == 0 &&
                  std::fread(hdr, 4, 2, f) == 2 && hdr[0] == o && hdr[1] >= 0 &&
                  std::fread(p->norm, 4, 224, f) == 224 && std::fread(p->hP.data(), 4, o, f) == (size_t)o &&
                  std::fread(p->hm.data(), 4, o, f) == (size_t)o && std::fread(p->hv.data(), 4, o, f) == (size_t)o;
        std::fclose(f);
        if (!ok) {
            delete p;
            return pfail(nullptr, MPPI_EINVAL, std::string("malformed checkpoint ") + ckpt);
        }
        p->steps = hdr[1];
    }
    layout(p);
    *out = p;
    return MPPI_OK;
}

void mppi_policy_destroy(mppi_policy* p) { delete p; }

size_t mppi_policy_workspace_bytes(const mppi_policy* p) { return p ? p->total : 0; }

mppi_status mppi_policy_bind(mppi_policy* p, void* ws, size_t bytes, void* stream)
{
    if (!p || !ws) return pfail(p, MPPI_EINVAL, "null policy or workspace");
    if (((uintptr_t)ws & 255) != 0) return pfail(p, MPPI_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < p->total) return pfail(p, MPPI_ENOMEM, "workspace smaller than mppi_policy_workspace_bytes()");
    p->ws = ws;
    p->ws_bytes = bytes;
    p->stream = (hipStream_t)stream;
    hipStream_t st = p->stream;
    const size_t n = p->hP.size();
    mppi_status s;
    if ((s = phip(p, hipMemcpyAsync(at<float>(p, p->o_P), p->hP.data(), 4 * n, hipMemcpyHostToDevice, st),
                  "upload parameters")) ||
        (s = phip(p, hipMemcpyAsync(at<float>(p, p->o_m), p->hm.data(), 4 * n, hipMemcpyHostToDevice, st),
                  "upload moments")) ||
        (s = phip(p, hipMemcpyAsync(at<float>(p, p->o_v), p->hv.data(), 4 * n, hipMemcpyHostToDevice, st),
                  "upload moments")) ||
        (s = phip(p, hipMemcpyAsync(at<float>(p, p->o_norm), p->norm, 4 * 224, hipMemcpyHostToDevice, st),
                  "upload normalisation")) ||
        (s = phip(p, hipMemsetAsync(at<char>(p, p->shadow_begin), 0, p->shadow_end - p->shadow_begin, st),
                  "clear shadows")))
        return s;
    if ((s = refresh_shadows(p, st))) return s;
    return phip(p, hipStreamSynchronize(st), "bind synchronise");
}

mppi_status mppi_policy_set_normalization(mppi_policy* p, const float* in_mean, const float* in_std,
                                          const float* out_mean, const float* out_std)
{
    if (!p || !in_mean || !in_std || !out_mean || !out_std) return pfail(p, MPPI_EINVAL, "null argument");
    for (int i = 0; i < 40; ++i)
        if (!(in_std[i] > 0.f) || !std::isfinite(in_std[i]) || !std::isfinite(in_mean[i]))
            return pfail(p, MPPI_EINVAL, "input std must be finite and > 0");
    for (int i = 0; i < 72; ++i)
        if (!(out_std[i] > 0.f) || !std::isfinite(out_std[i]) || !std::isfinite(out_mean[i]))
            return pfail(p, MPPI_EINVAL, "output std must be finite and > 0");
    std::memcpy(p->norm, in_mean, 160);
    std::memcpy(p->norm + 40, in_std, 160);
    std::memcpy(p->norm + 80, out_mean, 288);
    std::memcpy(p->norm + 152, out_std, 288);
    if (!p->ws) return MPPI_OK;
    mppi_status s = phip(p, hipMemcpyAsync(at<float>(p, p->o_norm), p->norm, 4 * 224, hipMemcpyHostToDevice,
                                           p->stream), "upload normalisation");
    if (s) return s;
    return phip(p, hipStreamSynchronize(p->stream), "normalisation synchronise");
}

mppi_status mppi_policy_get_normalization(const mppi_policy* p, float* in_mean, float* in_std, float* out_mean,
                                          float* out_std)
{
    if (!p) return pfail(nullptr, MPPI_EINVAL, "null policy");
    if (in_mean) std::memcpy(in_mean, p->norm, 160);
    if (in_std) std::memcpy(in_std, p->norm + 40, 160);
    if (out_mean) std::memcpy(out_mean, p->norm + 80, 288);
    if (out_std) std::memcpy(out_std, p->norm + 152, 288);
    return MPPI_OK;
}

mppi_status mppi_policy_get_params(mppi_policy* p, float* d_params)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    if (!d_params) return pfail(p, MPPI_EINVAL, "null output");
    return phip(p, hipMemcpyAsync(d_params, at<float>(p, p->o_P), 4 * p->hP.size(), hipMemcpyDeviceToDevice,
                                  p->stream), "copy parameters");
}

mppi_status mppi_policy_set_params(mppi_policy* p, const float* d_params)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    if (!d_params) return pfail(p, MPPI_EINVAL, "null input");
    if ((s = phip(p, hipMemcpyAsync(at<float>(p, p->o_P), d_params, 4 * p->hP.size(), hipMemcpyDeviceToDevice,
                                    p->stream), "copy parameters")))
        return s;
    return refresh_shadows(p, p->stream);
}

mppi_status mppi_policy_forward(mppi_policy* p, const float* d_in, int B, float* d_out)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    if (!d_in || !d_out) return pfail(p, MPPI_EINVAL, "null input or output");
    if ((s = check_batch(p, B))) return s;
    return forward(p, d_in, nullptr, B, d_out, false, p->stream);
}

mppi_status mppi_policy_grad(mppi_policy* p, const float* d_in, const float* d_target, const int* d_index, int B,
                             float* d_grad, float* d_loss)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    if (!d_in || !d_target) return pfail(p, MPPI_EINVAL, "null input or target");
    if ((s = check_batch(p, B))) return s;
    return grad(p, d_in, d_target, d_index, B, d_grad ? d_grad : at<float>(p, p->o_G), d_loss, p->stream);
}

mppi_status mppi_policy_nll(mppi_policy* p, const float* d_in, const float* d_target, const int* d_index, int B,
                            float* d_loss)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    if (!d_in || !d_target || !d_loss) return pfail(p, MPPI_EINVAL, "null input, target or loss");
    if ((s = check_batch(p, B))) return s;
    const int bp = pad64(B);
    float* out = at<float>(p, p->o_out);
    if ((s = forward(p, d_in, d_index, B, out, false, p->stream))) return s;
    const float* nrm = at<float>(p, p->o_norm);
    // the loss kernel of a gradient step; its error outputs are scratch here
    LossArgs la{out, d_target, d_index, B, bp, nrm + 80, nrm + 152, at<__bf16>(p, p->o_dZ[0]),
                at<__bf16>(p, p->o_dZt[0]), at<float>(p, p->o_bpart[kLayers - 1]), at<float>(p, p->o_lpart)};
    if ((s = phip(p, launch_loss(la, p->stream), "loss launch"))) return s;
    return phip(p, launch_loss_sum(at<float>(p, p->o_lpart), bp / loss_rows_per_block(),
                                   (float)(1.0 / ((double)B * 72.0)), d_loss, p->stream),
                "loss sum launch");
}

mppi_status mppi_policy_pairs(int n_rec, int steps, int n_knots, const float* d_records, const float* d_origin_cmd,
                              float fall_z, float* d_feat, float* d_target, int* d_count, void* hip_stream)
{
    if (n_rec < 1 || steps < 1) return pfail(nullptr, MPPI_EINVAL, "n_rec and steps must be >= 1");
    if (n_knots < 2 || n_knots > 8) return pfail(nullptr, MPPI_EINVAL, "n_knots must be in [2, 8]");
    if (!d_records || !d_origin_cmd || !d_feat || !d_target || !d_count)
        return pfail(nullptr, MPPI_EINVAL, "null buffer");
    if (!std::isfinite(fall_z)) return pfail(nullptr, MPPI_EINVAL, "fall_z must be finite");
    PairsArgs a{};
    a.rec = d_records;
    a.oc = d_origin_cmd;
    a.n_rec = n_rec;
    a.steps = steps;
    a.nk = n_knots;
    a.fall_z = fall_z;
    // knot i of 6 at fraction i / 5 of the horizon from the not-a-knot spline through the
    // record's knots (the identity for 6 knots)
    for (int i = 0; i < kKnots; ++i)
        for (int k = 0; k < n_knots; ++k)
            a.R[i][k] = n_knots == kKnots ? (i == k ? 1.f : 0.f)
                                          : (float)mppi_host::spline_basis_at(n_knots, 1.0, k, i / (kKnots - 1.0));
    a.feat = d_feat;
    a.tgt = d_target;
    a.count = d_count;
    return phip(nullptr, launch_pairs(a, (hipStream_t)hip_stream), "pairs launch");
}

mppi_status mppi_policy_adam(mppi_policy* p, const float* d_grad, float lr)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    if (!d_grad) return pfail(p, MPPI_EINVAL, "null gradient");
    if (!(lr >= 0.f) || !std::isfinite(lr)) return pfail(p, MPPI_EINVAL, "learning rate must be finite and >= 0");
    return adam(p, d_grad, lr, p->stream);
}

mppi_status mppi_policy_train_step(mppi_policy* p, const float* d_in, const float* d_target, const int* d_index,
                                   int B, float lr, float* d_loss)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    if (!d_in || !d_target) return pfail(p, MPPI_EINVAL, "null input or target");
    if ((s = check_batch(p, B))) return s;
    if (!(lr >= 0.f) || !std::isfinite(lr)) return pfail(p, MPPI_EINVAL, "learning rate must be finite and >= 0");
    ReduceArgs ra;
    if ((s = backward(p, d_in, d_target, d_index, B, ra, p->stream))) return s;
    ra.loss = d_loss;
    if ((s = phip(p, launch_reduce_adam(ra, adam_args(p, nullptr, lr), p->stream), "reduce-adam launch"))) return s;
    p->steps += 1;
    return MPPI_OK;
}

int mppi_policy_steps(const mppi_policy* p) { return p ? p->steps : 0; }

mppi_status mppi_policy_save(mppi_policy* p, const char* path)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    if (!path) return pfail(p, MPPI_EINVAL, "null path");
    const size_t n = p->hP.size();
    std::vector<float> P(n), m(n), v(n);
    if ((s = phip(p, hipStreamSynchronize(p->stream), "synchronise")) ||
        (s = phip(p, hipMemcpy(P.data(), at<float>(p, p->o_P), 4 * n, hipMemcpyDeviceToHost), "read parameters")) ||
        (s = phip(p, hipMemcpy(m.data(), at<float>(p, p->o_m), 4 * n, hipMemcpyDeviceToHost), "read moments")) ||
        (s = phip(p, hipMemcpy(v.data(), at<float>(p, p->o_v), 4 * n, hipMemcpyDeviceToHost), "read moments")))
        return s;
    FILE* f = std::fopen(path, "wb");
    if (!f) return pfail(p, MPPI_EINVAL, std::string("cannot write ") + path);
    const int32_t hdr[2] = {(int32_t)n, (int32_t)p->steps};
    bool ok = std::fwrite("MPPIPOL1", 1, 8, f) == 8 && std::fwrite(hdr, 4, 2, f) == 2 &&
              std::fwrite(p->norm, 4, 224, f) == 224 && std::fwrite(P.data(), 4, n, f) == n &&
              std::fwrite(m.data(), 4, n, f) == n && std::fwrite(v.data(), 4, n, f) == n;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? MPPI_OK : pfail(p, MPPI_EINVAL, std::string("write failed: ") + path);
}

mppi_status mppi_policy_head(mppi_policy* p, const float* d_out, int nk, float sigma_max, float* d_center,
                             float* d_sd)
{
    mppi_status s;
    if ((s = need_bound(p))) return s;
    if (!d_out || !d_center || !d_sd) return pfail(p, MPPI_EINVAL, "null argument");
    if (nk < 2 || nk > 8) return pfail(p, MPPI_EINVAL, "n_knots must be in [2, 8]");
    if (!(sigma_max > 0.f) || !std::isfinite(sigma_max)) return pfail(p, MPPI_EINVAL, "sigma_max must be > 0");
    HeadArgs h{};
    h.out = d_out;
    h.omean = at<float>(p, p->o_norm) + 80;
    h.ostd = at<float>(p, p->o_norm) + 152;
    h.nk = nk;
    resample_matrix(nk, h.R);
    h.log_lo = std::log(0.02f);
    h.log_hi = std::log(sigma_max);
    h.center = d_center;
    h.sd = d_sd;
    return phip(p, launch_head(h, p->stream), "head launch");
}

const char* mppi_policy_last_error(const mppi_policy* p) { return mppi_host::policy_error(p); }

}  // extern "C"
