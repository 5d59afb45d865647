// C ABI of the whole-body MPPI library: validation, workspace layout, spline matrices,
// and kernel launches on the caller's stream.  No device allocation happens here: the
// caller provides the workspace.
#include "mppi.h"
#include "mppi_policy.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mppi_device.h"
#include "mppi_launch.h"
#include "policy_internal.h"
#include "proposal_launch.h"
#include "tracking_launch.h"

// MPPI_LANES_DEFAULT picks the lane-split rollout where its LDS fits
constexpr bool kSplitByDefault = true;

struct mppi_model {
    mppi_model_desc desc;
    std::vector<float> hf;
    mppi::DevModelF dev_f;
    mppi::DevModelD dev_d;
    int nx;
};

struct mppi_ctx {
    mppi_model model;     // private copy
    mppi_params p;
    std::vector<double> B;
    std::vector<float> S;
    int D;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    size_t off_B, off_S, off_hf, off_mu, off_eps, off_costs, off_w, off_status, total;
    // learned proposal: command and origin, centre, std, proposal costs and noise
    size_t off_cmd, off_center, off_sd, off_costs_p, off_eps_p;
    size_t off_eps_pair, off_costs_pair;  // the concurrent gated step's two sets in one launch
    uint32_t step = 0;
    mppi_policy* policy = nullptr;
    int k_prop = 0, prop_gate = 0;
    float cmd_origin[8] = {};
    // the gated proposal step runs the proposal rollout on `side` beside the plain
    // rollout on the bound stream (fork and join through the two events); the counters of
    // accepted and all proposal steps are device ints (off_pstats)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    size_t off_pstats = 0;
    size_t off_gate = 0;  // gate costs (2 floats) and the skip flag of the fallback rollout
    // Eq. 3 / Eq. 4 tracking cost (p.cost == MPPI_COST_TRACKING): parameters and the
    // trajectory region the cost kernel reads
    track::TrackDev track{};
    bool track_set = false;
    size_t off_traj = 0, off_uref = 0;
    bool split = false;  // rollouts on the lane-split kernel (16 lanes per sample)
    std::string err;
};

namespace {

thread_local std::string g_err;

mppi_status fail(mppi_ctx* c, mppi_status s, const std::string& msg)
{
    if (c) c->err = msg;
    g_err = msg;
    return s;
}

mppi_status hip_check(mppi_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return MPPI_OK;
    return fail(c, MPPI_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool finite_pos(float v) { return std::isfinite(v) && v > 0.f; }

// Not-a-knot cubic spline through nk evenly spaced knots on [0, T], written in terms of
// the second derivatives m_i at the knots (uniform spacing h):
//   interior:   m_{i-1} + 4 m_i + m_{i+1} = 6 (y_{i-1} - 2 y_i + y_{i+1}) / h^2
//   not-a-knot: equal third derivatives on both sides of the second and the
//               second-to-last knot (m_0 - 2 m_1 + m_2 = 0, and mirrored);
// three knots give the interpolating parabola (constant m), two the line (m = 0).
void second_derivatives(int n, double h, const double* y, double* m)
{
    if (n == 2) {
        m[0] = m[1] = 0.0;
        return;
    }
    std::vector<double> A((size_t)n * n, 0.0), r(n, 0.0);
    auto at = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    if (n == 3) {
        at(0, 0) = 1; at(0, 1) = -1;
        at(1, 0) = 1; at(1, 1) = 4; at(1, 2) = 1;
        r[1] = 6.0 * (y[0] - 2 * y[1] + y[2]) / (h * h);
        at(2, 1) = 1; at(2, 2) = -1;
    } else {
        at(0, 0) = 1; at(0, 1) = -2; at(0, 2) = 1;
        for (int i = 1; i < n - 1; ++i) {
            at(i, i - 1) = 1; at(i, i) = 4; at(i, i + 1) = 1;
            r[i] = 6.0 * (y[i - 1] - 2 * y[i] + y[i + 1]) / (h * h);
        }
        at(n - 1, n - 3) = 1; at(n - 1, n - 2) = -2; at(n - 1, n - 1) = 1;
    }
    for (int c = 0; c < n; ++c) {  // Gaussian elimination, partial pivoting
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (std::fabs(at(i, c)) > std::fabs(at(piv, c))) piv = i;
        if (piv != c) {
            for (int j = 0; j < n; ++j) std::swap(at(c, j), at(piv, j));
            std::swap(r[c], r[piv]);
        }
        for (int i = c + 1; i < n; ++i) {
            const double f = at(i, c) / at(c, c);
            for (int j = c; j < n; ++j) at(i, j) -= f * at(c, j);
            r[i] -= f * r[c];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = r[i];
        for (int j = i + 1; j < n; ++j) s -= at(i, j) * m[j];
        m[i] = s / at(i, i);
    }
}

double spline_value(int n, double h, const double* y, const double* m, double t)
{
    int s = (int)std::floor(t / h);
    if (s < 0) s = 0;
    if (s > n - 2) s = n - 2;
    const double tau = t - s * h, u = h - tau;
    return m[s] * u * u * u / (6 * h) + m[s + 1] * tau * tau * tau / (6 * h) + (y[s] / h - m[s] * h / 6) * u +
           (y[s + 1] / h - m[s + 1] * h / 6) * tau;
}

// weight of knot j in the lower-order interpolants at time t (knot spacing h); the
// zeroth-order hold switches to a knot at its time, taken to within 1e-9 of an interval
// so that k dt landing on a knot time holds that knot whatever the rounding of k dt / h
double low_order_weight(int basis, int nk, double h, int j, double t)
{
    if (basis == MPPI_BASIS_ZERO) {
        const int s = (int)std::floor(t / h + 1e-9);
        return std::min(std::max(s, 0), nk - 1) == j ? 1.0 : 0.0;
    }
    int s = (int)std::floor(t / h);
    s = std::min(std::max(s, 0), nk - 2);
    const double a = (t - s * h) / h;
    return j == s ? 1.0 - a : j == s + 1 ? a : 0.0;
}

// B[k][j]: weight of knot j in the joint target of step k; S[i][j]: weight of old knot j
// in new knot i (the interpolant one step later, held at the horizon end)
void build_spline(int nk, int H, double dt, int basis, std::vector<double>& B, std::vector<float>& S)
{
    const double T = H * dt, h = T / (nk - 1);
    B.assign((size_t)H * nk, 0.0);
    S.assign((size_t)nk * nk, 0.f);
    if (basis == MPPI_BASIS_DIRECT) {  // nk == H: identity, one-step advance with the last value held
        for (int k = 0; k < H; ++k) B[(size_t)k * nk + k] = 1.0;
        for (int i = 0; i < nk; ++i) S[(size_t)i * nk + std::min(i + 1, nk - 1)] = 1.f;
        return;
    }
    std::vector<double> y(nk), m(nk);
    for (int j = 0; j < nk; ++j) {
        std::fill(y.begin(), y.end(), 0.0);
        y[j] = 1.0;
        second_derivatives(nk, h, y.data(), m.data());
        auto value = [&](double t) {
            return basis == MPPI_BASIS_CUBIC ? spline_value(nk, h, y.data(), m.data(), t)
                                             : low_order_weight(basis, nk, h, j, t);
        };
        for (int k = 0; k < H; ++k) B[(size_t)k * nk + j] = value(k * dt);
        for (int i = 0; i < nk; ++i) S[(size_t)i * nk + j] = (float)value(std::min(i * h + dt, T));
    }
}

// device model constants; derived quantities computed in double from the FP32 inputs
template <typename R>
void fill_model(const mppi_model_desc& d, mppi::ModelT<R>& D)
{
    D = mppi::ModelT<R>{};
    const double sx = d.trunk_size[0], sy = d.trunk_size[1], sz = d.trunk_size[2], m0 = d.trunk_mass;
    D.tsx = (R)sx; D.tsy = (R)sy; D.tsz = (R)sz;
    D.m0 = (R)m0;
    D.I0x = (R)(m0 * (sy * sy + sz * sz) / 12.0);
    D.I0y = (R)(m0 * (sx * sx + sz * sz) / 12.0);
    D.I0z = (R)(m0 * (sx * sx + sy * sy) / 12.0);
    D.hip_x = (R)d.hip_x; D.hip_y = (R)d.hip_y;
    const double l1 = d.thigh_len, m1 = d.thigh_mass, l2 = d.calf_len, m2 = d.calf_mass;
    D.l1 = (R)l1; D.m1 = (R)m1; D.k1 = (R)(m1 * l1 * l1 / 12.0);
    D.l2 = (R)l2; D.m2 = (R)m2; D.k2 = (R)(m2 * l2 * l2 / 12.0);
    D.mtot = (R)(m0 + 4.0 * (m1 + m2));
    D.foot_r = (R)d.foot_r; D.g = (R)d.gravity;
    D.ck = (R)d.contact_k; D.cc = (R)d.contact_c; D.cmu = (R)d.friction_mu;
    D.inv_vs = (R)(1.0 / (double)d.slip_velocity);
    D.scene = d.scene;
    D.hf_nx = d.hf_nx; D.hf_ny = d.hf_ny;
    D.hf_inv_cell = d.scene == MPPI_SCENE_HEIGHTFIELD ? (R)(1.0 / (double)d.hf_cell) : R(0);
    D.hf_x0 = (R)d.hf_x0; D.hf_y0 = (R)d.hf_y0;
    D.sb_cx = (R)d.sbox_center[0]; D.sb_cy = (R)d.sbox_center[1]; D.sb_cz = (R)d.sbox_center[2];
    D.sb_hx = (R)d.sbox_half[0]; D.sb_hy = (R)d.sbox_half[1]; D.sb_hz = (R)d.sbox_half[2];
    const double bx = 2.0 * d.box_half[0], by = 2.0 * d.box_half[1], bz = 2.0 * d.box_half[2], bm = d.box_mass;
    D.bx_hx = (R)d.box_half[0]; D.bx_hy = (R)d.box_half[1]; D.bx_hz = (R)d.box_half[2]; D.bx_m = (R)bm;
    D.bx_Ix = (R)(bm * (by * by + bz * bz) / 12.0);
    D.bx_Iy = (R)(bm * (bx * bx + bz * bz) / 12.0);
    D.bx_Iz = (R)(bm * (bx * bx + by * by) / 12.0);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

mppi::DevParams dev_params(const mppi_ctx* c)
{
    mppi::DevParams P{};
    const mppi_params& p = c->p;
    P.K = p.K; P.H = p.H; P.nk = p.n_knots; P.nx = c->model.nx;
    P.dt = p.dt; P.sigma = p.sigma; P.inv_lambda = 1.0f / p.lambda; P.kp = p.kp; P.kd = p.kd;
    P.w_h = p.w_height; P.h_ref = p.h_ref; P.w_o = p.w_upright; P.w_v = p.w_vel; P.v_ref = p.v_ref;
    P.w_tau = p.w_torque; P.w_reach = p.w_reach; P.w_box = p.w_box; P.goal_x = p.goal[0]; P.goal_y = p.goal[1];
    P.seed_lo = (uint32_t)(p.seed & 0xffffffffu);
    P.seed_hi = (uint32_t)(p.seed >> 32);
    P.instance = p.instance;
    P.step = c->step;
    return P;
}

float* wsf(mppi_ctx* c, size_t off) { return (float*)((char*)c->ws + off); }

mppi_status need_bound(mppi_ctx* c)
{
    if (!c) return fail(nullptr, MPPI_EINVAL, "null context");
    if (!c->ws) return fail(c, MPPI_ESTATE, "no workspace bound (call mppi_bind)");
    return MPPI_OK;
}

// a start state the host can read (managed or mapped host memory) is checked on the host;
// device memory is checked by the lane-split rollout itself
mppi_status check_host_state(mppi_ctx* c, const float* x0)
{
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, x0) != hipSuccess) {
        (void)hipGetLastError();  // unknown to the runtime: leave the check to the device
        return MPPI_OK;
    }
    if (at.type != hipMemoryTypeHost && at.type != hipMemoryTypeManaged && !at.isManaged) return MPPI_OK;
    const float* hx = at.type == hipMemoryTypeHost && at.hostPointer ? (const float*)at.hostPointer : x0;
    if (at.type == hipMemoryTypeManaged || at.isManaged) {
        mppi_status s;
        if ((s = hip_check(c, hipStreamSynchronize(c->stream), "synchronise before reading the state"))) return s;
    }
    for (int i = 0; i < c->model.nx; ++i)
        if (!std::isfinite(hx[i])) return fail(c, MPPI_ENONFINITE_INPUT, "the start state is not finite");
    return MPPI_OK;
}

// the rollout launch of a controller: the lane-split or the quad kernel
hipError_t launch_roll(const mppi_ctx* c, const mppi::DevParams& P, const mppi::RolloutArgs& a, hipStream_t st)
{
    return c->split ? mppi::launch_rollout16(c->model.dev_f, c->model.dev_d, c->p.arith, P, a, st)
                    : mppi::launch_rollout(c->model.dev_f, c->model.dev_d, c->p.arith, P, a, st);
}

}  // namespace

namespace mppi_host {
bool model_info(const mppi_model* m, int* scene, int* nx, const float** hf, int* hf_cells, const void** dev_f,
                const void** dev_d)
{
    *scene = m->desc.scene;
    *nx = m->nx;
    *hf = m->hf.empty() ? nullptr : m->hf.data();
    *hf_cells = (int)m->hf.size();
    *dev_f = &m->dev_f;
    *dev_d = &m->dev_d;
    return true;
}
void spline_matrices(int nk, int H, double dt, int basis, std::vector<double>& B, std::vector<float>& S)
{
    build_spline(nk, H, dt, basis, B, S);
}
double spline_basis_at(int nk, double T, int k, double t)
{
    std::vector<double> y(nk, 0.0), m(nk);
    y[k] = 1.0;
    const double h = T / (nk - 1);
    second_derivatives(nk, h, y.data(), m.data());
    return spline_value(nk, h, y.data(), m.data(), t);
}
}  // namespace mppi_host

extern "C" {

const char* mppi_status_str(mppi_status s)
{
    switch (s) {
    case MPPI_OK: return "ok";
    case MPPI_WARN_ALL_NONFINITE: return "all samples non-finite; nominal kept";
    case MPPI_WARN_FALLBACK: return "the proposal step fell back to plain MPPI";
    case MPPI_WARN_NONFINITE_INPUT: return "start state not finite; nothing rolled out, nominal kept";
    case MPPI_ENONFINITE_INPUT: return "start state not finite";
    case MPPI_EINVAL: return "invalid argument";
    case MPPI_ENOMEM: return "workspace too small";
    case MPPI_EHIP: return "HIP runtime error";
    case MPPI_ESTATE: return "call out of order";
    case MPPI_EBUDGET: return "does not fit in the HBM budget";
    }
    return "unknown status";
}

const char* mppi_last_error(const mppi_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

mppi_status mppi_model_create(const mppi_model_desc* d, mppi_model** out)
{
    if (!d || !out) return fail(nullptr, MPPI_EINVAL, "null argument");
    *out = nullptr;
    const float pos[] = {d->trunk_size[0], d->trunk_size[1], d->trunk_size[2], d->trunk_mass, d->thigh_len,
                         d->thigh_mass,    d->calf_len,      d->calf_mass,     d->foot_r,     d->contact_k,
                         d->slip_velocity};
    for (float v : pos)
        if (!finite_pos(v)) return fail(nullptr, MPPI_EINVAL, "robot sizes, masses and contact constants must be > 0");
    if (!(d->contact_c >= 0.f) || !(d->friction_mu >= 0.f) || !std::isfinite(d->gravity))
        return fail(nullptr, MPPI_EINVAL, "contact damping and friction must be >= 0");
    if (d->scene < MPPI_SCENE_FLAT || d->scene > MPPI_SCENE_FREE_BOX)
        return fail(nullptr, MPPI_EINVAL, "unknown scene");
    if (d->scene == MPPI_SCENE_FREE_BOX) {
        for (int i = 0; i < 3; ++i)
            if (!finite_pos(d->box_half[i])) return fail(nullptr, MPPI_EINVAL, "free box needs positive half sizes");
        if (!finite_pos(d->box_mass)) return fail(nullptr, MPPI_EINVAL, "free box needs a positive mass");
    }
    if (d->scene == MPPI_SCENE_STATIC_BOX) {
        for (int i = 0; i < 3; ++i)
            if (!finite_pos(d->sbox_half[i]) || !std::isfinite(d->sbox_center[i]))
                return fail(nullptr, MPPI_EINVAL, "static box needs finite centre and positive half sizes");
    }
    mppi_model* m = new (std::nothrow) mppi_model();
    if (!m) return fail(nullptr, MPPI_ENOMEM, "host allocation failed");
    m->desc = *d;
    m->desc.heightfield = nullptr;
    if (d->scene == MPPI_SCENE_HEIGHTFIELD) {
        const long cells = (long)d->hf_nx * d->hf_ny;
        if (!d->heightfield || d->hf_nx < 2 || d->hf_ny < 2 || cells > MPPI_MAX_HEIGHTFIELD || !finite_pos(d->hf_cell)) {
            delete m;
            return fail(nullptr, MPPI_EINVAL, "heightfield needs 2 <= nx, ny, nx*ny <= 14336, cell > 0, data");
        }
        m->hf.assign(d->heightfield, d->heightfield + cells);
        for (float v : m->hf)
            if (!std::isfinite(v)) {
                delete m;
                return fail(nullptr, MPPI_EINVAL, "heightfield has non-finite heights");
            }
    }
    fill_model(*d, m->dev_f);
    fill_model(*d, m->dev_d);
    m->nx = d->scene == MPPI_SCENE_FREE_BOX ? 50 : 37;
    *out = m;
    return MPPI_OK;
}

void mppi_model_destroy(mppi_model* m) { delete m; }

int mppi_model_nx(const mppi_model* m) { return m ? m->nx : 0; }

mppi_status mppi_create(const mppi_model* model, const mppi_params* p, mppi_ctx** out)
{
    if (!model || !p || !out) return fail(nullptr, MPPI_EINVAL, "null argument");
    *out = nullptr;
    if (p->K < 1) return fail(nullptr, MPPI_EINVAL, "K must be >= 1");
    if (p->H < 1 || p->H > MPPI_MAX_HORIZON) return fail(nullptr, MPPI_EINVAL, "H must be in [1, 256]");
    if (p->basis == MPPI_BASIS_DIRECT) {
        if (p->n_knots != p->H) return fail(nullptr, MPPI_EINVAL, "MPPI_BASIS_DIRECT needs n_knots == H");
        if (p->lanes == MPPI_LANES_QUAD || p->cost != MPPI_COST_RUNNING)
            return fail(nullptr, MPPI_EINVAL, "MPPI_BASIS_DIRECT needs the lane-split rollout and the running cost");
    } else if (p->n_knots < 2 || p->n_knots > MPPI_MAX_KNOTS) {
        return fail(nullptr, MPPI_EINVAL, "n_knots must be in [2, 8]");
    }
    if (!finite_pos(p->dt)) return fail(nullptr, MPPI_EINVAL, "dt must be > 0");
    if (p->arith != MPPI_ARITH_FP64 && p->arith != MPPI_ARITH_FP32 && p->arith != MPPI_ARITH_MIXED)
        return fail(nullptr, MPPI_EINVAL, "arith must be MPPI_ARITH_FP64, _FP32 or _MIXED");
    if (!finite_pos(p->lambda)) return fail(nullptr, MPPI_EINVAL, "lambda must be > 0");
    if (!(p->sigma >= 0.f) || !std::isfinite(p->sigma)) return fail(nullptr, MPPI_EINVAL, "sigma must be >= 0");
    if (!std::isfinite(p->kp) || !std::isfinite(p->kd) || p->kd < 0.f)
        return fail(nullptr, MPPI_EINVAL, "kp must be finite, kd >= 0");
    if ((long)p->K * p->H > (1L << 31)) return fail(nullptr, MPPI_EINVAL, "K * H too large");
    if (p->basis < MPPI_BASIS_CUBIC || p->basis > MPPI_BASIS_DIRECT)
        return fail(nullptr, MPPI_EINVAL, "basis must be MPPI_BASIS_CUBIC, _LINEAR, _ZERO or _DIRECT");
    if (p->cost != MPPI_COST_RUNNING && p->cost != MPPI_COST_TRACKING)
        return fail(nullptr, MPPI_EINVAL, "cost must be MPPI_COST_RUNNING or MPPI_COST_TRACKING");
    if (p->lanes != MPPI_LANES_DEFAULT && p->lanes != MPPI_LANES_QUAD && p->lanes != MPPI_LANES_SPLIT)
        return fail(nullptr, MPPI_EINVAL, "lanes must be MPPI_LANES_DEFAULT, _QUAD or _SPLIT");
    const bool split_fits = mppi::rollout16_fits(p->arith, model->desc.scene, (int)model->hf.size());
    if (p->lanes == MPPI_LANES_SPLIT && !split_fits)
        return fail(nullptr, MPPI_EINVAL, "the lane-split rollout's LDS does not fit this heightfield");
    mppi_ctx* c = new (std::nothrow) mppi_ctx();
    if (!c) return fail(nullptr, MPPI_ENOMEM, "host allocation failed");
    const bool needs_split = p->arith == MPPI_ARITH_MIXED || p->basis == MPPI_BASIS_DIRECT;
    if (needs_split && (p->lanes == MPPI_LANES_QUAD || !split_fits)) {
        delete c;
        return fail(nullptr, MPPI_EINVAL, "MPPI_ARITH_MIXED and MPPI_BASIS_DIRECT need the lane-split rollout");
    }
    c->split = p->lanes == MPPI_LANES_SPLIT ||
               (p->lanes == MPPI_LANES_DEFAULT && split_fits && (kSplitByDefault || needs_split));
    c->model = *model;
    c->p = *p;
    c->D = 12 * p->n_knots;
    build_spline(p->n_knots, p->H, p->dt, p->basis, c->B, c->S);
    size_t o = 0;
    c->off_B = o; o = align256(o + sizeof(double) * c->B.size());
    c->off_S = o; o = align256(o + sizeof(float) * c->S.size());
    c->off_hf = o; o = align256(o + sizeof(float) * c->model.hf.size());
    c->off_mu = o; o = align256(o + sizeof(float) * c->D);
    c->off_eps = o; o = align256(o + sizeof(float) * (size_t)c->D * p->K);
    c->off_costs = o; o = align256(o + sizeof(float) * p->K);
    c->off_w = o; o = align256(o + sizeof(float) * p->K);
    c->off_status = o; o = align256(o + sizeof(int) * 16);
    c->off_cmd = o; o = align256(o + sizeof(float) * 8);
    c->off_center = o; o = align256(o + sizeof(float) * c->D);
    c->off_sd = o; o = align256(o + sizeof(float) * c->D);
    c->off_costs_p = o; o = align256(o + sizeof(float) * p->K);
    c->off_eps_p = o; o = align256(o + sizeof(float) * (size_t)c->D * p->K);
    // both sample sets of the concurrent gated step (K plain, then k_prop <= K proposal
    // samples): offsets from the nominal and costs
    c->off_eps_pair = o; o = align256(o + sizeof(float) * (size_t)c->D * 2 * p->K);
    c->off_costs_pair = o; o = align256(o + sizeof(float) * 2 * p->K);
    c->off_pstats = o; o = align256(o + sizeof(int) * 2);
    c->off_gate = o; o = align256(o + sizeof(float) * 4);
    if (p->cost == MPPI_COST_TRACKING) {
        c->off_traj = o;
        o = align256(o + sizeof(float) * (size_t)p->K * (p->H + 1) * model->nx);
        c->off_uref = o;
        o = align256(o + track::tracking_table_bytes(p->H));
    }
    c->total = o;
    *out = c;
    return MPPI_OK;
}

static void release_side(mppi_ctx* c)
{
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->side) (void)hipStreamDestroy(c->side);
    c->ev_fork = c->ev_join = nullptr;
    c->side = nullptr;
}

void mppi_destroy(mppi_ctx* c)
{
    if (!c) return;
    if (c->side) (void)hipStreamSynchronize(c->side);
    release_side(c);
    delete c;
}

size_t mppi_workspace_bytes(const mppi_ctx* c) { return c ? c->total : 0; }

mppi_status mppi_get_basis(const mppi_ctx* c, double* B_out, float* S_out)
{
    if (!c) return fail(nullptr, MPPI_EINVAL, "null context");
    if (B_out) std::memcpy(B_out, c->B.data(), sizeof(double) * c->B.size());
    if (S_out) std::memcpy(S_out, c->S.data(), sizeof(float) * c->S.size());
    return MPPI_OK;
}

mppi_status mppi_bind(mppi_ctx* c, void* ws, size_t bytes, void* stream)
{
    if (!c || !ws) return fail(c, MPPI_EINVAL, "null context or workspace");
    if (((uintptr_t)ws & 255) != 0) return fail(c, MPPI_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < c->total) return fail(c, MPPI_ENOMEM, "workspace smaller than mppi_workspace_bytes()");
    c->ws = ws;
    c->ws_bytes = bytes;
    c->stream = (hipStream_t)stream;
    c->step = 0;
    hipStream_t st = c->stream;
    mppi_status s;
    if ((s = hip_check(c, hipMemcpyAsync(wsf(c, c->off_B), c->B.data(), sizeof(double) * c->B.size(),
                                         hipMemcpyHostToDevice, st), "upload spline basis")))
        return s;
    if ((s = hip_check(c, hipMemcpyAsync(wsf(c, c->off_S), c->S.data(), sizeof(float) * c->S.size(),
                                         hipMemcpyHostToDevice, st), "upload shift matrix")))
        return s;
    if (!c->model.hf.empty() &&
        (s = hip_check(c, hipMemcpyAsync(wsf(c, c->off_hf), c->model.hf.data(), sizeof(float) * c->model.hf.size(),
                                         hipMemcpyHostToDevice, st), "upload heightfield")))
        return s;
    if ((s = hip_check(c, hipMemsetAsync(wsf(c, c->off_mu), 0, sizeof(float) * c->D, st), "clear nominal"))) return s;
    if ((s = hip_check(c, hipMemsetAsync(wsf(c, c->off_status), 0, sizeof(int) * 16, st), "clear status"))) return s;
    if ((s = hip_check(c, hipMemsetAsync(wsf(c, c->off_pstats), 0, sizeof(int) * 2, st), "clear proposal counters")))
        return s;
    // the stream and events of the gated proposal step (default priority)
    release_side(c);
    if ((s = hip_check(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "create side stream")) ||
        (s = hip_check(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "create event")) ||
        (s = hip_check(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "create event"))) {
        release_side(c);
        return s;
    }
    return hip_check(c, hipStreamSynchronize(st), "bind synchronise");
}

mppi_status mppi_set_nominal(mppi_ctx* c, const float* d_knots)
{
    mppi_status s;
    if ((s = need_bound(c))) return s;
    if (!d_knots) return fail(c, MPPI_EINVAL, "null knots");
    return hip_check(c, hipMemcpyAsync(wsf(c, c->off_mu), d_knots, sizeof(float) * c->D, hipMemcpyDeviceToDevice,
                                       c->stream), "set nominal");
}

mppi_status mppi_get_nominal(mppi_ctx* c, float* d_knots)
{
    mppi_status s;
    if ((s = need_bound(c))) return s;
    if (!d_knots) return fail(c, MPPI_EINVAL, "null knots");
    return hip_check(c, hipMemcpyAsync(d_knots, wsf(c, c->off_mu), sizeof(float) * c->D, hipMemcpyDeviceToDevice,
                                       c->stream), "get nominal");
}

mppi_status mppi_set_step(mppi_ctx* c, uint32_t step)
{
    if (!c) return fail(nullptr, MPPI_EINVAL, "null context");
    c->step = step;
    return MPPI_OK;
}

uint32_t mppi_get_step(const mppi_ctx* c) { return c ? c->step : 0; }

mppi_status mppi_sample(mppi_ctx* c, float* d_eps, uint32_t* d_raw)
{
    mppi_status s;
    if ((s = need_bound(c))) return s;
    if (!d_eps && !d_raw) return fail(c, MPPI_EINVAL, "nothing to write");
    const mppi::DevParams P = dev_params(c);
    return hip_check(c, mppi::launch_sample(P, c->D, d_eps, d_raw, c->stream), "sample launch");
}

static mppi_status rollout(mppi_ctx* c, const float* d_x0, const float* d_eps, float* d_costs, float* d_traj,
                           const int* d_skip = nullptr)
{
    const bool tracking = c->p.cost == MPPI_COST_TRACKING;
    if (tracking && !c->track_set) return fail(c, MPPI_ESTATE, "tracking cost not set (call mppi_set_tracking_cost)");
    if (tracking && !d_traj) d_traj = wsf(c, c->off_traj);
    const mppi::DevParams P = dev_params(c);
    mppi::RolloutArgs a{};
    a.B = (const double*)wsf(c, c->off_B);
    a.hf = wsf(c, c->off_hf);
    a.mu = wsf(c, c->off_mu);
    a.x0 = d_x0;
    a.eps_in = d_eps;
    a.eps_sn = c->D;
    a.eps_sd = 1;
    a.eps_out = d_eps ? nullptr : wsf(c, c->off_eps);
    a.costs = d_costs;
    a.traj = d_traj;
    a.samples_per_block = 16;
    a.direct = c->p.basis == MPPI_BASIS_DIRECT;
    a.skip = d_skip;
    a.input_status = (int*)wsf(c, c->off_status) + 1;
    mppi_status s;
    if ((s = hip_check(c, launch_roll(c, P, a, c->stream),
                       "rollout launch")) ||
        !tracking)
        return s;
    // Eq. 3 / Eq. 4 on the trajectories just written (replaces the running cost)
    track::TrackArgs t{};
    t.c = c->track;
    t.traj = d_traj;
    t.B = a.B;
    t.mu = a.mu;
    if (d_eps) {
        t.eps = d_eps; t.eps_sn = c->D; t.eps_sd = 1;
    } else {
        t.eps = a.eps_out; t.eps_sn = 1; t.eps_sd = c->p.K;
    }
    t.sigma = c->p.sigma;
    t.K = c->p.K; t.H = c->p.H; t.nk = c->p.n_knots; t.nx = c->model.nx;
    t.dt = c->p.dt;
    t.step = c->step;
    t.costs = d_costs;
    const int track_arith = c->p.arith == MPPI_ARITH_FP64 ? MPPI_ARITH_FP64 : MPPI_ARITH_FP32;
    return hip_check(c, track::launch_tracking_cost(track_arith, t, d_x0, wsf(c, c->off_uref), c->stream),
                     "tracking cost launch");
}

mppi_status mppi_rollout_batch(mppi_ctx* c, const float* d_x0, const float* d_eps, float* d_costs, float* d_traj)
{
    mppi_status s;
    if ((s = need_bound(c))) return s;
    if (!d_x0 || !d_costs) return fail(c, MPPI_EINVAL, "null state or cost buffer");
    return rollout(c, d_x0, d_eps, d_costs, d_traj);
}

static mppi_status update(mppi_ctx* c, const float* d_costs, const float* d_eps, float* knots_out, float* nominal_out,
                          float* u0_out, float* weights_out)
{
    const mppi::DevParams P = dev_params(c);
    mppi::UpdateArgs a{};
    a.costs = d_costs;
    if (d_eps) {
        a.eps = d_eps; a.eps_sn = c->D; a.eps_sd = 1;
    } else {
        a.eps = wsf(c, c->off_eps); a.eps_sn = 1; a.eps_sd = c->p.K;
    }
    a.mu = wsf(c, c->off_mu);
    a.S = wsf(c, c->off_S);
    a.knots_out = knots_out;
    a.nominal_out = nominal_out;
    a.u0_out = u0_out;
    a.weights_out = weights_out;
    a.status = (int*)wsf(c, c->off_status);
    return hip_check(c, mppi::launch_update(P, a, c->stream), "update launch");
}

mppi_status mppi_update(mppi_ctx* c, const float* d_costs, const float* d_eps, float* d_knots_out,
                        float* d_weights_out)
{
    mppi_status s;
    if ((s = need_bound(c))) return s;
    if (!d_costs || !d_knots_out) return fail(c, MPPI_EINVAL, "null costs or output");
    return update(c, d_costs, d_eps, d_knots_out, nullptr, nullptr, d_weights_out);
}

// GATE_COST, GATE_NONE or GATE_BEST, the gated two with the CONCURRENT bit allowed
static bool valid_gate(int gate)
{
    const int g = gate & ~MPPI_PROPOSAL_CONCURRENT;
    if (g != MPPI_PROPOSAL_GATE_COST && g != MPPI_PROPOSAL_GATE_NONE && g != MPPI_PROPOSAL_GATE_BEST) return false;
    return !((gate & MPPI_PROPOSAL_CONCURRENT) && g == MPPI_PROPOSAL_GATE_NONE);
}

// Proposal step on the plain kernels: the k_prop samples theta_n = c + e_n are rolled out
// through the explicit-noise path with unit scale, where e holds Philox noise scaled by
// sd for n >= 2, zero for the centre (n = 0) and nominal - c for n = 1.  A gated step
// takes the proposal when its cost under the gate (the centre's, or the least of its
// samples other than the nominal) is finite and not above the nominal's, and falls back to
// a plain step with K samples around the nominal otherwise.  With the lane-split rollout
// the gate is decided on the device right after the proposal rollout and the plain
// rollout runs only on a fallback (it returns at once when the proposal was taken), so a
// step rolls out k_prop + K samples only when it falls back.  With the gate's
// MPPI_PROPOSAL_CONCURRENT bit one rollout launch, centred on the nominal, covers both
// sets on every step; with the quad rollout the plain rollout runs beside the proposal's
// on an internal stream; the gate kernel follows both.  The update kernel reads the gate
// costs and updates over whichever set was chosen; no host round trip.  Accepted:
// mu' = c + sum w_n e_n / sum w_n, the weighted mean of theta (centre c, unit scale).
// Ungated: the proposal rollout alone.
static mppi_status step_proposal(mppi_ctx* c, const float* d_x0, const float* d_center, const float* d_sd, int kp,
                                 int gate, float* d_u0_out)
{
    mppi_status s;
    mppi::DevParams Pp = dev_params(c);
    Pp.K = kp;
    Pp.sigma = 1.0f;
    float* e = wsf(c, c->off_eps_p);
    float* costs_p = wsf(c, c->off_costs_p);
    float* g = wsf(c, c->off_gate);
    int* skip = (int*)(g + 2);
    if ((s = hip_check(c, mppi::launch_sample(Pp, c->D, e, nullptr, c->stream), "proposal noise launch"))) return s;
    if ((s = hip_check(c, prop::launch_proposal_noise(kp, c->D, e, d_center, d_sd, wsf(c, c->off_mu), c->stream),
                       "proposal scale launch")))
        return s;
    mppi::RolloutArgs a{};
    a.B = (const double*)wsf(c, c->off_B);
    a.hf = wsf(c, c->off_hf);
    a.mu = d_center;
    a.x0 = d_x0;
    a.eps_in = e;
    a.eps_sn = c->D;
    a.eps_sd = 1;
    a.costs = costs_p;
    a.samples_per_block = 16;
    a.direct = c->p.basis == MPPI_BASIS_DIRECT;
    const bool concurrent = (gate & MPPI_PROPOSAL_CONCURRENT) != 0;
    gate &= ~MPPI_PROPOSAL_CONCURRENT;
    const bool gated = gate == MPPI_PROPOSAL_GATE_COST || gate == MPPI_PROPOSAL_GATE_BEST;
    const int best = gate == MPPI_PROPOSAL_GATE_BEST;
    float* costs = wsf(c, c->off_costs);
    if (gated && c->split && !concurrent) {
        // proposal rollout, the gate, then the plain rollout (skipped when the gate takes
        // the proposal), all on the bound stream
        if ((s = hip_check(c, launch_roll(c, Pp, a, c->stream), "proposal rollout launch")) ||
            (s = hip_check(c, prop::launch_gate(kp, costs_p, best, g, skip, c->stream), "gate launch")) ||
            (s = rollout(c, d_x0, nullptr, costs, nullptr, skip)))
            return s;
    } else if (gated && concurrent) {
        // one rollout launch over both sample sets, centred on the nominal mu with unit
        // scale: the plain step's K samples (mu + sigma eps, drawn from its counters), then
        // the proposal's kp as offsets (c - mu) + e_n; the gate reads the proposal's costs,
        // the update the plain ones on a fallback
        const mppi::DevParams P = dev_params(c);
        float* E = wsf(c, c->off_eps_pair);
        float* cpair = wsf(c, c->off_costs_pair);
        mppi::DevParams P2 = Pp;
        P2.K = c->p.K + kp;
        a.mu = wsf(c, c->off_mu);
        a.eps_in = E;
        a.costs = cpair;
        a.input_status = (int*)wsf(c, c->off_status) + 1;
        costs = cpair;
        costs_p = cpair + c->p.K;
        if ((s = hip_check(c, mppi::launch_sample(P, c->D, E, nullptr, c->stream), "plain noise launch")) ||
            (s = hip_check(c, prop::launch_pair_noise(kp, c->p.K, c->D, c->p.sigma, E, e, wsf(c, c->off_mu), d_center,
                                                      wsf(c, c->off_eps), c->stream),
                           "paired offsets launch")) ||
            (s = hip_check(c, launch_roll(c, P2, a, c->stream), "paired rollout launch")) ||
            (s = hip_check(c, prop::launch_gate(kp, costs_p, best, g, skip, c->stream), "gate launch")))
            return s;
    } else if (gated) {
        if (!c->side) return fail(c, MPPI_ESTATE, "no side stream (bind the controller again)");
        if ((s = hip_check(c, hipEventRecord(c->ev_fork, c->stream), "fork record")) ||
            (s = hip_check(c, hipStreamWaitEvent(c->side, c->ev_fork, 0), "fork wait")) ||
            (s = hip_check(c, launch_roll(c, Pp, a, c->side), "proposal rollout launch")) ||
            (s = hip_check(c, hipEventRecord(c->ev_join, c->side), "join record")))
            return s;
        mppi_status rs = rollout(c, d_x0, nullptr, costs, nullptr);
        // join before returning, also after a failed launch, so that no work is left on the side stream
        if ((s = hip_check(c, hipStreamWaitEvent(c->stream, c->ev_join, 0), "join wait"))) return s;
        if (rs) return rs;
        if ((s = hip_check(c, prop::launch_gate(kp, costs_p, best, g, skip, c->stream), "gate launch"))) return s;
    } else if ((s = hip_check(c, launch_roll(c, Pp, a, c->stream), "proposal rollout launch"))) {
        return s;
    }
    const mppi::DevParams P = dev_params(c);
    mppi::UpdateArgs u{};
    u.costs = costs;  // the plain step (read only when the gate rejects)
    u.eps = wsf(c, c->off_eps);
    u.eps_sn = 1;
    u.eps_sd = c->p.K;
    u.mu = wsf(c, c->off_mu);
    u.prop = 1;
    u.Kp = kp;
    u.gate = gated ? g : nullptr;
    u.costs_p = costs_p;
    u.eps_p = e;
    u.mu_p = d_center;
    u.pstats = (int*)wsf(c, c->off_pstats);
    u.S = wsf(c, c->off_S);
    u.nominal_out = wsf(c, c->off_mu);
    u.u0_out = d_u0_out;
    u.status = (int*)wsf(c, c->off_status);
    if ((s = hip_check(c, mppi::launch_update(P, u, c->stream), "proposal update launch"))) return s;
    c->step += 1;
    return MPPI_OK;
}

mppi_status mppi_step(mppi_ctx* c, const float* d_x0, float* d_u0_out)
{
    mppi_status s;
    if ((s = need_bound(c))) return s;
    if (!d_x0 || !d_u0_out) return fail(c, MPPI_EINVAL, "null state or control buffer");
    if ((s = check_host_state(c, d_x0))) return s;
    if (c->policy) {
        float* center = wsf(c, c->off_center);
        float* sd = wsf(c, c->off_sd);
        if ((s = mppi_host::policy_infer(c->policy, d_x0, wsf(c, c->off_cmd), c->p.n_knots, c->p.sigma, center, sd,
                                         c->stream)))
            return fail(c, s, std::string("proposal: ") + mppi_host::policy_error(c->policy));
        return step_proposal(c, d_x0, center, sd, c->k_prop, c->prop_gate, d_u0_out);
    }
    float* costs = wsf(c, c->off_costs);
    if ((s = rollout(c, d_x0, nullptr, costs, nullptr))) return s;
    if ((s = update(c, costs, nullptr, nullptr, wsf(c, c->off_mu), d_u0_out, nullptr))) return s;
    c->step += 1;
    return MPPI_OK;
}

mppi_status mppi_update_shift(mppi_ctx* c, const float* d_costs, float* d_u0_out, float* d_weights_out)
{
    mppi_status s;
    if ((s = need_bound(c))) return s;
    if (!d_costs || !d_u0_out) return fail(c, MPPI_EINVAL, "null costs or control buffer");
    if ((s = update(c, d_costs, nullptr, nullptr, wsf(c, c->off_mu), d_u0_out, d_weights_out))) return s;
    c->step += 1;
    return MPPI_OK;
}

}  // extern "C"

namespace mppi_host {
// One plain control step of an unbound controller with its whole workspace placed in the
// device region [region, region + bytes) (the library's static scratch): the spline
// matrices and heightfield are uploaded, the nominal is copied in from d_nominal, the
// step runs as mppi_step does, and the shifted nominal is copied back to d_nominal.  The
// controller is left unbound.  Nothing is allocated.  Nothing in the region has to start
// at zero: every buffer the step reads is written earlier in the same step (the status
// words too, which nothing reads on this path), so the previous call's contents do no harm.
mppi_status step_in_region(mppi_ctx* c, void* region, size_t bytes, const float* d_x0, float* d_nominal,
                           float* d_u0_out, hipStream_t st)
{
    if (!c) return fail(nullptr, MPPI_EINVAL, "null context");
    if (!region) return fail(c, MPPI_EHIP, "no device region for the step");
    if (!d_x0 || !d_nominal || !d_u0_out) return fail(c, MPPI_EINVAL, "null state, nominal or control buffer");
    if (c->ws) return fail(c, MPPI_ESTATE, "the controller has a bound workspace (use mppi_step)");
    if (c->policy || c->p.cost != MPPI_COST_RUNNING)
        return fail(c, MPPI_EINVAL, "the static step runs the plain method with the running cost");
    if (c->total > bytes)
        return fail(c, MPPI_EINVAL, "the controller's workspace (" + std::to_string(c->total) +
                                        " bytes) exceeds the static scratch (" + std::to_string(bytes) + " bytes)");
    c->ws = region;
    c->ws_bytes = bytes;
    c->stream = st;
    mppi_status s;
    float* mu = wsf(c, c->off_mu);
    float* costs = wsf(c, c->off_costs);
    if (!(s = hip_check(c, hipMemcpyAsync(wsf(c, c->off_B), c->B.data(), sizeof(double) * c->B.size(),
                                          hipMemcpyHostToDevice, st), "upload spline basis")) &&
        !(s = hip_check(c, hipMemcpyAsync(wsf(c, c->off_S), c->S.data(), sizeof(float) * c->S.size(),
                                          hipMemcpyHostToDevice, st), "upload shift matrix")) &&
        !(s = c->model.hf.empty() ? MPPI_OK
                                  : hip_check(c, hipMemcpyAsync(wsf(c, c->off_hf), c->model.hf.data(),
                                                                sizeof(float) * c->model.hf.size(),
                                                                hipMemcpyHostToDevice, st), "upload heightfield")) &&
        !(s = hip_check(c, hipMemcpyAsync(mu, d_nominal, sizeof(float) * c->D, hipMemcpyDeviceToDevice, st),
                        "copy nominal in")) &&
        !(s = rollout(c, d_x0, nullptr, costs, nullptr)) &&
        !(s = update(c, costs, nullptr, nullptr, mu, d_u0_out, nullptr)) &&
        !(s = hip_check(c, hipMemcpyAsync(d_nominal, mu, sizeof(float) * c->D, hipMemcpyDeviceToDevice, st),
                        "copy nominal out")))
        c->step += 1;
    c->ws = nullptr;
    c->ws_bytes = 0;
    c->stream = nullptr;
    return s;
}
}  // namespace mppi_host

extern "C" {

mppi_status mppi_set_tracking_cost(mppi_ctx* c, const mppi_tracking_cost* t)
{
    if (!c || !t) return fail(c, MPPI_EINVAL, "null argument");
    if (c->p.cost != MPPI_COST_TRACKING) return fail(c, MPPI_EINVAL, "controller created with the running cost");
    auto nonneg = [](float v) { return std::isfinite(v) && v >= 0.f; };
    for (float v : t->Q)
        if (!nonneg(v)) return fail(c, MPPI_EINVAL, "Q must be finite and >= 0");
    for (float v : t->R)
        if (!nonneg(v)) return fail(c, MPPI_EINVAL, "R must be finite and >= 0");
    const float fin[] = {t->p_ref0[0], t->p_ref0[1], t->p_ref0[2], t->v_cmd[0], t->v_cmd[1], t->raibert_gain,
                         t->box_goal[0], t->box_goal[1]};
    for (float v : fin)
        if (!std::isfinite(v)) return fail(c, MPPI_EINVAL, "references and gains must be finite");
    if (!finite_pos(t->period) || !(t->duty > 0.f && t->duty < 1.f))
        return fail(c, MPPI_EINVAL, "period must be > 0 and duty in (0, 1)");
    if (!finite_pos(t->stand_height) || !nonneg(t->swing_height) || !nonneg(t->box_weight))
        return fail(c, MPPI_EINVAL, "stand_height must be > 0, swing_height and box_weight >= 0");
    if ((t->gait != 0 && t->gait != 1) || t->reserved != 0)
        return fail(c, MPPI_EINVAL, "gait must be 0 (stand) or 1 (trot), reserved 0");
    track::TrackDev& g = c->track;
    std::memcpy(g.Q, t->Q, sizeof(g.Q));
    std::memcpy(g.R, t->R, sizeof(g.R));
    for (int i = 0; i < 3; ++i) g.p_ref0[i] = t->p_ref0[i];
    g.v_cmd[0] = t->v_cmd[0];
    g.v_cmd[1] = t->v_cmd[1];
    g.period = t->period;
    g.duty = t->duty;
    g.swing_h = t->swing_height;
    g.stand_h = t->stand_height;
    g.raibert_k = t->raibert_gain;
    g.box_w = t->box_weight;
    g.box_goal[0] = t->box_goal[0];
    g.box_goal[1] = t->box_goal[1];
    g.l1 = c->model.desc.thigh_len;
    g.l2 = c->model.desc.calf_len;
    g.gait = t->gait;
    g.box = c->model.nx == 50;
    c->track_set = true;
    return MPPI_OK;
}

mppi_status mppi_sync_status(mppi_ctx* c)
{
    mppi_status s;
    if ((s = need_bound(c))) return s;
    int st[3] = {0, 0, 0};  // all non-finite, non-finite start state, proposal fallback
    if ((s = hip_check(c, hipMemcpyAsync(st, wsf(c, c->off_status), sizeof(st), hipMemcpyDeviceToHost, c->stream),
                       "read status")))
        return s;
    if ((s = hip_check(c, hipStreamSynchronize(c->stream), "synchronise"))) return s;
    if (st[1]) return MPPI_WARN_NONFINITE_INPUT;
    if (st[0]) return MPPI_WARN_ALL_NONFINITE;
    return st[2] ? MPPI_WARN_FALLBACK : MPPI_OK;
}

mppi_status mppi_step_proposal(mppi_ctx* c, const float* d_x0, const float* d_center, const float* d_sd, int k_prop,
                               int gate, float* d_u0_out)
{
    mppi_status s;
    if ((s = need_bound(c))) return s;
    if (!d_x0 || !d_center || !d_sd || !d_u0_out) return fail(c, MPPI_EINVAL, "null argument");
    if (k_prop < 2 || k_prop > c->p.K) return fail(c, MPPI_EINVAL, "k_prop must be in [2, K]");
    if (!valid_gate(gate)) return fail(c, MPPI_EINVAL, "unknown gate");
    if (c->p.cost != MPPI_COST_RUNNING) return fail(c, MPPI_EINVAL, "the proposal step uses the running cost");
    return step_proposal(c, d_x0, d_center, d_sd, k_prop, gate, d_u0_out);
}

mppi_status mppi_set_proposal(mppi_ctx* c, mppi_policy* pol, int k_prop, int gate, const float* cmd,
                              const float* origin_xy)
{
    mppi_status s;
    if ((s = need_bound(c))) return s;
    if (!pol) {
        c->policy = nullptr;
        return MPPI_OK;
    }
    if (c->model.nx != 37) return fail(c, MPPI_EINVAL, "the proposal needs a 37-float state model");
    if (c->p.cost != MPPI_COST_RUNNING) return fail(c, MPPI_EINVAL, "the proposal step uses the running cost");
    if (k_prop < 2 || k_prop > c->p.K) return fail(c, MPPI_EINVAL, "k_prop must be in [2, K]");
    if (!cmd || !origin_xy) return fail(c, MPPI_EINVAL, "null command or origin");
    if (!valid_gate(gate)) return fail(c, MPPI_EINVAL, "unknown gate");
    if (!(c->p.sigma > 0.f)) return fail(c, MPPI_EINVAL, "the proposal needs sigma > 0 (upper std clamp)");
    for (int i = 0; i < 3; ++i) c->cmd_origin[i] = cmd[i];
    c->cmd_origin[3] = origin_xy[0];
    c->cmd_origin[4] = origin_xy[1];
    if ((s = hip_check(c, hipMemcpyAsync(wsf(c, c->off_cmd), c->cmd_origin, sizeof(float) * 8, hipMemcpyHostToDevice,
                                         c->stream), "upload command")) ||
        (s = hip_check(c, hipStreamSynchronize(c->stream), "synchronise")))
        return s;
    c->policy = pol;
    c->k_prop = k_prop;
    c->prop_gate = gate;
    return MPPI_OK;
}

mppi_status mppi_proposal_stats(mppi_ctx* c, int* accepted, int* steps)
{
    if (!c) return fail(nullptr, MPPI_EINVAL, "null context");
    int st[2] = {0, 0};
    if (c->ws) {
        mppi_status s;
        if ((s = hip_check(c, hipMemcpyAsync(st, wsf(c, c->off_pstats), sizeof(st), hipMemcpyDeviceToHost, c->stream),
                           "read proposal counters")) ||
            (s = hip_check(c, hipStreamSynchronize(c->stream), "synchronise")))
            return s;
    }
    if (accepted) *accepted = st[0];
    if (steps) *steps = st[1];
    return MPPI_OK;
}

mppi_status mppi_sim_step(const mppi_model* m, int arith, int n, const float* d_x, const float* d_u, float kp,
                          float kd, float dt, float* d_x_out, float* d_tau_out, const float* d_hf, void* stream)
{
    if (arith != MPPI_ARITH_FP64 && arith != MPPI_ARITH_FP32 && arith != MPPI_ARITH_MIXED)
        return fail(nullptr, MPPI_EINVAL, "bad arith");
    if (arith == MPPI_ARITH_MIXED) arith = MPPI_ARITH_FP64;  // the plant step has no mixed variant
    if (!m || n < 0 || !d_x || !d_u || !d_x_out) return fail(nullptr, MPPI_EINVAL, "null argument or n < 0");
    if (!finite_pos(dt) || !std::isfinite(kp) || !(kd >= 0.f)) return fail(nullptr, MPPI_EINVAL, "bad dt/kp/kd");
    if (m->desc.scene == MPPI_SCENE_HEIGHTFIELD && !d_hf) return fail(nullptr, MPPI_EINVAL, "heightfield scene needs d_hf");
    if (n == 0) return MPPI_OK;
    return hip_check(nullptr,
                     mppi::launch_sim_step(m->dev_f, m->dev_d, arith, n, m->nx, d_x, d_u, kp, kd, dt, d_x_out,
                                           d_tau_out, d_hf, (hipStream_t)stream),
                     "sim step launch");
}

}  // extern "C"
