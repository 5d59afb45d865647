// Device-code check: the library's host code and its rollout, sampling, update, plant,
// proposal-noise and tracking-cost kernels, built for the CPU against the emulated
// device model (hip/hip_runtime.h, emu.cpp), run under the sanitizers on the launch
// sequences of the GPU tests: full control steps on flat ground, the heightfield and
// the free-box scene, rollouts with caller noise and trajectories, the proposal step
// (explicit centre and spread), the tracking cost and batched serving in both launch
// modes (per-scene kernels, one kernel for every scene).  Every result is compared with the
// FP64 oracle (knots and controls within 1e-3, 10-step costs within 1e-4 relative), so a
// kernel that reads undefined memory or races on LDS also shows up as a wrong value.
// Prints one line per case and "failures: N"; the exit status is 0 only when N is 0.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "mppi.h"
#include "mppi_policy.h"
extern "C" {
#include "mppi_oracle.h"
}

static int g_fail = 0;

static void check(const char* what, double err, double tol)
{
    const bool ok = std::isfinite(err) && err <= tol;
    std::printf("  %-58s max error %.3e (bar %.0e) %s\n", what, err, tol, ok ? "ok" : "FAIL");
    if (!ok) ++g_fail;
}

static void must(const char* what, mppi_status s)
{
    if (s < 0) {
        std::printf("  %s: status %d (%s)\n", what, (int)s, mppi_last_error(nullptr));
        std::exit(2);
    }
}

static std::vector<void*> g_mem;
static float* dev(size_t n)
{
    void* p = std::aligned_alloc(256, (4 * n + 255) / 256 * 256);
    g_mem.push_back(p);
    return static_cast<float*>(p);
}

// robot and scenes of the synthetic workloads (FP32 values on both sides)
static const float kTrunk[3] = {0.38f, 0.094f, 0.114f};
// the static box of scene 2: centre and half extents (set per case)
static float g_sbox[6] = {0.71f, 0.f, 0.15f, 0.5f, 0.5f, 0.15f};

static void fill(int scene, mppi_model_desc& d, orc_model& o, std::vector<float>& hf, std::vector<double>& hfd)
{
    d = mppi_model_desc{};
    d.trunk_size[0] = kTrunk[0]; d.trunk_size[1] = kTrunk[1]; d.trunk_size[2] = kTrunk[2];
    d.trunk_mass = 5.2f; d.hip_x = 0.188f; d.hip_y = 0.047f; d.thigh_len = 0.213f; d.thigh_mass = 1.0f;
    d.calf_len = 0.213f; d.calf_mass = 0.2f; d.foot_r = 0.02f; d.gravity = 9.81f; d.contact_k = 2e4f;
    d.contact_c = 500.f; d.friction_mu = 0.8f; d.slip_velocity = 0.01f; d.scene = scene;
    if (scene == MPPI_SCENE_HEIGHTFIELD) {
        d.hf_nx = d.hf_ny = 16; d.hf_cell = 0.2f; d.hf_x0 = d.hf_y0 = -1.5f;
        hf.resize(256);
        for (int i = 0; i < 256; ++i) hf[i] = 0.015f * std::sin(0.7f * (i % 16)) * std::cos(0.45f * (i / 16));
        d.heightfield = hf.data();
    }
    if (scene == MPPI_SCENE_FREE_BOX) {
        d.box_half[0] = d.box_half[1] = 0.2f; d.box_half[2] = 0.15f; d.box_mass = 2.f;
    }
    if (scene == MPPI_SCENE_STATIC_BOX)
        for (int i = 0; i < 3; ++i) {
            d.sbox_center[i] = g_sbox[i];
            d.sbox_half[i] = g_sbox[3 + i];
        }
    o = orc_model{};
    for (int i = 0; i < 3; ++i) o.trunk_size[i] = d.trunk_size[i];
    o.trunk_mass = d.trunk_mass; o.hip_x = d.hip_x; o.hip_y = d.hip_y; o.thigh_len = d.thigh_len;
    o.thigh_mass = d.thigh_mass; o.calf_len = d.calf_len; o.calf_mass = d.calf_mass; o.foot_r = d.foot_r;
    o.gravity = d.gravity; o.k = d.contact_k; o.c = d.contact_c; o.mu = d.friction_mu; o.vs = d.slip_velocity;
    o.scene = scene;
    if (scene == MPPI_SCENE_HEIGHTFIELD) {
        hfd.assign(hf.begin(), hf.end());
        o.hf_nx = d.hf_nx; o.hf_ny = d.hf_ny; o.hf_cell = d.hf_cell; o.hf_x0 = d.hf_x0; o.hf_y0 = d.hf_y0;
        o.hf = hfd.data();
    }
    for (int i = 0; i < 3; ++i) o.box_half[i] = d.box_half[i];
    o.box_mass = d.box_mass;
    for (int i = 0; i < 3; ++i) {
        o.sbox_center[i] = d.sbox_center[i];
        o.sbox_half[i] = d.sbox_half[i];
    }
}

static int g_lanes = MPPI_LANES_QUAD;  // rollout decomposition of the controllers made here
static int g_basis = 0;  // knot interpolation of the controllers made here

static void params(int K, int H, int nk, float dt, mppi_params& p, orc_params& o)
{
    p = mppi_params{};
    p.lanes = g_lanes;
    p.basis = g_basis;
    p.K = K; p.H = H; p.n_knots = nk; p.dt = dt; p.sigma = 0.3f; p.lambda = 0.1f; p.kp = 40.f; p.kd = 1.f;
    p.w_height = 100.f; p.h_ref = 0.27f; p.w_upright = 10.f; p.w_vel = 1.f; p.v_ref = 0.5f; p.w_torque = 1e-3f;
    p.w_reach = 1.f; p.w_box = 2.f; p.goal[0] = 2.0f; p.goal[1] = -0.5f; p.seed = 0x1234abcdull; p.instance = 3;
    o = orc_params{};
    o.K = K; o.H = H; o.nk = nk; o.dt = p.dt; o.sigma = p.sigma; o.lambda = p.lambda; o.kp = p.kp; o.kd = p.kd;
    o.w_h = p.w_height; o.h_ref = p.h_ref; o.w_o = p.w_upright; o.w_v = p.w_vel; o.v_ref = p.v_ref;
    o.w_tau = p.w_torque; o.w_reach = p.w_reach; o.w_box = p.w_box; o.goal[0] = p.goal[0]; o.goal[1] = p.goal[1];
    o.seed = p.seed; o.instance = p.instance;
    o.basis = p.basis;
}

// standing pose with small deterministic joint offsets (and the box 1 m ahead)
// free box at box_x ahead (1 m: away from the feet; 0.4 m: against the front feet)
static std::vector<float> start_state(int nx, int seed, float box_x = 1.f)
{
    std::vector<float> x(nx, 0.f);
    x[2] = 0.2835f; x[3] = 1.f;
    uint32_t r = 2654435761u * (uint32_t)(seed + 1);
    for (int l = 0; l < 4; ++l) {
        const float q[3] = {0.f, 0.9f, -1.8f};
        for (int j = 0; j < 3; ++j) {
            r = r * 1664525u + 1013904223u;
            x[7 + 3 * l + j] = q[j] + 0.05f * ((float)(r >> 8) / 16777216.f * 2.f - 1.f);
        }
    }
    if (nx == 50) {
        x[37] = box_x; x[39] = 0.15f - 2.f * 9.81f / 8e4f; x[40] = 1.f;
    }
    return x;
}

static std::vector<float> stance_knots(int nk, int seed)
{
    std::vector<float> mu(12 * nk);
    uint32_t r = 97u * (uint32_t)(seed + 3);
    for (int j = 0; j < 12; ++j)
        for (int i = 0; i < nk; ++i) {
            r = r * 1664525u + 1013904223u;
            const float q[3] = {0.f, 0.9f, -1.8f};
            mu[j * nk + i] = q[j % 3] + 0.05f * ((float)(r >> 8) / 16777216.f * 2.f - 1.f);
        }
    return mu;
}

static std::vector<double> to_d(const float* p, size_t n) { return std::vector<double>(p, p + n); }

static double max_abs_diff(const float* a, const double* b, size_t n)
{
    double m = 0;
    for (size_t i = 0; i < n; ++i) m = std::fmax(m, std::fabs((double)a[i] - b[i]));
    return m;
}

static mppi_ctx* controller(mppi_model* m, const mppi_params& p)
{
    mppi_ctx* c = nullptr;
    must("create", mppi_create(m, &p, &c));
    const size_t n = mppi_workspace_bytes(c);
    must("bind", mppi_bind(c, dev(n / 4 + 64), n, nullptr));
    return c;
}

// full control steps against the oracle's Algorithm 1 (the Philox path without a
// trajectory buffer, where the faulted builds of the rollout kernel stopped)
static void steps_case(const char* name, int scene, int K, int H, int nk, float dt, int steps)
{
    mppi_model_desc d; orc_model o; std::vector<float> hf; std::vector<double> hfd;
    fill(scene, d, o, hf, hfd);
    mppi_model* m = nullptr;
    must("model", mppi_model_create(&d, &m));
    mppi_params p; orc_params op;
    params(K, H, nk, dt, p, op);
    mppi_ctx* c = controller(m, p);
    const int nx = mppi_model_nx(m), D = 12 * nk;
    float *x = dev(nx), *u0 = dev(12), *mu = dev(D);
    for (int s = 0; s < steps; ++s) {
        std::vector<float> xs = start_state(nx, s), ms = stance_knots(nk, s);
        std::memcpy(x, xs.data(), 4 * nx);
        std::memcpy(mu, ms.data(), 4 * D);
        must("set nominal", mppi_set_nominal(c, mu));
        must("set step", mppi_set_step(c, (uint32_t)s));
        must("step", mppi_step(c, x, u0));
        must("status", mppi_sync_status(c));
        must("get nominal", mppi_get_nominal(c, mu));
        std::vector<double> ox = to_d(xs.data(), nx), omu = to_d(ms.data(), D), ou0(12);
        orc_mppi_step(&o, &op, (uint32_t)s, ox.data(), omu.data(), ou0.data(), nullptr, 1);
        char what[128];
        std::snprintf(what, sizeof what, "%s step %d: first control and nominal", name, s);
        check(what, std::fmax(max_abs_diff(u0, ou0.data(), 12), max_abs_diff(mu, omu.data(), D)), 1e-3);
    }
    mppi_destroy(c);
    mppi_model_destroy(m);
}

// 10-step rollouts with caller noise and trajectories, and with Philox noise and
// trajectories, against the oracle's rollouts
static void rollout_case(int scene, int K, int nk, float box_x = 1.f)
{
    mppi_model_desc d; orc_model o; std::vector<float> hf; std::vector<double> hfd;
    fill(scene, d, o, hf, hfd);
    mppi_model* m = nullptr;
    must("model", mppi_model_create(&d, &m));
    mppi_params p; orc_params op;
    params(K, 10, nk, 0.01f, p, op);
    mppi_ctx* c = controller(m, p);
    const int nx = mppi_model_nx(m), D = 12 * nk;
    float *x = dev(nx), *mu = dev(D), *eps = dev((size_t)K * D), *costs = dev(K), *traj = dev((size_t)K * 11 * nx);
    std::vector<float> xs = start_state(nx, 7, box_x), ms = stance_knots(nk, 7);
    std::memcpy(x, xs.data(), 4 * nx);
    std::memcpy(mu, ms.data(), 4 * D);
    must("set nominal", mppi_set_nominal(c, mu));
    uint32_t r = 12345;
    for (size_t i = 0; i < (size_t)K * D; ++i) {
        r = r * 1664525u + 1013904223u;
        eps[i] = 1.5f * ((float)(r >> 8) / 16777216.f * 2.f - 1.f);
    }
    std::vector<double> ox = to_d(xs.data(), nx), omu = to_d(ms.data(), D), oe = to_d(eps, (size_t)K * D), oc(K);
    for (int pass = 0; pass < 2; ++pass) {
        const bool given = pass == 0;
        must("rollout", mppi_rollout_batch(c, x, given ? eps : nullptr, costs, traj));
        if (!given) orc_sample_eps(&op, 0, oe.data());
        orc_rollout_batch(&o, &op, ox.data(), omu.data(), oe.data(), oc.data(), nullptr, 1);
        double e = 0;
        for (int n = 0; n < K; ++n) e = std::fmax(e, std::fabs(costs[n] - oc[n]) / std::fabs(oc[n]));
        char what[128];
        std::snprintf(what, sizeof what, "scene %d rollout%s, %s noise, 10-step costs", scene,
                      box_x < 0.5f ? " (feet on the box)" : "", given ? "caller" : "Philox");
        check(what, e, 1e-4);
    }
    mppi_destroy(c);
    mppi_model_destroy(m);
}

// the proposal step with an explicit centre and spread (each gate, with and without the
// concurrent flag, and ungated); quick: the falling-back inputs only, and of the gates
// the cost gate, no gate, and the best-sample gate with the flag
static void proposal_case(bool quick)
{
    mppi_model_desc d; orc_model o; std::vector<float> hf; std::vector<double> hfd;
    fill(MPPI_SCENE_FLAT, d, o, hf, hfd);
    mppi_model* m = nullptr;
    must("model", mppi_model_create(&d, &m));
    mppi_params p; orc_params op;
    params(24, 8, 4, 0.02f, p, op);
    mppi_ctx* c = controller(m, p);
    const int D = 48, Kp = 8;
    float *x = dev(37), *u0 = dev(12), *mu = dev(D), *center = dev(D), *sd = dev(D);
    for (int bad_nominal = 0; bad_nominal < (quick ? 1 : 2); ++bad_nominal)
    for (int gate : {(int)MPPI_PROPOSAL_GATE_COST, (int)MPPI_PROPOSAL_GATE_NONE, (int)MPPI_PROPOSAL_GATE_BEST,
                     MPPI_PROPOSAL_GATE_COST | MPPI_PROPOSAL_CONCURRENT,
                     MPPI_PROPOSAL_GATE_BEST | MPPI_PROPOSAL_CONCURRENT}) {
        if (quick && (gate == MPPI_PROPOSAL_GATE_BEST || gate == (MPPI_PROPOSAL_GATE_COST | MPPI_PROPOSAL_CONCURRENT)))
            continue;
        std::vector<float> xs = start_state(37, 5), ms = stance_knots(4, 5), cs = stance_knots(4, 6);
        if (bad_nominal)  // a nominal far off the stance, so that the gates take the proposal
            for (float& v : ms) v += 0.5f;
        std::memcpy(x, xs.data(), 4 * 37);
        std::memcpy(mu, ms.data(), 4 * D);
        std::memcpy(center, cs.data(), 4 * D);
        for (int i = 0; i < D; ++i) sd[i] = 0.05f + 0.002f * i;
        must("set nominal", mppi_set_nominal(c, mu));
        must("set step", mppi_set_step(c, 5));
        must("proposal step", mppi_step_proposal(c, x, center, sd, Kp, gate, u0));
        must("get nominal", mppi_get_nominal(c, mu));
        std::vector<double> ox = to_d(xs.data(), 37), omu = to_d(ms.data(), D), oc = to_d(cs.data(), D),
                            osd = to_d(sd, D), ou0(12);
        int acc = 0;
        orc_mppi_step_proposal(&o, &op, 5, ox.data(), omu.data(), oc.data(), osd.data(), Kp,
                               gate & ~MPPI_PROPOSAL_CONCURRENT, ou0.data(), nullptr, nullptr, &acc, 1);
        char what[128];
        std::snprintf(what, sizeof what, "proposal step (gate %d, oracle %s)", gate, acc ? "accepted" : "fell back");
        check(what, std::fmax(max_abs_diff(u0, ou0.data(), 12), max_abs_diff(mu, omu.data(), D)), 1e-3);
    }
    mppi_destroy(c);
    mppi_model_destroy(m);
}

// a control step with the Eq. 3 / Eq. 4 tracking cost
static void tracking_case(int scene)
{
    mppi_model_desc d; orc_model o; std::vector<float> hf; std::vector<double> hfd;
    fill(scene, d, o, hf, hfd);
    mppi_model* m = nullptr;
    must("model", mppi_model_create(&d, &m));
    mppi_params p; orc_params op;
    params(32, 20, 6, 0.01f, p, op);
    p.cost = MPPI_COST_TRACKING;
    mppi_ctx* c = controller(m, p);
    mppi_tracking_cost t{};
    orc_tracking ot{};
    const float Q[36] = {1, 1, 100, 10, 10, 1, 0.1f, 0.1f, 0.1f, 0.1f, 0.1f, 0.1f, 0.1f, 0.1f, 0.1f, 0.1f, 0.1f, 0.1f,
                         1, 1, 0.1f, 0.1f, 0.1f, 0.1f, 1e-3f, 1e-3f, 1e-3f, 1e-3f, 1e-3f, 1e-3f, 1e-3f, 1e-3f, 1e-3f,
                         1e-3f, 1e-3f, 1e-3f};
    for (int i = 0; i < 36; ++i) ot.Q[i] = t.Q[i] = Q[i];
    for (int j = 0; j < 12; ++j) ot.R[j] = t.R[j] = 0.5f;
    t.p_ref0[2] = 0.27f; t.v_cmd[0] = 0.5f; t.period = 0.4f; t.duty = 0.5f; t.swing_height = 0.08f;
    t.stand_height = 0.25f; t.raibert_gain = 0.1f; t.gait = 1;
    t.box_weight = scene == MPPI_SCENE_FREE_BOX ? 10.f : 0.f; t.box_goal[0] = 2.f; t.box_goal[1] = -0.5f;
    ot.p_ref0[2] = t.p_ref0[2]; ot.v_cmd[0] = t.v_cmd[0]; ot.period = t.period; ot.duty = t.duty;
    ot.swing_height = t.swing_height; ot.stand_height = t.stand_height; ot.raibert_k = t.raibert_gain;
    ot.box_w = t.box_weight; ot.box_goal[0] = t.box_goal[0]; ot.box_goal[1] = t.box_goal[1]; ot.gait = 1;
    must("tracking cost", mppi_set_tracking_cost(c, &t));
    const int nx = mppi_model_nx(m), D = 72;
    float *x = dev(nx), *u0 = dev(12), *mu = dev(D);
    std::vector<float> xs = start_state(nx, 2), ms = stance_knots(6, 2);
    xs[19] = 0.2f;
    std::memcpy(x, xs.data(), 4 * nx);
    std::memcpy(mu, ms.data(), 4 * D);
    must("set nominal", mppi_set_nominal(c, mu));
    must("set step", mppi_set_step(c, 9));
    must("step", mppi_step(c, x, u0));
    must("get nominal", mppi_get_nominal(c, mu));
    std::vector<double> ox = to_d(xs.data(), nx), omu = to_d(ms.data(), D), ou0(12);
    orc_mppi_step_tracking(&o, &op, &ot, 9, ox.data(), omu.data(), ou0.data(), nullptr, 1);
    char what[128];
    std::snprintf(what, sizeof what, "scene %d tracking-cost step", scene);
    check(what, std::fmax(max_abs_diff(u0, ou0.data(), 12), max_abs_diff(mu, omu.data(), D)), 1e-3);
    mppi_destroy(c);
    mppi_model_destroy(m);
}

// batched serving: three instances (flat ground, heightfield, free box; ragged tiles)
// stepped twice by the per-scene persistent kernels and by the single kernel over every
// scene's tiles.  The first step's controls match the oracle's control step; states,
// controls, nominals, running costs and counters of the two launch modes agree bit for bit.
static void batch_case()
{
    struct Spec { int scene, K, H, nk; float dt; };
    const Spec sp[3] = {{MPPI_SCENE_FLAT, 20, 8, 4, 0.02f},
                        {MPPI_SCENE_HEIGHTFIELD, 18, 6, 6, 0.01f},
                        {MPPI_SCENE_FREE_BOX, 17, 6, 8, 0.01f}};
    mppi_model_desc d[3]; orc_model o[3]; std::vector<float> hf[3]; std::vector<double> hfd[3];
    mppi_model* m[3];
    for (int i = 0; i < 3; ++i) {
        fill(sp[i].scene, d[i], o[i], hf[i], hfd[i]);
        must("model", mppi_model_create(&d[i], &m[i]));
    }
    std::vector<float> out[2];
    for (int mode = 0; mode < 2; ++mode) {
        mppi_batch* b = nullptr;
        must("batch create", mppi_batch_create(4, 16, 256, 0, &b));
        const size_t bytes = mppi_batch_control_bytes(4, 0) + (8u << 20);
        must("batch bind", mppi_batch_bind(b, dev(bytes / 4 + 64), bytes, nullptr));
        must("launch mode", mppi_batch_set_launch_mode(b, mode));
        int ids[3];
        mppi_params p[3]; orc_params op[3];
        std::vector<float> xs[3], ms[3];
        for (int i = 0; i < 3; ++i) {
            int slot = -1;
            must("add model", mppi_batch_add_model(b, m[i], &slot));
            params(sp[i].K, sp[i].H, sp[i].nk, sp[i].dt, p[i], op[i]);
            p[i].instance = op[i].instance = 5 + i;
            xs[i] = start_state(mppi_model_nx(m[i]), i);
            ms[i] = stance_knots(sp[i].nk, i);
            must("admit", mppi_batch_admit(b, slot, &p[i], xs[i].data(), ms[i].data(), &ids[i]));
        }
        for (int s = 0; s < 2; ++s) {
            must("batch step", mppi_batch_step(b));
            for (int i = 0; i < 3 && s == 0; ++i) {
                const int nx = mppi_model_nx(m[i]), D = 12 * sp[i].nk;
                std::vector<float> u0(12);
                must("batch read", mppi_batch_read(b, ids[i], nullptr, u0.data(), nullptr, nullptr, nullptr));
                std::vector<double> ox = to_d(xs[i].data(), nx), omu = to_d(ms[i].data(), D), ou0(12);
                orc_mppi_step(&o[i], &op[i], 0, ox.data(), omu.data(), ou0.data(), nullptr, 1);
                char what[128];
                std::snprintf(what, sizeof what, "batch (launch mode %d) scene %d first step: first control", mode,
                              sp[i].scene);
                check(what, max_abs_diff(u0.data(), ou0.data(), 12), 1e-3);
            }
        }
        for (int i = 0; i < 3; ++i) {
            const int nx = mppi_model_nx(m[i]), D = 12 * sp[i].nk;
            std::vector<float> x(nx), u0(12), mu(D);
            float acc = 0.f;
            uint32_t step = 0;
            must("batch read", mppi_batch_read(b, ids[i], x.data(), u0.data(), mu.data(), &acc, &step));
            if (step != 2) ++g_fail;
            out[mode].insert(out[mode].end(), x.begin(), x.end());
            out[mode].insert(out[mode].end(), u0.begin(), u0.end());
            out[mode].insert(out[mode].end(), mu.begin(), mu.end());
            out[mode].push_back(acc);
        }
        mppi_batch_destroy(b);
    }
    double diff = out[0].size() == out[1].size() ? 0.0 : INFINITY;
    for (size_t k = 0; k < out[0].size() && k < out[1].size(); ++k)
        diff = std::fmax(diff, std::memcmp(&out[0][k], &out[1][k], 4) ? std::fabs(out[0][k] - out[1][k]) + 1e-30 : 0.0);
    check("batch: single launch against per-scene kernels, 2 steps", diff, 0.0);
    for (int i = 0; i < 3; ++i) mppi_model_destroy(m[i]);
}

int main(int argc, char** argv)
{
    const bool quick = argc > 1 && std::strcmp(argv[1], "quick") == 0;
    // "no-batch": the batch runtime's first-fit allocator keeps a std::map, whose tree
    // rebalancing runs inside the (uninstrumented) C++ library, so MemorySanitizer would
    // report the tree's own links as uninitialised
    const bool no_batch = argc > 2 && std::strcmp(argv[2], "no-batch") == 0;
    steps_case("flat K=64 H=25", MPPI_SCENE_FLAT, 64, 25, 4, 0.02f, quick ? 1 : 3);
    rollout_case(MPPI_SCENE_FLAT, 20, 4);
    proposal_case(quick);
    if (!quick) {
        steps_case("heightfield K=16 H=12", MPPI_SCENE_HEIGHTFIELD, 16, 12, 6, 0.01f, 1);
        steps_case("free box K=16 H=10", MPPI_SCENE_FREE_BOX, 16, 10, 8, 0.01f, 1);
        rollout_case(MPPI_SCENE_FREE_BOX, 8, 8);
        tracking_case(MPPI_SCENE_FLAT);
        tracking_case(MPPI_SCENE_FREE_BOX);
    }
    // the same controller checks on the lane-split rollout (16 lanes per sample)
    g_lanes = MPPI_LANES_SPLIT;
    steps_case("split flat K=64 H=25", MPPI_SCENE_FLAT, 64, 25, 4, 0.02f, 1);
    rollout_case(MPPI_SCENE_FLAT, 21, 4);
    rollout_case(MPPI_SCENE_FREE_BOX, 9, 8);  // the contact passes read only what the tests wrote
    rollout_case(MPPI_SCENE_FREE_BOX, 9, 8, 0.4f);  // front feet on the ground and against the box
    proposal_case(quick);  // gated: the proposal and the fallback in one launch, or one after the other
    if (!quick) {
        // the static box: front feet against its face, then on its top
        rollout_case(MPPI_SCENE_STATIC_BOX, 9, 6);
        g_sbox[0] = 0.6f; g_sbox[2] = -0.13f;
        rollout_case(MPPI_SCENE_STATIC_BOX, 9, 6);
        g_sbox[0] = 0.71f; g_sbox[2] = 0.15f;
        steps_case("split heightfield K=16 H=12", MPPI_SCENE_HEIGHTFIELD, 16, 12, 6, 0.01f, 1);
        steps_case("split free box K=18 H=10", MPPI_SCENE_FREE_BOX, 18, 10, 8, 0.01f, 1);
    }
    // direct per-step sampling (one value per step, drawn in the step loop)
    g_basis = MPPI_BASIS_DIRECT;
    steps_case("split direct flat K=21 H=12", MPPI_SCENE_FLAT, 21, 12, 12, 0.02f, 1);
    g_basis = 0;
    g_lanes = MPPI_LANES_QUAD;
    if (!no_batch) batch_case();
    for (void* p : g_mem) std::free(p);
    std::printf("failures: %d\n", g_fail);
    return g_fail ? 1 : 0;
}
