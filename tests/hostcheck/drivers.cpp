// Host range check: the library's host code (controller, batch runtime, policy runtime)
// is built for the CPU against the stand-in runtime and launchers, and driven through
// the C ABI over buffers registered as device memory.  Every copy, fill and kernel launch
// the host code issues is checked against those buffers (launchers.cpp).  Prints the
// number of out-of-range accesses; the exit status is 0 only when there are none.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mppi.h"
#include "mppi_policy.h"

void range_register(const void* p, size_t bytes);
extern int g_bad, g_batch_tiles, g_prop_rows;

static std::vector<void*> g_alloc;
static void* dev(size_t n)
{
    void* p = std::aligned_alloc(256, (n + 255) / 256 * 256);
    range_register(p, n);
    g_alloc.push_back(p);
    return p;
}
static float* devf(size_t n) { return static_cast<float*>(dev(4 * n)); }

static int expect(const char* what, mppi_status s, bool ok)
{
    if ((s >= 0) != ok) {
        std::printf("  UNEXPECTED STATUS %s: %d\n", what, (int)s);
        ++g_bad;
    }
    return s;
}
#define OK(call) expect(#call, (call), true)
#define REFUSED(call) expect(#call, (call), false)

static mppi_model_desc robot(int scene)
{
    mppi_model_desc d{};
    d.trunk_size[0] = 0.38f; d.trunk_size[1] = 0.094f; d.trunk_size[2] = 0.114f; d.trunk_mass = 5.2f;
    d.hip_x = 0.188f; d.hip_y = 0.047f; d.thigh_len = 0.213f; d.thigh_mass = 1.0f; d.calf_len = 0.213f;
    d.calf_mass = 0.2f; d.foot_r = 0.02f; d.gravity = 9.81f; d.contact_k = 2e4f; d.contact_c = 500.f;
    d.friction_mu = 0.8f; d.slip_velocity = 0.01f;
    d.scene = scene;
    d.box_half[0] = d.box_half[1] = 0.2f; d.box_half[2] = 0.15f; d.box_mass = 2.f;
    d.sbox_center[0] = 1.1f; d.sbox_center[2] = 0.15f;
    d.sbox_half[0] = d.sbox_half[1] = 0.5f; d.sbox_half[2] = 0.15f;
    return d;
}

static mppi_params params(int K, int H, int nk, int basis = 0, int arith = 0, int cost = MPPI_COST_RUNNING)
{
    mppi_params p{};
    p.K = K; p.H = H; p.n_knots = nk; p.dt = 0.02f; p.sigma = 0.3f; p.lambda = 0.1f; p.kp = 40; p.kd = 1;
    p.basis = basis; p.arith = arith; p.cost = cost;
    return p;
}

// a controller with the Eq. 3 / Eq. 4 tracking cost: rollouts with and without caller
// noise and trajectories, full steps, and the calls it refuses
static void tracking(mppi_model* m, mppi_policy* pol, int nx, int K, int H, int nk, int arith)
{
    mppi_params p = params(K, H, nk, 0, arith, MPPI_COST_TRACKING);
    mppi_ctx* c = nullptr;
    if (OK(mppi_create(m, &p, &c)) < 0) return;
    const size_t n = mppi_workspace_bytes(c);
    OK(mppi_bind(c, dev(n), n, nullptr));
    const int D = 12 * nk;
    float *x = devf(nx), *u0 = devf(12), *costs = devf(K), *eps = devf((size_t)K * D);
    float *traj = devf((size_t)K * (H + 1) * nx), *center = devf(D), *sd = devf(D);
    REFUSED(mppi_rollout_batch(c, x, nullptr, costs, nullptr));  // parameters not set yet
    mppi_tracking_cost t{};
    for (float& q : t.Q) q = 1.f;
    for (float& r : t.R) r = 0.5f;
    t.period = 0.5f; t.duty = 0.5f; t.swing_height = 0.08f; t.stand_height = 0.25f; t.gait = 1;
    t.box_weight = nx == 50 ? 2.f : 0.f;
    mppi_tracking_cost bad = t;
    bad.duty = 1.f;
    REFUSED(mppi_set_tracking_cost(c, &bad));
    bad = t;
    bad.reserved = 1;
    REFUSED(mppi_set_tracking_cost(c, &bad));
    OK(mppi_set_tracking_cost(c, &t));
    OK(mppi_rollout_batch(c, x, nullptr, costs, nullptr));
    OK(mppi_rollout_batch(c, x, eps, costs, traj));
    OK(mppi_rollout_batch(c, x, nullptr, costs, traj));
    OK(mppi_step(c, x, u0));
    OK(mppi_update_shift(c, costs, u0, nullptr));
    if (K >= 2) REFUSED(mppi_step_proposal(c, x, center, sd, 2, MPPI_PROPOSAL_GATE_NONE, u0));
    const float cmd[3] = {0.5f, 0, 0}, org[2] = {0, 0};
    if (nx == 37) REFUSED(mppi_set_proposal(c, pol, 2, MPPI_PROPOSAL_GATE_NONE, cmd, org));
    OK(mppi_sync_status(c));
    mppi_destroy(c);
    // a running-cost controller refuses tracking parameters
    mppi_params q = params(K, H, nk);
    if (OK(mppi_create(m, &q, &c)) < 0) return;
    REFUSED(mppi_set_tracking_cost(c, &t));
    mppi_destroy(c);
}

static void controller(mppi_model* m, mppi_policy* pol, int nx, int K, int H, int nk, int basis)
{
    mppi_params p = params(K, H, nk, basis);
    mppi_ctx* c = nullptr;
    if (OK(mppi_create(m, &p, &c)) < 0) return;
    const size_t n = mppi_workspace_bytes(c);
    OK(mppi_bind(c, dev(n), n, nullptr));
    const int D = 12 * nk;
    float *x = devf(nx), *u0 = devf(12), *knots = devf(D), *costs = devf(K), *eps = devf((size_t)K * D);
    float *traj = devf((size_t)K * (H + 1) * nx), *w = devf(K), *center = devf(D), *sd = devf(D);
    uint32_t* raw = static_cast<uint32_t*>(dev(4ull * K * 4 * ((D + 3) / 4)));
    OK(mppi_set_nominal(c, knots));
    OK(mppi_get_nominal(c, knots));
    OK(mppi_sample(c, eps, raw));
    OK(mppi_rollout_batch(c, x, nullptr, costs, nullptr));
    OK(mppi_rollout_batch(c, x, eps, costs, traj));
    OK(mppi_update(c, costs, eps, knots, w));
    OK(mppi_update(c, costs, nullptr, knots, nullptr));
    OK(mppi_update_shift(c, costs, u0, w));
    OK(mppi_step(c, x, u0));
    if (nx == 37 && K >= 2) {
        for (int gate : {(int)MPPI_PROPOSAL_GATE_COST, (int)MPPI_PROPOSAL_GATE_NONE, (int)MPPI_PROPOSAL_GATE_BEST,
                         MPPI_PROPOSAL_GATE_COST | MPPI_PROPOSAL_CONCURRENT,
                         MPPI_PROPOSAL_GATE_BEST | MPPI_PROPOSAL_CONCURRENT}) {
            OK(mppi_step_proposal(c, x, center, sd, 2, gate, u0));
            OK(mppi_step_proposal(c, x, center, sd, K, gate, u0));
        }
        const float cmd[3] = {0.5f, 0, 0}, org[2] = {0, 0};
        OK(mppi_set_proposal(c, pol, K / 4 >= 2 ? K / 4 : 2, MPPI_PROPOSAL_GATE_COST, cmd, org));
        OK(mppi_step(c, x, u0));
        OK(mppi_set_proposal(c, pol, 2, MPPI_PROPOSAL_GATE_BEST | MPPI_PROPOSAL_CONCURRENT, cmd, org));
        OK(mppi_step(c, x, u0));
        REFUSED(mppi_set_proposal(c, pol, 2, MPPI_PROPOSAL_GATE_NONE | MPPI_PROPOSAL_CONCURRENT, cmd, org));
        REFUSED(mppi_step_proposal(c, x, center, sd, 2, MPPI_PROPOSAL_GATE_NONE | MPPI_PROPOSAL_CONCURRENT, u0));
        REFUSED(mppi_step_proposal(c, x, center, sd, 2, 3, u0));
        OK(mppi_set_proposal(c, nullptr, 0, 0, nullptr, nullptr));
    }
    REFUSED(mppi_step_proposal(c, x, center, sd, K + 1, MPPI_PROPOSAL_GATE_NONE, u0));
    if (K < 2) REFUSED(mppi_step_proposal(c, x, center, sd, K, MPPI_PROPOSAL_GATE_NONE, u0));
    OK(mppi_sync_status(c));
    mppi_destroy(c);
}

static void policy(mppi_policy* p)
{
    const int N = mppi_policy_n_params();
    float *X = devf(600 * 40), *Y = devf(600 * 72), *G = devf(N), *L = devf(1), *P = devf(N);
    int* idx = static_cast<int*>(dev(4 * 512));
    for (int B : {1, 37, 64, 100, 128, 256, 512}) {
        float* out = devf((size_t)B * 144);
        OK(mppi_policy_forward(p, X, B, out));
        OK(mppi_policy_grad(p, X, Y, nullptr, B, G, L));
        OK(mppi_policy_grad(p, X, Y, idx, B, G, L));
        OK(mppi_policy_train_step(p, X, Y, idx, B, 1e-3f, L));
        OK(mppi_policy_nll(p, X, Y, nullptr, B, L));
        OK(mppi_policy_nll(p, X, Y, idx, B, L));
        float *c = devf(96), *s = devf(96);
        for (int nk = 2; nk <= 8; ++nk) OK(mppi_policy_head(p, out, nk, 0.25f, c, s));
    }
    OK(mppi_policy_adam(p, G, 1e-3f));
    OK(mppi_policy_get_params(p, P));
    OK(mppi_policy_set_params(p, P));
    REFUSED(mppi_policy_forward(p, X, 513, devf(513 * 144)));
    REFUSED(mppi_policy_nll(p, X, Y, nullptr, 4, nullptr));
    // training pairs of closed-loop records (no policy involved)
    for (int nk : {2, 4, 6, 8}) {
        const int n_rec = 3, steps = 17;
        float *rec = devf((size_t)n_rec * steps * (37 + 12 * nk)), *oc = devf(3 * n_rec);
        float *feat = devf((size_t)n_rec * steps * 40), *tgt = devf((size_t)n_rec * steps * 72);
        int* cnt = static_cast<int*>(dev(4 * n_rec));
        OK(mppi_policy_pairs(n_rec, steps, nk, rec, oc, 0.12f, feat, tgt, cnt, nullptr));
        REFUSED(mppi_policy_pairs(n_rec, steps, 9, rec, oc, 0.12f, feat, tgt, cnt, nullptr));
        REFUSED(mppi_policy_pairs(0, steps, nk, rec, oc, 0.12f, feat, tgt, cnt, nullptr));
        REFUSED(mppi_policy_pairs(n_rec, steps, nk, rec, oc, 0.12f, feat, tgt, nullptr, nullptr));
    }
}

static void batch(mppi_model* flat, mppi_model* terrain, mppi_model* push, mppi_policy* pol, int arith)
{
    mppi_batch* b = nullptr;
    if (OK(mppi_batch_create(16, 80, 4096, arith, &b)) < 0) return;
    const size_t total = mppi_batch_control_bytes(16, arith) + (64u << 20);
    OK(mppi_batch_bind(b, dev(total), total, nullptr));
    int sf, st, sp;
    OK(mppi_batch_add_model(b, flat, &sf));
    OK(mppi_batch_add_model(b, terrain, &st));
    OK(mppi_batch_add_model(b, push, &sp));
    struct Spec {
        int slot, K, H, nk, basis, prop;
    } specs[] = {{st, 64, 30, 6, 0, 1}, {sf, 48, 20, 4, 1, 1}, {sf, 32, 20, 4, 2, 0}, {sp, 257, 20, 8, 0, 0},
                 {sf, 4096, 80, 8, 0, 1}, {st, 2, 10, 2, 0, 1}, {sf, 17, 10, 5, 0, 1}};
    std::vector<int> ids;
    const float cmd[3] = {0.5f, 0, 0}, org[2] = {0, 0};
    for (const Spec& s : specs) {
        mppi_params p = params(s.K, s.H, s.nk, s.basis);
        std::vector<float> x0(50, 0.f), mu(96, 0.5f);
        int id = -1;
        mppi_params pt = p;
        pt.cost = MPPI_COST_TRACKING;
        REFUSED(mppi_batch_admit(b, s.slot, &pt, x0.data(), mu.data(), &id));
        OK(mppi_batch_admit(b, s.slot, &p, x0.data(), mu.data(), &id));
        ids.push_back(id);
        if (s.prop) OK(mppi_batch_set_proposal(b, id, pol, cmd, org));
        if (s.slot == sp) REFUSED(mppi_batch_set_proposal(b, id, pol, cmd, org));  // 50-float state
    }
    for (int k = 0; k < 3; ++k) OK(mppi_batch_step(b));
    REFUSED(mppi_batch_set_launch_mode(b, 2));
    OK(mppi_batch_set_launch_mode(b, 1));  // one kernel over the combined queue
    for (int order = 0; order < 2; ++order) {
        OK(mppi_batch_set_tuning(b, 4, order));
        OK(mppi_batch_step(b));
    }
    int tb = 0, to = 0, tm = 0;
    OK(mppi_batch_get_tuning(b, &tb, &to, &tm));
    if (tb != 4 || to != 1 || tm != 1) {
        std::printf("BAD tuning read back %d %d %d\n", tb, to, tm);
        ++g_bad;
    }
    OK(mppi_batch_set_launch_mode(b, 0));
    OK(mppi_batch_set_proposal(b, ids[0], nullptr, nullptr, nullptr));
    OK(mppi_batch_remove(b, ids[1]));
    OK(mppi_batch_record(b, ids[2], devf(7 * (37 + 48)), 7));
    int bb = 0, bo = 0;
    float ms = 0;
    OK(mppi_batch_autotune(b, 1, &bb, &bo, &ms));
    for (int k = 0; k < 2; ++k) OK(mppi_batch_step(b));
    OK(mppi_batch_set_launch_mode(b, 1));  // after a removal and a proposal change
    for (int k = 0; k < 2; ++k) OK(mppi_batch_step(b));
    std::vector<float> x(50), u0(12), mu(96);
    float acc;
    uint32_t step;
    OK(mppi_batch_read(b, ids[2], x.data(), u0.data(), mu.data(), &acc, &step));
    mppi_batch_destroy(b);
}

int main()
{
    std::vector<float> hf(64 * 64, 0.01f);
    mppi_model_desc df = robot(MPPI_SCENE_FLAT), dh = robot(MPPI_SCENE_HEIGHTFIELD), db = robot(MPPI_SCENE_FREE_BOX);
    mppi_model_desc dc = robot(MPPI_SCENE_STATIC_BOX);
    dh.hf_nx = dh.hf_ny = 64; dh.hf_cell = 0.05f; dh.hf_x0 = dh.hf_y0 = -1.6f; dh.heightfield = hf.data();
    mppi_model *flat, *terrain, *push, *climb;
    OK(mppi_model_create(&df, &flat));
    OK(mppi_model_create(&dh, &terrain));
    OK(mppi_model_create(&db, &push));
    OK(mppi_model_create(&dc, &climb));
    mppi_policy* pol = nullptr;
    OK(mppi_policy_create(nullptr, 1, 512, &pol));
    const size_t pn = mppi_policy_workspace_bytes(pol);
    OK(mppi_policy_bind(pol, dev(pn), pn, nullptr));

    controller(flat, pol, 37, 64, 25, 4, 0);
    controller(terrain, pol, 37, 1024, 50, 6, 1);
    controller(climb, pol, 37, 5, 3, 3, 2);
    controller(push, pol, 50, 257, 60, 8, 0);
    controller(flat, pol, 37, 1, 1, 2, 0);
    tracking(flat, pol, 37, 64, 25, 4, 0);
    tracking(terrain, pol, 37, 100, 50, 6, 1);
    tracking(push, pol, 50, 257, 60, 8, 0);
    tracking(flat, pol, 37, 1, 256, 8, 0);
    policy(pol);
    batch(flat, terrain, push, pol, 0);
    batch(flat, terrain, push, pol, 1);

    mppi_policy_destroy(pol);
    for (mppi_model* m : {flat, terrain, push, climb}) mppi_model_destroy(m);
    for (void* p : g_alloc) std::free(p);
    std::printf("batch tiles checked: %d, proposal rows: %d\n", g_batch_tiles, g_prop_rows);
    std::printf("out of range: %d\n", g_bad);
    return g_bad ? 1 : 0;
}
