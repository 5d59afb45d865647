// Eq. 3 / Eq. 4 sample cost on rollout trajectories (gfx950).
//
// One 64-lane workgroup per sample.  The lanes first build, in LDS, the joint reference
// u_ref(t_k) of the trotting gait for every rollout time (Sec. IV-B names a Raibert-
// heuristic gait; its footholds and arcs are the library's reading), the knot
// interpolation matrix and the sample's knots theta = mu + sigma eps.  Each lane then
// takes the stages k = lane, lane + 64, ... of the horizon: the post-step state x_{k+1}
// (one contiguous row of the trajectory, so the workgroup's loads are coalesced), the
// interpolated control u_k, and the weighted squared deviations of Eq. 3 plus Eq. 4's l1
// box distance.  A fixed-order butterfly sums the lanes.  Work per sample is H x (36 + 12
// + 12 nk) multiply-adds next to a rollout of H full dynamics steps, and the trajectory
// is read once, so the kernel is a small HBM stream after the rollout.
#include <hip/hip_runtime.h>

#include "tracking_launch.h"

namespace track {

constexpr int kLanes = 64;
constexpr int kMaxKnots = 8;

template <typename R>
struct Math;
template <>
struct Math<double> {
    __device__ static double atan2_(double y, double x) { return ::atan2(y, x); }
    __device__ static double acos_(double x) { return ::acos(x); }
    __device__ static double sin_(double x) { return ::sin(x); }
    __device__ static double cos_(double x) { return ::cos(x); }
    __device__ static double sqrt_(double x) { return ::sqrt(x); }
    __device__ static double floor_(double x) { return ::floor(x); }
    __device__ static double abs_(double x) { return ::fabs(x); }
};
template <>
struct Math<float> {
    __device__ static float atan2_(float y, float x) { return atan2f(y, x); }
    __device__ static float acos_(float x) { return acosf(x); }
    __device__ static float sin_(float x) { return sinf(x); }
    __device__ static float cos_(float x) { return cosf(x); }
    __device__ static float sqrt_(float x) { return sqrtf(x); }
    __device__ static float floor_(float x) { return floorf(x); }
    __device__ static float abs_(float x) { return fabsf(x); }
};

// joint angles (abduction, flexion, knee) that put the foot centre at p relative to the
// hip: abduction turns the leg plane about x; in that plane the two links reach the
// clamped distance with the knee bent backwards
template <typename R>
__device__ void leg_ik(R l1, R l2, const R p[3], R q[3])
{
    using M = Math<R>;
    const R r = M::sqrt_(p[1] * p[1] + p[2] * p[2]);
    const R a = M::atan2_(p[1], -p[2]);
    const R xs = p[0], zs = -r;
    R d = M::sqrt_(xs * xs + zs * zs);
    const R dmin = M::abs_(l1 - l2) + R(0.05) * (l1 + l2), dmax = R(0.999) * (l1 + l2);
    d = d < dmin ? dmin : d;
    d = d > dmax ? dmax : d;
    R ck = (d * d - l1 * l1 - l2 * l2) / (R(2) * l1 * l2);
    ck = ck > R(1) ? R(1) : ck;
    ck = ck < R(-1) ? R(-1) : ck;
    const R k = -M::acos_(ck);
    q[0] = a;
    q[1] = M::atan2_(-xs, -zs) - M::atan2_(l2 * M::sin_(k), l1 + l2 * M::cos_(k));
    q[2] = k;
}

// foot target of `leg` relative to its hip at gait time t (heading-frame velocity v and
// command c)
template <typename R>
__device__ void gait_foot(const TrackDev& g, int leg, R t, const R v[2], const R c[2], R p[3])
{
    using M = Math<R>;
    if (g.gait == 0) {
        p[0] = R(0); p[1] = R(0); p[2] = -R(g.stand_h);
        return;
    }
    const R T = g.period, duty = g.duty, Tst = duty * T;
    const R off = (leg == 1 || leg == 2) ? R(0.5) : R(0);  // diagonal pairs
    R ph = t / T + off;
    ph -= M::floor_(ph);
    R land[2], xy[2], lift = R(0);
    for (int i = 0; i < 2; ++i) land[i] = R(0.5) * c[i] * Tst + R(g.raibert_k) * (v[i] - c[i]);
    if (ph < duty) {
        const R s = ph / duty;
        for (int i = 0; i < 2; ++i) xy[i] = land[i] - c[i] * Tst * s;
    } else {
        const R s = (ph - duty) / (R(1) - duty);
        const R pi = R(3.14159265358979323846);
        const R w = R(0.5) * (R(1) - M::cos_(pi * s));
        for (int i = 0; i < 2; ++i) {
            const R lo = land[i] - c[i] * Tst;
            xy[i] = lo + (land[i] - lo) * w;
        }
        lift = R(g.swing_h) * M::sin_(pi * s);
    }
    p[0] = xy[0];
    p[1] = xy[1];
    p[2] = -R(g.stand_h) + lift;
}

template <typename R>
__global__ __launch_bounds__(kLanes) void tracking_cost_kernel(TrackArgs a)
{
    using M = Math<R>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int H = a.H, nk = a.nk, nx = a.nx, D = 12 * nk;
    R* sRef = reinterpret_cast<R*>(lds_raw);  // (H + 1) x 12
    R* sB = sRef + (size_t)(H + 1) * 12;      // H x nk
    R* sTh = sB + (size_t)H * nk;             // 12 x nk
    const int n = blockIdx.x, lane = threadIdx.x;
    const float* tr = a.traj + (size_t)n * (H + 1) * nx;

    // heading frame of the start state (row 0, the same for every sample)
    const R qw = tr[3], qx = tr[4], qy = tr[5], qz = tr[6];
    const R psi = M::atan2_(R(2) * (qw * qz + qx * qy), R(1) - R(2) * (qy * qy + qz * qz));
    const R cs = M::cos_(psi), sn = M::sin_(psi);
    const R vx = tr[19], vy = tr[20];
    const R vh[2] = {cs * vx + sn * vy, -sn * vx + cs * vy};
    const R ch[2] = {cs * R(a.c.v_cmd[0]) + sn * R(a.c.v_cmd[1]), -sn * R(a.c.v_cmd[0]) + cs * R(a.c.v_cmd[1])};
    for (int i = lane; i < (H + 1) * 4; i += kLanes) {
        const int k = i >> 2, leg = i & 3;
        const R t = R(a.step + (uint32_t)k) * R(a.dt);
        R p[3], q[3];
        gait_foot<R>(a.c, leg, t, vh, ch, p);
        leg_ik<R>(R(a.c.l1), R(a.c.l2), p, q);
        for (int j = 0; j < 3; ++j) sRef[k * 12 + 3 * leg + j] = q[j];
    }
    for (int i = lane; i < H * nk; i += kLanes) sB[i] = R(a.B[i]);
    for (int d = lane; d < D; d += kLanes)
        sTh[d] = R(a.mu[d]) + (n ? R(a.sigma) * R(a.eps[(size_t)n * a.eps_sn + (size_t)d * a.eps_sd]) : R(0));
    __syncthreads();

    R acc = R(0);
    for (int k = lane; k < H; k += kLanes) {
        const float* x = tr + (size_t)(k + 1) * nx;
        const R tx = R(a.step + (uint32_t)(k + 1)) * R(a.dt);
        const R* qref = sRef + (k + 1) * 12;
        const R* uref = sRef + k * 12;
        // weighted squares of the state error, in the order of the error vector
        R l = R(0);
        auto add = [&](int i, R e) { l += R(a.c.Q[i]) * e * e; };
        add(0, R(x[0]) - (R(a.c.p_ref0[0]) + R(a.c.v_cmd[0]) * tx));
        add(1, R(x[1]) - (R(a.c.p_ref0[1]) + R(a.c.v_cmd[1]) * tx));
        add(2, R(x[2]) - R(a.c.p_ref0[2]));
        const R sg = x[3] < 0.f ? R(-1) : R(1);
        for (int i = 0; i < 3; ++i) add(3 + i, R(2) * sg * R(x[4 + i]));
        for (int j = 0; j < 12; ++j) add(6 + j, R(x[7 + j]) - qref[j]);
        add(18, R(x[19]) - R(a.c.v_cmd[0]));
        add(19, R(x[20]) - R(a.c.v_cmd[1]));
        add(20, R(x[21]));
        for (int i = 0; i < 3; ++i) add(21 + i, R(x[22 + i]));
        for (int j = 0; j < 12; ++j) add(24 + j, R(x[25 + j]));
        for (int j = 0; j < 12; ++j) {
            R u = R(0);
            for (int i = 0; i < kMaxKnots; ++i)
                if (i < nk) u += sB[k * nk + i] * sTh[j * nk + i];
            const R du = u - uref[j];
            l += R(a.c.R[j]) * du * du;
        }
        if (a.c.box)
            l += R(a.c.box_w) * (M::abs_(R(a.c.box_goal[0]) - R(x[37])) + M::abs_(R(a.c.box_goal[1]) - R(x[38])));
        acc += R(a.dt) * l;
    }
    for (int o = kLanes / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kLanes);
    if (lane == 0) {
        float Lf = (float)acc;
        if (!(fabsf(Lf) <= 3.0e38f)) Lf = __int_as_float(0x7f800000);  // non-finite -> +inf
        a.costs[n] = Lf;
    }
}

size_t tracking_lds_bytes(int arith, int H, int nk)
{
    const size_t r = arith == 0 ? sizeof(double) : sizeof(float);
    return r * ((size_t)(H + 1) * 12 + (size_t)H * nk + 12 * (size_t)nk);
}

hipError_t launch_tracking_cost(int arith, const TrackArgs& a, hipStream_t st)
{
    if (a.K <= 0) return hipSuccess;
    const size_t lds = tracking_lds_bytes(arith, a.H, a.nk);
    if (arith == 0)
        hipLaunchKernelGGL(tracking_cost_kernel<double>, dim3(a.K), dim3(kLanes), lds, st, a);
    else
        hipLaunchKernelGGL(tracking_cost_kernel<float>, dim3(a.K), dim3(kLanes), lds, st, a);
    return hipGetLastError();
}

}  // namespace track
