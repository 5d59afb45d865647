// Eq. 3 / Eq. 4 sample cost on rollout trajectories (gfx950).
//
// gait_table_kernel builds the joint reference u_ref(t_k) of the gait for every rollout
// time once per control step (Sec. IV-B names a Raibert-heuristic trotting gait; its
// footholds and arcs are the library's reading); every sample shares it.
// tracking_cost_kernel: one 64-lane workgroup per sample, its knots theta = mu + sigma eps
// in LDS.  Each lane then takes the stages k = lane, lane + 64, ... of the horizon: the state
// x_{k+1}, the interpolated control u_k, and the weighted squared deviations of Eq. 3 plus
// Eq. 4's l1 box distance.  A fixed-order butterfly sums the lanes.  The trajectory is
// read once, so the kernel is an HBM stream after the rollout (H x nx x 4 bytes per
// sample).
#include <hip/hip_runtime.h>

#include "tracking_launch.h"

namespace track {

constexpr int kLanes = 64;
constexpr int kTableLanes = 256;
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

// joint reference u_ref(t_k), k = 0..H, of the gait in the heading frame of the start
// state x0: one workgroup, one (time, leg) pair per lane, written to uref[(H+1) x 12]
template <typename R>
__global__ __launch_bounds__(kTableLanes) void gait_table_kernel(TrackArgs a, const float* __restrict__ x0,
                                                                 R* __restrict__ uref)
{
    using M = Math<R>;
    const R qw = x0[3], qx = x0[4], qy = x0[5], qz = x0[6];
    const R psi = M::atan2_(R(2) * (qw * qz + qx * qy), R(1) - R(2) * (qy * qy + qz * qz));
    const R cs = M::cos_(psi), sn = M::sin_(psi);
    const R vx = x0[19], vy = x0[20];
    const R vh[2] = {cs * vx + sn * vy, -sn * vx + cs * vy};
    const R ch[2] = {cs * R(a.c.v_cmd[0]) + sn * R(a.c.v_cmd[1]), -sn * R(a.c.v_cmd[0]) + cs * R(a.c.v_cmd[1])};
    for (int i = threadIdx.x; i < (a.H + 1) * 4; i += kTableLanes) {
        const int k = i >> 2, leg = i & 3;
        const R t = R(a.step + (uint32_t)k) * R(a.dt);
        R p[3], q[3];
        gait_foot<R>(a.c, leg, t, vh, ch, p);
        leg_ik<R>(R(a.c.l1), R(a.c.l2), p, q);
        for (int j = 0; j < 3; ++j) uref[k * 12 + 3 * leg + j] = q[j];
    }
}

// one sample per workgroup: its knots theta go to LDS; lane k then loads its post-step
// state row straight from the trajectory (independent loads, so a lane waits for one
// memory round trip, not one per element), and reads the shared gait table and
// interpolation rows (L2-resident)
template <typename R>
__global__ __launch_bounds__(kLanes) void tracking_cost_kernel(TrackArgs a, const R* __restrict__ uref)
{
    using M = Math<R>;
    __shared__ R sTh[kMaxKnots * 12];
    const int H = a.H, nk = a.nk, nx = a.nx, D = 12 * nk;
    const int n = blockIdx.x, lane = threadIdx.x;
    const float* tr = a.traj + (size_t)n * (H + 1) * nx + nx;  // rows 1..H
    for (int d = lane; d < D; d += kLanes)
        sTh[d] = R(a.mu[d]) + (n ? R(a.sigma) * R(a.eps[(size_t)n * a.eps_sn + (size_t)d * a.eps_sd]) : R(0));
    __syncthreads();

    R acc = R(0);
    for (int k = lane; k < H; k += kLanes) {
        const float* x = tr + (size_t)k * nx;  // x_{k+1}
        const R tx = R(a.step + (uint32_t)(k + 1)) * R(a.dt);
        const R* qref = uref + (k + 1) * 12;
        const R* ur = uref + k * 12;
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
        const double* Bk = a.B + (size_t)k * nk;
        for (int j = 0; j < 12; ++j) {
            R u = R(0);
            for (int i = 0; i < kMaxKnots; ++i)
                if (i < nk) u += R(Bk[i]) * sTh[j * nk + i];
            const R du = u - ur[j];
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

size_t tracking_lds_bytes(int arith, int H, int nk, int nx)
{
    (void)H; (void)nk; (void)nx;
    return (arith == 0 ? sizeof(double) : sizeof(float)) * kMaxKnots * 12;  // static: theta
}

size_t tracking_table_bytes(int H) { return sizeof(double) * (size_t)(H + 1) * 12; }

hipError_t launch_tracking_cost(int arith, const TrackArgs& a, const float* x0, void* table, hipStream_t st)
{
    if (a.K <= 0) return hipSuccess;
    if (arith == 0) {
        hipLaunchKernelGGL(gait_table_kernel<double>, dim3(1), dim3(kTableLanes), 0, st, a, x0, (double*)table);
        hipLaunchKernelGGL(tracking_cost_kernel<double>, dim3(a.K), dim3(kLanes), 0, st, a, (const double*)table);
    } else {
        hipLaunchKernelGGL(gait_table_kernel<float>, dim3(1), dim3(kTableLanes), 0, st, a, x0, (float*)table);
        hipLaunchKernelGGL(tracking_cost_kernel<float>, dim3(a.K), dim3(kLanes), 0, st, a, (const float*)table);
    }
    return hipGetLastError();
}

}  // namespace track
