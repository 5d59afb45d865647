// Device code of the whole-body MPPI rollout for gfx950 (CDNA4, wave64).
//
// Decomposition: one sample per QUAD of lanes, one leg per lane.  Each lane does its
// leg's kinematics, mass-matrix columns, bias forces, foot contacts, two of the eight
// trunk-corner contacts and the elimination of its leg's 3x3 block from the implicit
// system.  The base's 6x6 Schur complement and right-hand side are summed across the
// quad with DPP quad permutes (bitwise identical in all four lanes); every lane then
// solves the 6x6 system redundantly and back-substitutes its own leg.
//
// Dynamics (in place of the MuJoCo simulator of Sec. III-A): floating-base rigid
// bodies expressed in trunk coordinates with generalized velocity
// nu = [omega_b, v_b, qd] (v_b = R^T v_world).  One step solves
//   (M + dt D) dnu = dt f,   f = S^T tau + sum J_c^T F_c - b(q, v),
//   D = kd (joints) + sum J_c^T D_c J_c,
// and maps the increment back to world linear velocity with the same R.  The bias b
// is the generalized force of the body wrenches needed for zero generalized
// acceleration (per-body Newton-Euler, projected), equal to the recursive
// Newton-Euler result.
//
// Arithmetic type R: the state lives in FP32 between steps; one step is computed in R.
// With R = double the per-step result is limited only by the FP32 state (the contact
// damping makes the implicit system too ill-conditioned for FP32 assembly to reach a
// 1e-5 relative per-step error); R = float is the faster, less precise variant.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mppi_launch.h"

namespace mppi {

constexpr int kMaxKnots = 8;
constexpr int kMaxHorizon = 256;
constexpr int kMaxHF = 14336;

template <typename R>
struct ModelT {
    R tsx, tsy, tsz;        // trunk size
    R m0, I0x, I0y, I0z;    // trunk mass and principal inertia
    R hip_x, hip_y;
    R l1, m1, k1;           // thigh length, mass, rod inertia m L^2 / 12
    R l2, m2, k2;           // calf
    R mtot;
    R foot_r, g;
    R ck, cc, cmu, inv_vs;  // contact stiffness, damping, friction, 1/slip velocity
    R hf_inv_cell, hf_x0, hf_y0;
    R sb_cx, sb_cy, sb_cz, sb_hx, sb_hy, sb_hz;                // static box
    R bx_hx, bx_hy, bx_hz, bx_m, bx_Ix, bx_Iy, bx_Iz;          // free box
    int scene, hf_nx, hf_ny, pad;
};
using DevModelF = ModelT<float>;
using DevModelD = ModelT<double>;


// ------------------------------------------------------------------------------
// math wrappers for both arithmetic types
// ------------------------------------------------------------------------------
__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_abs(float x) { return fabsf(x); }
__device__ __forceinline__ double m_abs(double x) { return fabs(x); }
__device__ __forceinline__ float m_min(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double m_min(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float m_max(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double m_max(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float m_floor(float x) { return floorf(x); }
__device__ __forceinline__ double m_floor(double x) { return floor(x); }
__device__ __forceinline__ float m_tanh(float x) { return tanhf(x); }
__device__ __forceinline__ double m_tanh(double x) { return tanh(x); }
__device__ __forceinline__ float m_sin(float x) { return sinf(x); }
__device__ __forceinline__ double m_sin(double x) { return sin(x); }
__device__ __forceinline__ float m_cos(float x) { return cosf(x); }
__device__ __forceinline__ double m_cos(double x) { return cos(x); }
// FP32 sine and cosine written out without branches (the device library's sincosf
// carries a large-argument path and branches that cost a wave about 45 instructions):
// x = k pi/2 + r with k = rint(2x/pi) and pi/2 taken in two parts (the float nearest pi/2
// and the remainder), so r is exact to a few ulps for the joint and rotation angles met
// here (|x| up to a few hundred); then the Taylor series of sin and cos on |r| <= pi/4 up
// to r^9 and r^10 (truncation below 3e-9 relative) and the quadrant's swap and signs.
// About 2 ulp (relative to max(|value|, 2^-10)) on a host check of 4 million arguments.
__device__ __forceinline__ void m_sincos(float x, float* sn, float* cs)
{
    const float k = rintf(x * 0.63661977236758134f);
    float r = fmaf(-k, 1.57079637050628662f, x);
    r = fmaf(-k, -4.37113900018624283e-8f, r);
    const float r2 = r * r;
    const float sp = r + r * r2 * fmaf(r2, fmaf(r2, fmaf(r2, 1.f / 362880.f, -1.f / 5040.f), 1.f / 120.f), -1.f / 6.f);
    const float cp =
        fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -1.f / 3628800.f, 1.f / 40320.f), -1.f / 720.f), 1.f / 24.f), -0.5f),
             1.f);
    const int q = int(k) & 3;
    const float s0 = (q & 1) ? cp : sp, c0 = (q & 1) ? sp : cp;
    *sn = (q & 2) ? -s0 : s0;
    *cs = ((q + 1) & 2) ? -c0 : c0;
}
__device__ __forceinline__ void m_sincos(double x, double* s, double* c) { sincos(x, s, c); }

// tanh(s) / s for s >= 0 (the friction law's secant factor).  FP32: below s = 1/2 its
// Taylor series in s^2 through s^14 (coefficients 1, -1/3, 2/15, -17/315, 62/2835,
// -1382/155925, 21844/6081075, -929569/638512875; the next term is under 1e-8), else
// (1 - e^-2s) / ((1 + e^-2s) s), where e^-2s <= 0.37 keeps the difference well
// conditioned; both are evaluated and one selected, so lanes do not diverge (about 3 ulp).
// FP64: the device library's tanh, and the series' first two terms below 1e-4.
__device__ __forceinline__ float tanh_ratio(float s)
{
    const float s2 = s * s;
    float ser = fmaf(s2, -929569.f / 638512875.f, 21844.f / 6081075.f);
    ser = fmaf(s2, ser, -1382.f / 155925.f);
    ser = fmaf(s2, ser, 62.f / 2835.f);
    ser = fmaf(s2, ser, -17.f / 315.f);
    ser = fmaf(s2, ser, 2.f / 15.f);
    ser = fmaf(s2, ser, -1.f / 3.f);
    ser = fmaf(s2, ser, 1.f);
    const float t = __expf(-2.f * s);
    const float big = (1.f - t) / ((1.f + t) * s);
    return s < 0.5f ? ser : big;
}
__device__ __forceinline__ double tanh_ratio(double s)
{
    return (s < 1e-4) ? 1.0 - s * s * (1.0 / 3.0) : tanh(s) / s;
}
__device__ __forceinline__ float m_log(float x) { return logf(x); }
__device__ __forceinline__ double m_log(double x) { return log(x); }
__device__ __forceinline__ void m_sincospi(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __forceinline__ void m_sincospi(double x, double* s, double* c) { sincospi(x, s, c); }

// sin(a)/a and cos(a) for the quaternion exponential.  FP32: one sine-cosine evaluation,
// sin(a)/a from its series below a = 1e-2; FP64: the library's sin and cos.
__device__ __forceinline__ void quat_exp(float a, float* sinc, float* c)
{
    float s;
    m_sincos(a, &s, c);
    const float a2 = a * a;
    *sinc = (a < 1e-2f) ? 1.f - a2 * (1.f / 6.f) + a2 * a2 * (1.f / 120.f) : s / a;
}
__device__ __forceinline__ void quat_exp(double a, double* sinc, double* c)
{
    *sinc = (a > 0.0) ? sin(a) / a : 1.0;
    *c = cos(a);
}

// ------------------------------------------------------------------------------
// small vector algebra
// ------------------------------------------------------------------------------
template <typename R>
struct V3 {
    R x, y, z;
};
template <typename R>
__device__ __forceinline__ V3<R> v3(R x, R y, R z)
{
    return V3<R>{x, y, z};
}
template <typename R>
__device__ __forceinline__ V3<R> operator+(V3<R> a, V3<R> b)
{
    return V3<R>{a.x + b.x, a.y + b.y, a.z + b.z};
}
template <typename R>
__device__ __forceinline__ V3<R> operator-(V3<R> a, V3<R> b)
{
    return V3<R>{a.x - b.x, a.y - b.y, a.z - b.z};
}
template <typename R>
__device__ __forceinline__ V3<R> operator*(R s, V3<R> a)
{
    return V3<R>{s * a.x, s * a.y, s * a.z};
}
template <typename R>
__device__ __forceinline__ R dot(V3<R> a, V3<R> b)
{
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename R>
__device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b)
{
    return V3<R>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// rod inertia about its centre, k (I - d d^T), applied to a
template <typename R>
__device__ __forceinline__ V3<R> rod_I(R k, V3<R> d, V3<R> a)
{
    return k * (a - dot(d, a) * d);
}

template <typename R>
struct M33 {
    R m[9];
};
template <typename R>
__device__ __forceinline__ V3<R> mul(const M33<R>& A, V3<R> a)
{
    return V3<R>{A.m[0] * a.x + A.m[1] * a.y + A.m[2] * a.z, A.m[3] * a.x + A.m[4] * a.y + A.m[5] * a.z,
                 A.m[6] * a.x + A.m[7] * a.y + A.m[8] * a.z};
}
template <typename R>
__device__ __forceinline__ V3<R> mulT(const M33<R>& A, V3<R> a)
{
    return V3<R>{A.m[0] * a.x + A.m[3] * a.y + A.m[6] * a.z, A.m[1] * a.x + A.m[4] * a.y + A.m[7] * a.z,
                 A.m[2] * a.x + A.m[5] * a.y + A.m[8] * a.z};
}
template <typename R>
__device__ __forceinline__ M33<R> quat_R(R w, R x, R y, R z)
{
    M33<R> A;
    const R one = R(1), two = R(2);
    A.m[0] = one - two * (y * y + z * z); A.m[1] = two * (x * y - w * z);       A.m[2] = two * (x * z + w * y);
    A.m[3] = two * (x * y + w * z);       A.m[4] = one - two * (x * x + z * z); A.m[5] = two * (y * z - w * x);
    A.m[6] = two * (x * z - w * y);       A.m[7] = two * (y * z + w * x);       A.m[8] = one - two * (x * x + y * y);
    return A;
}

// packed upper triangle of a symmetric 6x6
__device__ __forceinline__ constexpr int s6(int i, int j)
{
    return (i <= j) ? (i * 6 - (i * (i - 1)) / 2 + (j - i)) : (j * 6 - (j * (j - 1)) / 2 + (i - j));
}

// ------------------------------------------------------------------------------
// quad (4-lane) all-reduce with DPP: xor 1 then xor 2 inside each quad.  Addition is
// commutative in IEEE arithmetic, so all four lanes hold the bitwise same sum.
// ------------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const int lo = dpp_i<CTRL>(__double2loint(v)), hi = dpp_i<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <typename R>
__device__ __forceinline__ R quad_sum(R v)
{
    v = v + dpp<0xB1>(v);
    return v + dpp<0x4E>(v);
}

// ------------------------------------------------------------------------------
// counter-based Gaussian noise: Philox4x32-10 (Salmon et al., SC'11), 24-bit
// uniforms ((x >> 8) + 1/2) 2^-24, Box-Muller on word pairs (0,1) and (2,3).
// ------------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}
template <typename R>
__device__ __forceinline__ R u24(uint32_t x)
{
    return ((R)(x >> 8) + R(0.5)) * R(1.0 / 16777216.0);
}

// Gaussian noise element d of sample n for (step, instance) and key (seed_lo, seed_hi)
template <typename R>
__device__ __forceinline__ R gauss_elem(const DevParams& P, uint32_t n, uint32_t d)
{
    uint32_t c[4] = {d >> 2, n, P.step, P.instance};
    philox4x32_10(c, P.seed_lo, P.seed_hi);
    const uint32_t pair = (d >> 1) & 1u;
    const uint32_t a = pair ? c[2] : c[0], b = pair ? c[3] : c[1];
    const R r = m_sqrt(R(-2) * m_log(u24<R>(a)));
    R s, co;
    m_sincospi(R(2) * u24<R>(b), &s, &co);
    return (d & 1u) ? r * s : r * co;
}

// ------------------------------------------------------------------------------
// contact geometry
// ------------------------------------------------------------------------------
// terrain below a sphere (r > 0) or point (r = 0); ground plane z = 0 unless heightfield
template <int SCENE, typename R>
__device__ __forceinline__ bool terrain(const ModelT<R>& M, const float* __restrict__ hf, V3<R> c, R r, R& delta,
                                        V3<R>& n)
{
    R h = R(0), gx = R(0), gy = R(0);
    if constexpr (SCENE == 1) {
        const int nx = M.hf_nx, ny = M.hf_ny;
        R fx = (c.x - M.hf_x0) * M.hf_inv_cell, fy = (c.y - M.hf_y0) * M.hf_inv_cell;
        bool inx = true, iny = true;
        if (fx < R(0)) { fx = R(0); inx = false; }
        if (fx > R(nx - 1)) { fx = R(nx - 1); inx = false; }
        if (fy < R(0)) { fy = R(0); iny = false; }
        if (fy > R(ny - 1)) { fy = R(ny - 1); iny = false; }
        int i0 = (int)m_floor(fx), j0 = (int)m_floor(fy);
        i0 = max(0, min(i0, nx - 2));  // also maps a NaN coordinate to a valid cell
        j0 = max(0, min(j0, ny - 2));
        const R tx = fx - R(i0), ty = fy - R(j0);
        const R h00 = hf[j0 * nx + i0], h10 = hf[j0 * nx + i0 + 1];
        const R h01 = hf[(j0 + 1) * nx + i0], h11 = hf[(j0 + 1) * nx + i0 + 1];
        h = (R(1) - ty) * ((R(1) - tx) * h00 + tx * h10) + ty * ((R(1) - tx) * h01 + tx * h11);
        if (inx) gx = ((R(1) - ty) * (h10 - h00) + ty * (h11 - h01)) * M.hf_inv_cell;
        if (iny) gy = ((R(1) - tx) * (h01 - h00) + tx * (h11 - h10)) * M.hf_inv_cell;
    }
    const R inv = R(1) / m_sqrt(gx * gx + gy * gy + R(1));
    n = v3(-gx * inv, -gy * inv, inv);
    delta = (h + r - c.z) * n.z;
    return delta > R(0);
}

// sphere (centre l relative to an axis-aligned box, half sizes bh); n from box to sphere
template <typename R>
__device__ __forceinline__ bool sphere_aabox(V3<R> l, R r, V3<R> bh, R& delta, V3<R>& n)
{
    const bool inside = m_abs(l.x) <= bh.x && m_abs(l.y) <= bh.y && m_abs(l.z) <= bh.z;
    if (!inside) {
        const V3<R> q = v3(m_min(m_max(l.x, -bh.x), bh.x), m_min(m_max(l.y, -bh.y), bh.y),
                           m_min(m_max(l.z, -bh.z), bh.z));
        const V3<R> e = l - q;
        const R dist = m_sqrt(dot(e, e));
        if (!(dist < r)) return false;
        delta = r - dist;
        n = (R(1) / dist) * e;
    } else {
        const R dx = bh.x - m_abs(l.x), dy = bh.y - m_abs(l.y), dz = bh.z - m_abs(l.z);
        R depth = dx;
        n = v3(l.x >= R(0) ? R(1) : R(-1), R(0), R(0));
        if (dy < depth) { depth = dy; n = v3(R(0), l.y >= R(0) ? R(1) : R(-1), R(0)); }
        if (dz < depth) { depth = dz; n = v3(R(0), R(0), l.z >= R(0) ? R(1) : R(-1)); }
        delta = r + depth;
    }
    return true;
}

// point l (relative to an axis-aligned box) strictly inside: shallowest face depth, normal
template <typename R>
__device__ __forceinline__ bool point_aabox(V3<R> l, V3<R> bh, R& delta, V3<R>& n)
{
    if (!(m_abs(l.x) < bh.x && m_abs(l.y) < bh.y && m_abs(l.z) < bh.z)) return false;
    const R dx = bh.x - m_abs(l.x), dy = bh.y - m_abs(l.y), dz = bh.z - m_abs(l.z);
    R depth = dx;
    n = v3(l.x >= R(0) ? R(1) : R(-1), R(0), R(0));
    if (dy < depth) { depth = dy; n = v3(R(0), l.y >= R(0) ? R(1) : R(-1), R(0)); }
    if (dz < depth) { depth = dz; n = v3(R(0), R(0), l.z >= R(0) ? R(1) : R(-1)); }
    delta = depth;
    return true;
}

// Penalty law: Fn = k delta - c v_n while overlapping, friction -mu max(Fn,0) tanh(s) t,
// s = |v_t| / v_s, entered as a viscous force with the secant coefficient eta.  The
// damping is D = eta I + (c - eta) n n^T.
template <typename R>
__device__ __forceinline__ void contact_law(const ModelT<R>& M, R delta, V3<R> n, V3<R> vrel, V3<R>& F, R& eta)
{
    const R vn = dot(n, vrel);
    const R Fn = M.ck * delta - M.cc * vn;
    const V3<R> vt = vrel - vn * n;
    const R s = m_sqrt(dot(vt, vt)) * M.inv_vs;
    eta = M.cmu * m_max(Fn, R(0)) * M.inv_vs * tanh_ratio(s);
    F = Fn * n - eta * vt;
}

// ------------------------------------------------------------------------------
// per-quad state (R-typed registers; rounded to FP32 between steps)
// ------------------------------------------------------------------------------
template <typename R>
struct Base {
    V3<R> p;
    R qw, qx, qy, qz;
    V3<R> vw, w;
};
template <typename R>
struct Leg {
    R q[3], qd[3];
};

template <typename R>
__device__ __forceinline__ R to_f32(R v)
{
    return (R)(float)v;
}
template <typename R>
__device__ __forceinline__ void round_state(Base<R>& b, Leg<R>& lg)
{
    b.p = v3(to_f32(b.p.x), to_f32(b.p.y), to_f32(b.p.z));
    b.qw = to_f32(b.qw); b.qx = to_f32(b.qx); b.qy = to_f32(b.qy); b.qz = to_f32(b.qz);
    b.vw = v3(to_f32(b.vw.x), to_f32(b.vw.y), to_f32(b.vw.z));
    b.w = v3(to_f32(b.w.x), to_f32(b.w.y), to_f32(b.w.z));
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        lg.q[j] = to_f32(lg.q[j]);
        lg.qd[j] = to_f32(lg.qd[j]);
    }
}

template <typename R>
__device__ __forceinline__ void load_state(const float* __restrict__ x, int leg, Base<R>& b, Leg<R>& lg)
{
    b.p = v3<R>(x[0], x[1], x[2]);
    b.qw = x[3]; b.qx = x[4]; b.qy = x[5]; b.qz = x[6];
    b.vw = v3<R>(x[19], x[20], x[21]);
    b.w = v3<R>(x[22], x[23], x[24]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        lg.q[j] = x[7 + 3 * leg + j];
        lg.qd[j] = x[25 + 3 * leg + j];
    }
}

template <typename R>
__device__ __forceinline__ void store_state(float* __restrict__ o, int leg, const Base<R>& b, const Leg<R>& lg)
{
    if (leg == 0) {
        o[0] = (float)b.p.x; o[1] = (float)b.p.y; o[2] = (float)b.p.z;
        o[3] = (float)b.qw; o[4] = (float)b.qx; o[5] = (float)b.qy; o[6] = (float)b.qz;
        o[19] = (float)b.vw.x; o[20] = (float)b.vw.y; o[21] = (float)b.vw.z;
        o[22] = (float)b.w.x; o[23] = (float)b.w.y; o[24] = (float)b.w.z;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        o[7 + 3 * leg + j] = (float)lg.q[j];
        o[25 + 3 * leg + j] = (float)lg.qd[j];
    }
}

// The contact terms of base_contact below, arranged for fewer instructions: with
// J = [-(r x), I] and g = [r x n; n]
// the damping block is dt (eta J^T J + (c - eta) g g^T) and the right side gains
// dt [r x F; F].  dt eta and dt (c - eta) are folded into the operands first, so each
// entry is one or two fused multiply-adds.
template <typename S>
__device__ __forceinline__ void base_contact_folded(S eta, S c, V3<S> r, V3<S> n, V3<S> F, S dt, S* Q, S* rb)
{
    const V3<S> g0 = cross(r, n);
    const S de = dt * eta, dce = dt * (c - eta);
    const S ga[6] = {g0.x, g0.y, g0.z, n.x, n.y, n.z};
    S gs[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) gs[i] = dce * ga[i];
    const S rv[3] = {r.x, r.y, r.z};
    const S er[3] = {de * r.x, de * r.y, de * r.z};
    const S drr = de * dot(r, r);
    // angular block: de (|r|^2 I - r r^T) + dce g0 g0^T
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const S q = Q[s6(i, j)] + gs[i] * ga[j] - er[i] * rv[j];
            Q[s6(i, j)] = (i == j) ? q + drr : q;
        }
    // coupling block: de [r x] + dce g0 n^T ([r x] = {{0, -rz, ry}, {rz, 0, -rx}, {-ry, rx, 0}})
    Q[s6(0, 3)] += gs[0] * ga[3];
    Q[s6(0, 4)] += gs[0] * ga[4] - er[2];
    Q[s6(0, 5)] += gs[0] * ga[5] + er[1];
    Q[s6(1, 3)] += gs[1] * ga[3] + er[2];
    Q[s6(1, 4)] += gs[1] * ga[4];
    Q[s6(1, 5)] += gs[1] * ga[5] - er[0];
    Q[s6(2, 3)] += gs[2] * ga[3] - er[1];
    Q[s6(2, 4)] += gs[2] * ga[4] + er[0];
    Q[s6(2, 5)] += gs[2] * ga[5];
    // linear block: de I + dce n n^T
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const S q = Q[s6(3 + i, 3 + j)] + gs[3 + i] * ga[3 + j];
            Q[s6(3 + i, 3 + j)] = (i == j) ? q + de : q;
        }
    const V3<S> m = cross(r, F);
    rb[0] += dt * m.x; rb[1] += dt * m.y; rb[2] += dt * m.z;
    rb[3] += dt * F.x; rb[4] += dt * F.y; rb[5] += dt * F.z;
}

// contribution of a contact at trunk-frame point r (normal n, force F, secant eta) to
// the base rows: 6x6 damping block and generalized force
template <typename R>
__device__ __forceinline__ void base_contact(R eta, R c, V3<R> r, V3<R> n, V3<R> F, R dt, R* Q, R* rb)
{
    // J = [-(r x), I]; J^T D J = eta J^T J + (c - eta) g g^T, g = [r x n; n]
    const V3<R> g0 = cross(r, n);
    const R ce = c - eta;
    const R rr = dot(r, r);
    const R ga[6] = {g0.x, g0.y, g0.z, n.x, n.y, n.z};
    const R rv[3] = {r.x, r.y, r.z};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            Q[s6(i, j)] += dt * (eta * ((i == j ? rr : R(0)) - rv[i] * rv[j]) + ce * ga[i] * ga[j]);
    const R rx[9] = {R(0), -r.z, r.y, r.z, R(0), -r.x, -r.y, r.x, R(0)};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Q[s6(i, 3 + j)] += dt * (eta * rx[3 * i + j] + ce * ga[i] * ga[3 + j]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) Q[s6(3 + i, 3 + j)] += dt * ((i == j ? eta : R(0)) + ce * ga[3 + i] * ga[3 + j]);
    const V3<R> m = cross(r, F);
    rb[0] += dt * m.x; rb[1] += dt * m.y; rb[2] += dt * m.z;
    rb[3] += dt * F.x; rb[4] += dt * F.y; rb[5] += dt * F.z;
}

// FP32: the folded form above (FP64 keeps the original order of operations)
__device__ __forceinline__ void base_contact(float eta, float c, V3<float> r, V3<float> n, V3<float> F, float dt,
                                             float* Q, float* rb)
{
    base_contact_folded(eta, c, r, n, F, dt, Q, rb);
}

// 3x3 SPD Cholesky (lower) and solves
template <typename R>
struct Chol3 {
    R l10, l20, l21, i00, i11, i22;
};
template <typename R>
__device__ __forceinline__ Chol3<R> chol3(R a00, R a10, R a11, R a20, R a21, R a22)
{
    Chol3<R> c;
    const R l00 = m_sqrt(a00);
    c.i00 = R(1) / l00;
    c.l10 = a10 * c.i00;
    c.l20 = a20 * c.i00;
    const R l11 = m_sqrt(a11 - c.l10 * c.l10);
    c.i11 = R(1) / l11;
    c.l21 = (a21 - c.l20 * c.l10) * c.i11;
    const R l22 = m_sqrt(a22 - c.l20 * c.l20 - c.l21 * c.l21);
    c.i22 = R(1) / l22;
    return c;
}
template <typename R>
__device__ __forceinline__ void solve3(const Chol3<R>& c, R& b0, R& b1, R& b2)
{
    const R y0 = b0 * c.i00;
    const R y1 = (b1 - c.l10 * y0) * c.i11;
    const R y2 = (b2 - c.l20 * y0 - c.l21 * y1) * c.i22;
    b2 = y2 * c.i22;
    b1 = (y1 - c.l21 * b2) * c.i11;
    b0 = (y0 - c.l10 * b1 - c.l20 * b2) * c.i00;
}

// in-register 6x6 Cholesky of the packed symmetric Q, solving Q x = r in place
template <typename R>
__device__ __forceinline__ void chol6_solve(const R* Q, R* r)
{
    R L[21];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        R s = Q[s6(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= L[s6(j, k)] * L[s6(j, k)];
        const R id = R(1) / m_sqrt(s);
        L[s6(j, j)] = id;  // the reciprocal of the diagonal
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            R t = Q[s6(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= L[s6(i, k)] * L[s6(j, k)];
            L[s6(i, j)] = t * id;
        }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        R s = r[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[s6(i, k)] * r[k];
        r[i] = s * L[s6(i, i)];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        R s = r[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= L[s6(k, i)] * r[k];
        r[i] = s * L[s6(i, i)];
    }
}

// per-leg geometry, in trunk coordinates
template <typename R>
struct LegGeo {
    V3<R> ey, d1, d2, h, pk, pf, c1, c2;
};

// accumulators of one lane's leg (implicit system rows)
template <typename R>
struct LegSys {
    R A00, A01, A02, A11, A12, A22;  // A_ll
    R C[3][6];                       // A_l0
    R rl[3];                         // dt (tau + J^T F - b), joints
};

// a contact on this leg's calf at trunk-frame point r; vo is the velocity of the other
// body's material point there (trunk coordinates, zero for static geometry) and n points
// toward the robot.  Returns the force on the robot and the friction secant.
template <typename R>
__device__ __forceinline__ void leg_contact(const ModelT<R>& M, const LegGeo<R>& G, V3<R> vb, V3<R> w,
                                            const R qd[3], R delta, V3<R> n, V3<R> r, V3<R> vo, R dt, R* Q, R* rb,
                                            LegSys<R>& S, V3<R>& F, R& eta)
{
    const V3<R> ex = v3(R(1), R(0), R(0));
    const V3<R> ja = cross(ex, r - G.h), jf = cross(G.ey, r - G.h), jk = cross(G.ey, r - G.pk);
    const V3<R> vc = vb + cross(w, r) + qd[0] * ja + qd[1] * jf + qd[2] * jk - vo;
    contact_law(M, delta, n, vc, F, eta);
    const R ce = M.cc - eta;
    base_contact(eta, M.cc, r, n, F, dt, Q, rb);
    const R gj[3] = {dot(ja, n), dot(jf, n), dot(jk, n)};
    const V3<R> jv[3] = {ja, jf, jk};
    const V3<R> gA = cross(r, n);
    const R g0[6] = {gA.x, gA.y, gA.z, n.x, n.y, n.z};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const V3<R> rxj = cross(r, jv[j]);
        const R jb[6] = {rxj.x, rxj.y, rxj.z, jv[j].x, jv[j].y, jv[j].z};
#pragma unroll
        for (int i = 0; i < 6; ++i) S.C[j][i] += dt * (eta * jb[i] + ce * g0[i] * gj[j]);
        S.rl[j] += dt * dot(jv[j], F);
    }
    S.A00 += dt * (eta * dot(ja, ja) + ce * gj[0] * gj[0]);
    S.A01 += dt * (eta * dot(ja, jf) + ce * gj[0] * gj[1]);
    S.A02 += dt * (eta * dot(ja, jk) + ce * gj[0] * gj[2]);
    S.A11 += dt * (eta * dot(jf, jf) + ce * gj[1] * gj[1]);
    S.A12 += dt * (eta * dot(jf, jk) + ce * gj[1] * gj[2]);
    S.A22 += dt * (eta * dot(jk, jk) + ce * gj[2] * gj[2]);
}

// a contact on the trunk at trunk-frame point r (vo, n as for leg_contact)
template <typename R>
__device__ __forceinline__ void trunk_contact(const ModelT<R>& M, V3<R> vb, V3<R> w, R delta, V3<R> n, V3<R> r,
                                              V3<R> vo, R dt, R* Q, R* rb, V3<R>& F, R& eta)
{
    const V3<R> vc = vb + cross(w, r) - vo;
    contact_law(M, delta, n, vc, F, eta);
    base_contact(eta, M.cc, r, n, F, dt, Q, rb);
}

// ------------------------------------------------------------------------------
// free box (pushing scene): rigid body with generalized velocity [w_b, v_l] in its own
// body coordinates (v_l = R_b^T v_world), solved like the trunk's base block
// ------------------------------------------------------------------------------
template <typename R>
struct BoxS {
    V3<R> p;
    R qw, qx, qy, qz;
    V3<R> vw, w;
};
template <typename R>
struct BoxFrame {
    M33<R> Rb;
    V3<R> vl;  // body-frame linear velocity
};
template <typename R>
__device__ __forceinline__ void load_box(const float* __restrict__ x, BoxS<R>& bx)
{
    bx.p = v3<R>(x[37], x[38], x[39]);
    bx.qw = x[40]; bx.qx = x[41]; bx.qy = x[42]; bx.qz = x[43];
    bx.vw = v3<R>(x[44], x[45], x[46]);
    bx.w = v3<R>(x[47], x[48], x[49]);
}
template <typename R>
__device__ __forceinline__ void store_box(float* __restrict__ o, const BoxS<R>& bx)
{
    o[37] = (float)bx.p.x; o[38] = (float)bx.p.y; o[39] = (float)bx.p.z;
    o[40] = (float)bx.qw; o[41] = (float)bx.qx; o[42] = (float)bx.qy; o[43] = (float)bx.qz;
    o[44] = (float)bx.vw.x; o[45] = (float)bx.vw.y; o[46] = (float)bx.vw.z;
    o[47] = (float)bx.w.x; o[48] = (float)bx.w.y; o[49] = (float)bx.w.z;
}
template <typename R>
__device__ __forceinline__ void round_box(BoxS<R>& bx)
{
    bx.p = v3(to_f32(bx.p.x), to_f32(bx.p.y), to_f32(bx.p.z));
    bx.qw = to_f32(bx.qw); bx.qx = to_f32(bx.qx); bx.qy = to_f32(bx.qy); bx.qz = to_f32(bx.qz);
    bx.vw = v3(to_f32(bx.vw.x), to_f32(bx.vw.y), to_f32(bx.vw.z));
    bx.w = v3(to_f32(bx.w.x), to_f32(bx.w.y), to_f32(bx.w.z));
}
// world velocity of the box's material point at world position x
template <typename R>
__device__ __forceinline__ V3<R> box_point_vel(const BoxS<R>& bx, const BoxFrame<R>& bf, V3<R> x)
{
    return bx.vw + mul(bf.Rb, cross(bx.w, mulT(bf.Rb, x - bx.p)));
}
// the box's share of a contact: force Fw (world) on the box at world point x, damping
// secant eta along normal nw (sign irrelevant), into the box's 6x6 system
template <typename R>
__device__ __forceinline__ void box_share(const ModelT<R>& M, const BoxS<R>& bx, const BoxFrame<R>& bf, V3<R> x,
                                          V3<R> nw, V3<R> Fw, R eta, R dt, R* Qb, R* rbx)
{
    base_contact(eta, M.cc, mulT(bf.Rb, x - bx.p), mulT(bf.Rb, nw), mulT(bf.Rb, Fw), dt, Qb, rbx);
}
// quaternion update q <- normalize(q (x) exp(dt w / 2)) (body-frame angular velocity)
template <typename R>
__device__ __forceinline__ void quat_step(R& qw, R& qx, R& qy, R& qz, V3<R> w, R dt)
{
    const V3<R> ph = (R(0.5) * dt) * w;
    const R a = m_sqrt(dot(ph, ph));
    R sc, dw;
    quat_exp(a, &sc, &dw);
    const R dx = sc * ph.x, dy = sc * ph.y, dz = sc * ph.z;
    const R nw = qw * dw - qx * dx - qy * dy - qz * dz;
    const R nx = qw * dx + qx * dw + qy * dz - qz * dy;
    const R ny = qw * dy - qx * dz + qy * dw + qz * dx;
    const R nz = qw * dz + qx * dy - qy * dx + qz * dw;
    const R inv = R(1) / m_sqrt(nw * nw + nx * nx + ny * ny + nz * nz);
    qw = nw * inv; qx = nx * inv; qy = ny * inv; qz = nz * inv;
}

// ------------------------------------------------------------------------------
// one dynamics step of one sample; this lane owns leg `leg`.
// u: this leg's 3 joint targets.  tau2 receives (in all 4 lanes) sum over the robot
// of tau^2.
// ------------------------------------------------------------------------------
template <int SCENE, typename R>
__device__ __forceinline__ void quad_step(const ModelT<R>& M, const float* __restrict__ hf, R dt, R kp, R kd,
                                          int leg, Base<R>& b, Leg<R>& lg, BoxS<R>& bx, const R u[3], R& tau2)
{
    R tau[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) tau[j] = kp * (u[j] - lg.q[j]) - kd * lg.qd[j];
    const R t2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];

    const M33<R> Rm = quat_R(b.qw, b.qx, b.qy, b.qz);
    const V3<R> w = b.w;
    const V3<R> vb = mulT(Rm, b.vw);
    const V3<R> gb = (-M.g) * v3(Rm.m[6], Rm.m[7], Rm.m[8]);  // gravity in trunk coordinates

    // ---- leg kinematics in trunk coordinates
    LegGeo<R> G;
    R sa, ca, sf, cf, s12, c12;
    m_sincos(lg.q[0], &sa, &ca);
    m_sincos(lg.q[1], &sf, &cf);
    m_sincos(lg.q[1] + lg.q[2], &s12, &c12);
    const V3<R> ex = v3(R(1), R(0), R(0));
    G.ey = v3(R(0), ca, sa);
    G.d1 = v3(-sf, sa * cf, -ca * cf);
    G.d2 = v3(-s12, sa * c12, -ca * c12);
    G.h = v3((leg < 2) ? M.hip_x : -M.hip_x, (leg & 1) ? -M.hip_y : M.hip_y, R(0));
    G.pk = G.h + M.l1 * G.d1;
    G.pf = G.pk + M.l2 * G.d2;
    G.c1 = G.h + (R(0.5) * M.l1) * G.d1;
    G.c2 = G.pk + (R(0.5) * M.l2) * G.d2;
    const V3<R> ey = G.ey, d1 = G.d1, d2 = G.d2, h = G.h, pk = G.pk, c1 = G.c1, c2 = G.c2;
    const R dqa = lg.qd[0], dqf = lg.qd[1], dqk = lg.qd[2];

    // ---- mass matrix: base block (this leg's part), coupling columns, leg block
    R Q[21];
#pragma unroll
    for (int i = 0; i < 21; ++i) Q[i] = R(0);
    {
        const R r1 = dot(c1, c1), r2 = dot(c2, c2);
        const R cv1[3] = {c1.x, c1.y, c1.z}, cv2[3] = {c2.x, c2.y, c2.z};
        const R d1v[3] = {d1.x, d1.y, d1.z}, d2v[3] = {d2.x, d2.y, d2.z};
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                const R I = (i == j) ? R(1) : R(0);
                Q[s6(i, j)] = M.k1 * (I - d1v[i] * d1v[j]) + M.k2 * (I - d2v[i] * d2v[j]) +
                              M.m1 * (r1 * I - cv1[i] * cv1[j]) + M.m2 * (r2 * I - cv2[i] * cv2[j]);
            }
        const V3<R> hl = M.m1 * c1 + M.m2 * c2;  // ang-lin block [hl x]
        Q[s6(0, 4)] = -hl.z; Q[s6(0, 5)] = hl.y;
        Q[s6(1, 3)] = hl.z;  Q[s6(1, 5)] = -hl.x;
        Q[s6(2, 3)] = -hl.y; Q[s6(2, 4)] = hl.x;
    }
    LegSys<R> S;
    {
        // coupling columns h_j = [L_O; P] for unit rate of joint j (abduction, flexion, knee)
        const V3<R> ua1 = cross(ex, c1 - h), ua2 = cross(ex, c2 - h);
        const V3<R> uf1 = cross(ey, c1 - h), uf2 = cross(ey, c2 - h);
        const V3<R> uk2 = cross(ey, c2 - pk);
        const V3<R> Pa = M.m1 * ua1 + M.m2 * ua2;
        const V3<R> La = M.m1 * cross(c1, ua1) + M.m2 * cross(c2, ua2) + rod_I(M.k1, d1, ex) + rod_I(M.k2, d2, ex);
        const V3<R> Pf = M.m1 * uf1 + M.m2 * uf2;
        const V3<R> Lf = M.m1 * cross(c1, uf1) + M.m2 * cross(c2, uf2) + rod_I(M.k1, d1, ey) + rod_I(M.k2, d2, ey);
        const V3<R> Pk = M.m2 * uk2;
        const V3<R> Lk = M.m2 * cross(c2, uk2) + rod_I(M.k2, d2, ey);
        const V3<R> Ls[3] = {La, Lf, Lk}, Ps[3] = {Pa, Pf, Pk};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            S.C[j][0] = Ls[j].x; S.C[j][1] = Ls[j].y; S.C[j][2] = Ls[j].z;
            S.C[j][3] = Ps[j].x; S.C[j][4] = Ps[j].y; S.C[j][5] = Ps[j].z;
        }
        // leg block M_jk = S_j . h_k (j <= k), motion axes S_j = [a_j; o_j x a_j]
        const V3<R> oxa_a = cross(h, ex), oxa_f = cross(h, ey), oxa_k = cross(pk, ey);
        S.A00 = dot(ex, La) + dot(oxa_a, Pa);
        S.A01 = dot(ex, Lf) + dot(oxa_a, Pf);
        S.A02 = dot(ex, Lk) + dot(oxa_a, Pk);
        S.A11 = dot(ey, Lf) + dot(oxa_f, Pf);
        S.A12 = dot(ey, Lk) + dot(oxa_f, Pk);
        S.A22 = dot(ey, Lk) + dot(oxa_k, Pk);
    }

    // ---- bias forces (zero generalized acceleration, gravity)
    R rb[6];
    {
        const V3<R> w1 = w + dqa * ex + dqf * ey;
        const V3<R> al1 = dqa * cross(w, ex) + dqf * cross(w + dqa * ex, ey);
        const V3<R> ah = cross(w, cross(w, h));
        const V3<R> r1 = c1 - h, rk = pk - h;
        const V3<R> ac1 = ah + cross(al1, r1) + cross(w1, cross(w1, r1));
        const V3<R> apk = ah + cross(al1, rk) + cross(w1, cross(w1, rk));
        const V3<R> w2 = w1 + dqk * ey;
        const V3<R> al2 = al1 + dqk * cross(w1, ey);
        const V3<R> r2 = c2 - pk;
        const V3<R> ac2 = apk + cross(al2, r2) + cross(w2, cross(w2, r2));
        const V3<R> F1 = M.m1 * (ac1 - gb), F2 = M.m2 * (ac2 - gb);
        const V3<R> N1 = rod_I(M.k1, d1, al1) + cross(w1, rod_I(M.k1, d1, w1));
        const V3<R> N2 = rod_I(M.k2, d2, al2) + cross(w2, rod_I(M.k2, d2, w2));
        const V3<R> Tk = N2 + cross(r2, F2);
        const V3<R> Th = N1 + cross(r1, F1) + N2 + cross(c2 - h, F2);
        const V3<R> Tb = N1 + N2 + cross(c1, F1) + cross(c2, F2);
        const V3<R> Fb = F1 + F2;
        rb[0] = -dt * Tb.x; rb[1] = -dt * Tb.y; rb[2] = -dt * Tb.z;
        rb[3] = -dt * Fb.x; rb[4] = -dt * Fb.y; rb[5] = -dt * Fb.z;
        S.rl[0] = dt * (tau[0] - dot(ex, Th));
        S.rl[1] = dt * (tau[1] - dot(ey, Th));
        S.rl[2] = dt * (tau[2] - dot(ey, Tk));
    }
    S.A00 += dt * kd; S.A11 += dt * kd; S.A22 += dt * kd;  // joint damping (implicit)

    // ---- free box frame and its implicit-system accumulators (pushing scene)
    [[maybe_unused]] BoxFrame<R> bf;
    [[maybe_unused]] R Qb[21], rbx[6];
    const V3<R> zero = v3(R(0), R(0), R(0));
    V3<R> F;
    R eta;
    if constexpr (SCENE == 3) {
        bf.Rb = quat_R(bx.qw, bx.qx, bx.qy, bx.qz);
#pragma unroll
        for (int i = 0; i < 21; ++i) Qb[i] = R(0);
#pragma unroll
        for (int i = 0; i < 6; ++i) rbx[i] = R(0);
    }

    // ---- foot (sphere on the calf) against terrain and the static or free box
    {
        const V3<R> pfw = b.p + mul(Rm, G.pf);
        R delta;
        V3<R> nw;
        if (terrain<SCENE>(M, hf, pfw, M.foot_r, delta, nw)) {
            const V3<R> n = mulT(Rm, nw);
            leg_contact(M, G, vb, w, lg.qd, delta, n, G.pf - M.foot_r * n, zero, dt, Q, rb, S, F, eta);
        }
        if constexpr (SCENE == 2) {
            const V3<R> l = pfw - v3(M.sb_cx, M.sb_cy, M.sb_cz);
            if (sphere_aabox(l, M.foot_r, v3(M.sb_hx, M.sb_hy, M.sb_hz), delta, nw)) {
                const V3<R> n = mulT(Rm, nw);
                leg_contact(M, G, vb, w, lg.qd, delta, n, G.pf - M.foot_r * n, zero, dt, Q, rb, S, F, eta);
            }
        }
        if constexpr (SCENE == 3) {
            V3<R> nl;
            if (sphere_aabox(mulT(bf.Rb, pfw - bx.p), M.foot_r, v3(M.bx_hx, M.bx_hy, M.bx_hz), delta, nl)) {
                const V3<R> nb = mul(bf.Rb, nl);  // box -> foot (world)
                const V3<R> pcw = pfw - M.foot_r * nb;
                const V3<R> n = mulT(Rm, nb);
                const V3<R> vo = mulT(Rm, box_point_vel(bx, bf, pcw));
                leg_contact(M, G, vb, w, lg.qd, delta, n, G.pf - M.foot_r * n, vo, dt, Q, rb, S, F, eta);
                box_share(M, bx, bf, pcw, nb, R(-1) * mul(Rm, F), eta, dt, Qb, rbx);
            }
        }
    }
    // ---- two trunk corners per lane
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
        const int ci = 2 * leg + cc;
        const V3<R> rloc = v3((ci & 1 ? R(0.5) : R(-0.5)) * M.tsx, (ci & 2 ? R(0.5) : R(-0.5)) * M.tsy,
                              (ci & 4 ? R(0.5) : R(-0.5)) * M.tsz);
        const V3<R> pw = b.p + mul(Rm, rloc);
        R delta;
        V3<R> nw;
        if (terrain<SCENE>(M, hf, pw, R(0), delta, nw))
            trunk_contact(M, vb, w, delta, mulT(Rm, nw), rloc, zero, dt, Q, rb, F, eta);
        if constexpr (SCENE == 2) {
            if (point_aabox(pw - v3(M.sb_cx, M.sb_cy, M.sb_cz), v3(M.sb_hx, M.sb_hy, M.sb_hz), delta, nw))
                trunk_contact(M, vb, w, delta, mulT(Rm, nw), rloc, zero, dt, Q, rb, F, eta);
        }
        if constexpr (SCENE == 3) {
            V3<R> nl;
            if (point_aabox(mulT(bf.Rb, pw - bx.p), v3(M.bx_hx, M.bx_hy, M.bx_hz), delta, nl)) {
                const V3<R> nb = mul(bf.Rb, nl);  // box face normal, toward the corner
                const V3<R> vo = mulT(Rm, box_point_vel(bx, bf, pw));
                trunk_contact(M, vb, w, delta, mulT(Rm, nb), rloc, vo, dt, Q, rb, F, eta);
                box_share(M, bx, bf, pw, nb, R(-1) * mul(Rm, F), eta, dt, Qb, rbx);
            }
        }
    }
    // ---- two box corners per lane: against the trunk and the ground
    if constexpr (SCENE == 3) {
        const V3<R> th = v3(R(0.5) * M.tsx, R(0.5) * M.tsy, R(0.5) * M.tsz);
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const int ci = 2 * leg + cc;
            const V3<R> cl = v3(ci & 1 ? M.bx_hx : -M.bx_hx, ci & 2 ? M.bx_hy : -M.bx_hy, ci & 4 ? M.bx_hz : -M.bx_hz);
            const V3<R> xw = bx.p + mul(bf.Rb, cl);
            R delta;
            V3<R> nt;
            const V3<R> lt = mulT(Rm, xw - b.p);
            if (point_aabox(lt, th, delta, nt)) {  // nt: trunk face normal, toward the box corner
                const V3<R> vo = mulT(Rm, box_point_vel(bx, bf, xw));
                trunk_contact(M, vb, w, delta, R(-1) * nt, lt, vo, dt, Q, rb, F, eta);
                box_share(M, bx, bf, xw, mul(Rm, nt), R(-1) * mul(Rm, F), eta, dt, Qb, rbx);
            }
            V3<R> nw;
            if (terrain<SCENE>(M, hf, xw, R(0), delta, nw)) {
                contact_law(M, delta, nw, box_point_vel(bx, bf, xw), F, eta);
                box_share(M, bx, bf, xw, nw, F, eta, dt, Qb, rbx);
            }
        }
    }

    // ---- eliminate this leg: W = A_ll^-1 A_l0, y = A_ll^-1 r_l
    const Chol3<R> L3 = chol3(S.A00, S.A01, S.A11, S.A02, S.A12, S.A22);
    R W[3][6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        R x0 = S.C[0][i], x1 = S.C[1][i], x2 = S.C[2][i];
        solve3(L3, x0, x1, x2);
        W[0][i] = x0; W[1][i] = x1; W[2][i] = x2;
    }
    R y0 = S.rl[0], y1 = S.rl[1], y2 = S.rl[2];
    solve3(L3, y0, y1, y2);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
        for (int j = i; j < 6; ++j) Q[s6(i, j)] -= S.C[0][i] * W[0][j] + S.C[1][i] * W[1][j] + S.C[2][i] * W[2][j];
        rb[i] -= S.C[0][i] * y0 + S.C[1][i] * y1 + S.C[2][i] * y2;
    }

    // ---- sum over the four legs (quad all-reduce)
#pragma unroll
    for (int i = 0; i < 21; ++i) Q[i] = quad_sum(Q[i]);
#pragma unroll
    for (int i = 0; i < 6; ++i) rb[i] = quad_sum(rb[i]);
    tau2 = quad_sum(t2);
    if constexpr (SCENE == 3) {
#pragma unroll
        for (int i = 0; i < 21; ++i) Qb[i] = quad_sum(Qb[i]);
#pragma unroll
        for (int i = 0; i < 6; ++i) rbx[i] = quad_sum(rbx[i]);
    }

    // ---- trunk's own terms: inertia, total mass, gyroscopic and gravity bias
    Q[s6(0, 0)] += M.I0x; Q[s6(1, 1)] += M.I0y; Q[s6(2, 2)] += M.I0z;
    Q[s6(3, 3)] += M.mtot; Q[s6(4, 4)] += M.mtot; Q[s6(5, 5)] += M.mtot;
    {
        const V3<R> Iw = v3(M.I0x * w.x, M.I0y * w.y, M.I0z * w.z);
        const V3<R> gy = cross(w, Iw);
        rb[0] -= dt * gy.x; rb[1] -= dt * gy.y; rb[2] -= dt * gy.z;
        rb[3] += dt * M.m0 * gb.x; rb[4] += dt * M.m0 * gb.y; rb[5] += dt * M.m0 * gb.z;
    }
    chol6_solve(Q, rb);  // rb <- base increment [d omega; d v_b]

    // ---- back-substitute this leg and integrate (semi-implicit Euler)
    R dq[3] = {y0, y1, y2};
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 6; ++i) dq[j] -= W[j][i] * rb[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        lg.qd[j] += dq[j];
        lg.q[j] += dt * lg.qd[j];
    }
    b.w = b.w + v3(rb[0], rb[1], rb[2]);
    b.vw = b.vw + mul(Rm, v3(rb[3], rb[4], rb[5]));
    b.p = b.p + dt * b.vw;
    quat_step(b.qw, b.qx, b.qy, b.qz, b.w, dt);

    // ---- free box: own 6x6 system (inertia, gyroscopic and gravity terms), then integrate
    if constexpr (SCENE == 3) {
        Qb[s6(0, 0)] += M.bx_Ix; Qb[s6(1, 1)] += M.bx_Iy; Qb[s6(2, 2)] += M.bx_Iz;
        Qb[s6(3, 3)] += M.bx_m; Qb[s6(4, 4)] += M.bx_m; Qb[s6(5, 5)] += M.bx_m;
        const V3<R> wbx = bx.w;
        const V3<R> gy = cross(wbx, v3(M.bx_Ix * wbx.x, M.bx_Iy * wbx.y, M.bx_Iz * wbx.z));
        const V3<R> gl = (-M.g) * v3(bf.Rb.m[6], bf.Rb.m[7], bf.Rb.m[8]);
        rbx[0] -= dt * gy.x; rbx[1] -= dt * gy.y; rbx[2] -= dt * gy.z;
        rbx[3] += dt * M.bx_m * gl.x; rbx[4] += dt * M.bx_m * gl.y; rbx[5] += dt * M.bx_m * gl.z;
        chol6_solve(Qb, rbx);
        bx.w = bx.w + v3(rbx[0], rbx[1], rbx[2]);
        bx.vw = bx.vw + mul(bf.Rb, v3(rbx[3], rbx[4], rbx[5]));
        bx.p = bx.p + dt * bx.vw;
        quat_step(bx.qw, bx.qx, bx.qy, bx.qz, bx.w, dt);
    }
}

// running cost at the post-step state (all lanes compute the same value): height,
// uprightness, torque, and forward velocity -- or, in the pushing scene, the distance
// of the trunk to the box and of the box to its goal (xy)
template <int SCENE, typename R>
__device__ __forceinline__ R stage_cost(const DevParams& P, const Base<R>& b, const BoxS<R>& bx, R tau2)
{
    const R Rzz = R(1) - R(2) * (b.qx * b.qx + b.qy * b.qy);
    const R dz = b.p.z - R(P.h_ref);
    R l = R(P.w_h) * dz * dz + R(P.w_o) * (R(1) - Rzz * Rzz) + R(P.w_tau) * tau2;
    if constexpr (SCENE == 3) {
        const R ex = b.p.x - bx.p.x, ey = b.p.y - bx.p.y;
        const R gx = bx.p.x - R(P.goal_x), gy = bx.p.y - R(P.goal_y);
        l += R(P.w_reach) * (ex * ex + ey * ey) + R(P.w_box) * (gx * gx + gy * gy);
    } else {
        const R dv = b.vw.x - R(P.v_ref);
        l += R(P.w_v) * dv * dv;
    }
    return l;
}

}  // namespace mppi
