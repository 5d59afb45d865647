// Lane-split rollout for gfx950: one sample per 16 lanes (four per leg), four samples per
// 64-lane workgroup, so that K = 4096 samples occupy 1024 waves -- one on every SIMD of
// the chip -- where the quad kernel (one lane per leg) leaves three SIMDs in four idle.
//
// The per-step instruction stream of a wave is what sets the time on a SIMD that holds
// one wave, so the split pays only where the 16 lanes run the same instructions on
// different data:
//   * knot interpolation: lane s < 3 of a leg interpolates joint s; the three targets are
//     broadcast in the quad (DPP quad_perm);
//   * trigonometry: lane s evaluates the sine and cosine of the leg's angle s (abduction,
//     flexion, flexion + knee) and broadcasts them;
//   * contacts with the trunk corners and the free box's corners: lane g < 8 takes trunk
//     corner g, lane g >= 8 box corner g - 8 (the quad kernel takes two of each per lane);
//   * the two 6x6 solves of the pushing scene: even lanes solve the trunk's system, odd
//     lanes the box's, from selected operands, and swap results with their neighbour.
// The leg's kinematics, mass-matrix and bias terms, its foot contacts and the elimination
// of its 3x3 block run in all four lanes of the leg (only lane 0's copy enters the
// sums).  The trunk and box systems (Sec. III-A's dynamics step: (M + dt D) dv = dt f,
// the legs eliminated first) are summed over the 16 lanes through LDS: every lane writes
// its partial terms, lane g adds entries g, g + 16, ... of all 16 lanes in a fixed order,
// and every lane reads the sums back.  The results do not depend on timing.
//
// The step computes the same discretisation as the quad kernel in the same arithmetic
// type R (the state is FP32 between steps); only summation orders differ.
#include "mppi_device.h"
#include "mppi_launch.h"

namespace mppi {
namespace r16 {

constexpr int kSamples = 4;     // samples per workgroup (one wave)
constexpr int kNVMax = 55;      // summed values: trunk system 21 + 6, torque^2, box system 21 + 6
constexpr int kPitch = 20;      // LDS row pitch of one summed value over the 16 lanes (16 used)
constexpr int kSumPitch = 64;   // per-sample row of the sums

template <int SCENE>
__device__ __forceinline__ constexpr int n_summed()
{
    return SCENE == 3 ? 55 : 28;
}

// fixed-order sum of the 16 partials of one value
template <typename R>
__device__ __forceinline__ R sum16(const R* p)
{
    R a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = p[2 * i] + p[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = a[2 * i] + a[2 * i + 1];
    return (a[0] + a[1]) + (a[2] + a[3]);
}

template <typename R>
__device__ __forceinline__ R sel(bool c, R a, R b)
{
    return c ? a : b;
}

// ------------------------------------------------------------------------------
// one dynamics step of one sample; lane g (0..15) of the sample, leg g >> 2, sub-lane
// g & 3.  uj: the joint target this lane interpolated (joint g & 3 of its leg, lanes 3
// repeat joint 2).  red / sred: this sample's LDS rows.  tau2 receives sum tau^2.
// ------------------------------------------------------------------------------
template <int SCENE, typename R>
__device__ __forceinline__ void step16(const ModelT<R>& M, const float* __restrict__ hf, R dt, R kp, R kd, int g,
                                       Base<R>& b, Leg<R>& lg, BoxS<R>& bx, R uj, R* red, R* sred, R& tau2)
{
    const int leg = g >> 2, sub = g & 3;
    const R u[3] = {dpp<0x00>(uj), dpp<0x55>(uj), dpp<0xAA>(uj)};
    R tau[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) tau[j] = kp * (u[j] - lg.q[j]) - kd * lg.qd[j];
    const R t2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];

    const M33<R> Rm = quat_R(b.qw, b.qx, b.qy, b.qz);
    const V3<R> w = b.w;
    const V3<R> vb = mulT(Rm, b.vw);
    const V3<R> gb = (-M.g) * v3(Rm.m[6], Rm.m[7], Rm.m[8]);

    // ---- leg kinematics: lane `sub` evaluates angle sub of the leg, the quad shares them
    R sn, cs;
    {
        const R ang = (sub == 0) ? lg.q[0] : (sub == 1) ? lg.q[1] : lg.q[1] + lg.q[2];
        m_sincos(ang, &sn, &cs);
    }
    const R sa = dpp<0x00>(sn), ca = dpp<0x00>(cs);
    const R sf = dpp<0x55>(sn), cf = dpp<0x55>(cs);
    const R s12 = dpp<0xAA>(sn), c12 = dpp<0xAA>(cs);
    LegGeo<R> G;
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

    // ---- the leg's mass-matrix terms: base block, coupling columns, leg block
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
        const V3<R> hl = M.m1 * c1 + M.m2 * c2;
        Q[s6(0, 4)] = -hl.z; Q[s6(0, 5)] = hl.y;
        Q[s6(1, 3)] = hl.z;  Q[s6(1, 5)] = -hl.x;
        Q[s6(2, 3)] = -hl.y; Q[s6(2, 4)] = hl.x;
    }
    LegSys<R> S;
    {
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
        const V3<R> oxa_a = cross(h, ex), oxa_f = cross(h, ey), oxa_k = cross(pk, ey);
        S.A00 = dot(ex, La) + dot(oxa_a, Pa);
        S.A01 = dot(ex, Lf) + dot(oxa_a, Pf);
        S.A02 = dot(ex, Lk) + dot(oxa_a, Pk);
        S.A11 = dot(ey, Lf) + dot(oxa_f, Pf);
        S.A12 = dot(ey, Lk) + dot(oxa_f, Pk);
        S.A22 = dot(ey, Lk) + dot(oxa_k, Pk);
    }

    // ---- bias forces of the leg (zero generalized acceleration, gravity)
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
    S.A00 += dt * kd; S.A11 += dt * kd; S.A22 += dt * kd;

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

    // ---- the leg's foot against terrain and the static or free box
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
                const V3<R> nb = mul(bf.Rb, nl);
                const V3<R> pcw = pfw - M.foot_r * nb;
                const V3<R> n = mulT(Rm, nb);
                const V3<R> vo = mulT(Rm, box_point_vel(bx, bf, pcw));
                leg_contact(M, G, vb, w, lg.qd, delta, n, G.pf - M.foot_r * n, vo, dt, Q, rb, S, F, eta);
                box_share(M, bx, bf, pcw, nb, R(-1) * mul(Rm, F), eta, dt, Qb, rbx);
            }
        }
    }

    // ---- eliminate the leg: W = A_ll^-1 A_l0, y = A_ll^-1 r_l
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

    // the leg's terms are the same in its four lanes: only sub-lane 0's copy is summed
    const bool keep = sub == 0;
#pragma unroll
    for (int i = 0; i < 21; ++i) Q[i] = sel(keep, Q[i], R(0));
#pragma unroll
    for (int i = 0; i < 6; ++i) rb[i] = sel(keep, rb[i], R(0));
    if constexpr (SCENE == 3) {
#pragma unroll
        for (int i = 0; i < 21; ++i) Qb[i] = sel(keep, Qb[i], R(0));
#pragma unroll
        for (int i = 0; i < 6; ++i) rbx[i] = sel(keep, rbx[i], R(0));
    }

    // ---- one corner per lane: trunk corner g (g < 8), free-box corner g - 8 (g >= 8)
    if (g < 8) {
        const V3<R> rloc = v3((g & 1 ? R(0.5) : R(-0.5)) * M.tsx, (g & 2 ? R(0.5) : R(-0.5)) * M.tsy,
                              (g & 4 ? R(0.5) : R(-0.5)) * M.tsz);
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
                const V3<R> nb = mul(bf.Rb, nl);
                const V3<R> vo = mulT(Rm, box_point_vel(bx, bf, pw));
                trunk_contact(M, vb, w, delta, mulT(Rm, nb), rloc, vo, dt, Q, rb, F, eta);
                box_share(M, bx, bf, pw, nb, R(-1) * mul(Rm, F), eta, dt, Qb, rbx);
            }
        }
    } else if constexpr (SCENE == 3) {
        const int ci = g - 8;
        const V3<R> th = v3(R(0.5) * M.tsx, R(0.5) * M.tsy, R(0.5) * M.tsz);
        const V3<R> cl = v3(ci & 1 ? M.bx_hx : -M.bx_hx, ci & 2 ? M.bx_hy : -M.bx_hy, ci & 4 ? M.bx_hz : -M.bx_hz);
        const V3<R> xw = bx.p + mul(bf.Rb, cl);
        R delta;
        V3<R> nt;
        const V3<R> lt = mulT(Rm, xw - b.p);
        if (point_aabox(lt, th, delta, nt)) {
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

    // ---- sum the trunk (and box) systems and the squared torques over the 16 lanes
    constexpr int NV = n_summed<SCENE>();
    {
        R v[NV];
#pragma unroll
        for (int i = 0; i < 21; ++i) v[i] = Q[i];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[21 + i] = rb[i];
        v[27] = sel(keep, t2, R(0));
        if constexpr (SCENE == 3) {
#pragma unroll
            for (int i = 0; i < 21; ++i) v[28 + i] = Qb[i];
#pragma unroll
            for (int i = 0; i < 6; ++i) v[49 + i] = rbx[i];
        }
#pragma unroll
        for (int e = 0; e < NV; ++e) red[e * kPitch + g] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < (NV + 15) / 16; ++m) {
        const int e = g + 16 * m;
        if (e < NV) sred[e] = sum16(red + e * kPitch);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 21; ++i) Q[i] = sred[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) rb[i] = sred[21 + i];
    tau2 = sred[27];
    if constexpr (SCENE == 3) {
#pragma unroll
        for (int i = 0; i < 21; ++i) Qb[i] = sred[28 + i];
#pragma unroll
        for (int i = 0; i < 6; ++i) rbx[i] = sred[49 + i];
    }

    // ---- the trunk's own terms: inertia, total mass, gyroscopic and gravity bias
    Q[s6(0, 0)] += M.I0x; Q[s6(1, 1)] += M.I0y; Q[s6(2, 2)] += M.I0z;
    Q[s6(3, 3)] += M.mtot; Q[s6(4, 4)] += M.mtot; Q[s6(5, 5)] += M.mtot;
    {
        const V3<R> Iw = v3(M.I0x * w.x, M.I0y * w.y, M.I0z * w.z);
        const V3<R> gy = cross(w, Iw);
        rb[0] -= dt * gy.x; rb[1] -= dt * gy.y; rb[2] -= dt * gy.z;
        rb[3] += dt * M.m0 * gb.x; rb[4] += dt * M.m0 * gb.y; rb[5] += dt * M.m0 * gb.z;
    }
    if constexpr (SCENE != 3) {
        chol6_solve(Q, rb);  // rb <- trunk increment [d omega; d v_b]
    } else {
        // the box's own terms, then one 6x6 solve per lane: trunk on even lanes, box on
        // odd lanes; neighbours swap their results
        Qb[s6(0, 0)] += M.bx_Ix; Qb[s6(1, 1)] += M.bx_Iy; Qb[s6(2, 2)] += M.bx_Iz;
        Qb[s6(3, 3)] += M.bx_m; Qb[s6(4, 4)] += M.bx_m; Qb[s6(5, 5)] += M.bx_m;
        const V3<R> wbx = bx.w;
        const V3<R> gyb = cross(wbx, v3(M.bx_Ix * wbx.x, M.bx_Iy * wbx.y, M.bx_Iz * wbx.z));
        const V3<R> gl = (-M.g) * v3(bf.Rb.m[6], bf.Rb.m[7], bf.Rb.m[8]);
        rbx[0] -= dt * gyb.x; rbx[1] -= dt * gyb.y; rbx[2] -= dt * gyb.z;
        rbx[3] += dt * M.bx_m * gl.x; rbx[4] += dt * M.bx_m * gl.y; rbx[5] += dt * M.bx_m * gl.z;
        const bool odd = (g & 1) != 0;
        R Qs[21], rs[6];
#pragma unroll
        for (int i = 0; i < 21; ++i) Qs[i] = sel(odd, Qb[i], Q[i]);
#pragma unroll
        for (int i = 0; i < 6; ++i) rs[i] = sel(odd, rbx[i], rb[i]);
        chol6_solve(Qs, rs);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const R other = dpp<0xB1>(rs[i]);  // the neighbour's result (lanes 0<->1, 2<->3)
            rb[i] = sel(odd, other, rs[i]);
            rbx[i] = sel(odd, rs[i], other);
        }
    }

    // ---- back-substitute the leg and integrate (semi-implicit Euler)
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
    if constexpr (SCENE == 3) {
        bx.w = bx.w + v3(rbx[0], rbx[1], rbx[2]);
        bx.vw = bx.vw + mul(bf.Rb, v3(rbx[3], rbx[4], rbx[5]));
        bx.p = bx.p + dt * bx.vw;
        quat_step(bx.qw, bx.qx, bx.qy, bx.qz, bx.w, dt);
    }
}

}  // namespace r16

// ------------------------------------------------------------------------------
// rollout kernel: workgroup of 64 lanes = 4 samples x 16 lanes.  LDS: the summation rows
// [4][kNVMax][kPitch], the sums [4][kSumPitch], then the heightfield (scene 1).
// eps addressing as in the quad kernel: eps_in[n * eps_sn + d * eps_sd] when given,
// otherwise Philox noise stored to eps_out[d * K + n].
// ------------------------------------------------------------------------------
template <int SCENE, typename R>
__global__ __launch_bounds__(64) void rollout16_kernel(ModelT<R> Mg, DevParams P, const double* __restrict__ gB,
                                                       const float* __restrict__ ghf, const float* __restrict__ mu,
                                                       const float* __restrict__ x0,
                                                       const float* __restrict__ eps_in, int eps_sn, int eps_sd,
                                                       float* __restrict__ eps_out, float* __restrict__ costs,
                                                       float* __restrict__ traj)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    // the model's constants are read from LDS (values in vector registers), which keeps the
    // scalar registers for the kernel's pointers and loop state
    __shared__ ModelT<R> sM;
    R* red = reinterpret_cast<R*>(lds_raw);
    R* sred = red + r16::kSamples * r16::kNVMax * r16::kPitch;
    float* sHF = reinterpret_cast<float*>(sred + r16::kSamples * r16::kSumPitch);
    if (threadIdx.x == 0) sM = Mg;
    if constexpr (SCENE == 1) {
        const int cells = Mg.hf_nx * Mg.hf_ny;
        for (int i = threadIdx.x; i < cells; i += blockDim.x) sHF[i] = ghf[i];
    }
    __syncthreads();
    const ModelT<R>& M = sM;

    const int tid = threadIdx.x;
    const int g = tid & 15, grp = tid >> 4;
    const int leg = g >> 2, sub = g & 3;
    const int jl = sub < 3 ? sub : 2;  // this lane's joint of its leg
    const int n = blockIdx.x * r16::kSamples + grp;
    const bool valid = n < P.K;
    const int ns = valid ? n : P.K - 1;
    const int nk = P.nk;
    const R sigma = P.sigma;

    // knots of this lane's joint, theta = mu + sigma eps (sample 0 is the nominal)
    R th[kMaxKnots];
#pragma unroll
    for (int i = 0; i < kMaxKnots; ++i) {
        th[i] = R(0);
        if (i < nk) {
            const int d = (3 * leg + jl) * nk + i;
            R e;
            if (eps_in) {
                e = eps_in[(size_t)ns * eps_sn + (size_t)d * eps_sd];
            } else {
                e = gauss_elem<R>(P, (uint32_t)ns, (uint32_t)d);
                if (valid && sub < 3 && eps_out) eps_out[(size_t)d * P.K + n] = (float)e;
            }
            th[i] = R(mu[d]) + (ns ? sigma * e : R(0));
        }
    }

    Base<R> b;
    Leg<R> lg;
    BoxS<R> bx{};
    load_state(x0, leg, b, lg);
    if constexpr (SCENE == 3) load_box(x0, bx);
    float* tr = (traj && valid && sub == 0) ? traj + (size_t)n * (P.H + 1) * P.nx : nullptr;
    if (tr) {
        store_state(tr, leg, b, lg);
        if (SCENE == 3 && leg == 0) store_box(tr, bx);
    }

    R* my_red = red + grp * r16::kNVMax * r16::kPitch;
    R* my_sum = sred + grp * r16::kSumPitch;
    const R dt = P.dt, kp = P.kp, kd = P.kd;
    R L = R(0);
    for (int k = 0; k < P.H; ++k) {
        R uj = R(0);
#pragma unroll
        for (int i = 0; i < kMaxKnots; ++i)
            if (i < nk) uj += R(gB[k * nk + i]) * th[i];
        R tau2;
        r16::step16<SCENE, R>(M, sHF, dt, kp, kd, g, b, lg, bx, uj, my_red, my_sum, tau2);
        round_state(b, lg);
        if constexpr (SCENE == 3) round_box(bx);
        L += dt * stage_cost<SCENE>(P, b, bx, tau2);
        if (tr) {
            store_state(tr + (size_t)(k + 1) * P.nx, leg, b, lg);
            if (SCENE == 3 && leg == 0) store_box(tr + (size_t)(k + 1) * P.nx, bx);
        }
    }
    float Lf = (float)L;
    if (!(fabsf(Lf) <= 3.0e38f)) Lf = __int_as_float(0x7f800000);  // non-finite -> +inf
    if (valid && g == 0) costs[n] = Lf;
}

namespace r16 {

template <typename R>
size_t lds_bytes(int scene, int hf_cells)
{
    size_t b = sizeof(R) * ((size_t)kSamples * kNVMax * kPitch + (size_t)kSamples * kSumPitch);
    if (scene == 1) b += sizeof(float) * (size_t)hf_cells;
    return b;
}

template <typename R>
hipError_t launch_t(const ModelT<R>& M, const DevParams& P, const RolloutArgs& a, hipStream_t st)
{
    const int blocks = (P.K + kSamples - 1) / kSamples;
    const size_t lds = lds_bytes<R>(M.scene, M.hf_nx * M.hf_ny);
    if (lds > 65536) return hipErrorInvalidValue;
#define MPPI_LAUNCH_R16(S)                                                                                     \
    hipLaunchKernelGGL((rollout16_kernel<S, R>), dim3(blocks), dim3(64), lds, st, M, P, a.B, a.hf, a.mu, a.x0, \
                       a.eps_in, a.eps_sn, a.eps_sd, a.eps_out, a.costs, a.traj)
    switch (M.scene) {
    case 0: MPPI_LAUNCH_R16(0); break;
    case 1: MPPI_LAUNCH_R16(1); break;
    case 2: MPPI_LAUNCH_R16(2); break;
    case 3: MPPI_LAUNCH_R16(3); break;
    default: return hipErrorInvalidValue;
    }
#undef MPPI_LAUNCH_R16
    return hipGetLastError();
}

}  // namespace r16

bool rollout16_fits(int arith, int scene, int hf_cells)
{
    const size_t b = arith == 1 ? r16::lds_bytes<float>(scene, hf_cells) : r16::lds_bytes<double>(scene, hf_cells);
    return b <= 65536;
}

hipError_t launch_rollout16(const DevModelF& Mf, const DevModelD& Md, int arith, const DevParams& P,
                            const RolloutArgs& a, hipStream_t st)
{
    return arith == 1 ? r16::launch_t(Mf, P, a, st) : r16::launch_t(Md, P, a, st);
}

}  // namespace mppi
