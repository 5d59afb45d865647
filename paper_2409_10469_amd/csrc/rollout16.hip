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

template <typename R>
__device__ __forceinline__ V3<R> selv(bool c, V3<R> a, V3<R> b)
{
    return v3(c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z);
}

// pose and velocity of a rigid body (the trunk or the free box): rotation to world,
// position, world linear velocity, body-frame angular velocity
template <typename R>
struct Pose {
    M33<R> Rt;
    V3<R> p, vw, w;
};
template <typename R>
__device__ __forceinline__ V3<R> pose_point_vel(const Pose<R>& B, V3<R> x)
{
    return B.vw + mul(B.Rt, cross(B.w, mulT(B.Rt, x - B.p)));
}
template <typename R>
__device__ __forceinline__ Pose<R> sel_pose(bool c, const Pose<R>& a, const Pose<R>& b)
{
    Pose<R> o;
#pragma unroll
    for (int i = 0; i < 9; ++i) o.Rt.m[i] = c ? a.Rt.m[i] : b.Rt.m[i];
    o.p = selv(c, a.p, b.p);
    o.vw = selv(c, a.vw, b.vw);
    o.w = selv(c, a.w, b.w);
    return o;
}

template <typename T, typename U>
__device__ __forceinline__ V3<T> cv(V3<U> a)
{
    return V3<T>{T(a.x), T(a.y), T(a.z)};
}

// a contact on the leg's calf with weight wgt (1: applied, 0: nothing added).  The contact
// velocity and the law are evaluated in the geometry type R; the force and damping terms
// on the trunk's base rows and on the leg's joint rows accumulate in the system type S.
template <typename R, typename S>
__device__ __forceinline__ void leg_contact_w(const ModelT<R>& M, const LegGeo<R>& G, V3<R> vb, V3<R> w,
                                              const R qd[3], R delta, V3<R> n, V3<R> r, V3<R> vo, S dt, R wgt, S* Q,
                                              S* rb, LegSys<S>& L, V3<R>& F, R& eta)
{
    const V3<R> ex = v3(R(1), R(0), R(0));
    const V3<R> ja = cross(ex, r - G.h), jf = cross(G.ey, r - G.h), jk = cross(G.ey, r - G.pk);
    const V3<R> vc = vb + cross(w, r) + qd[0] * ja + qd[1] * jf + qd[2] * jk - vo;
    contact_law(M, delta, n, vc, F, eta);
    F = wgt * F;
    eta = wgt * eta;
    const S e = S(eta), cw = S(wgt) * S(M.cc);
    const S ce = cw - e;
    const V3<S> rs = cv<S>(r), ns = cv<S>(n), Fs = cv<S>(F);
    base_contact_folded(e, cw, rs, ns, Fs, dt, Q, rb);
    // the leg's rows: dt (e J_l^T J + ce g_l g^T) with g_l = J_l^T n, dt e and dt ce folded
    // into the operands
    const S de = dt * e;
    const V3<S> jv[3] = {cv<S>(ja), cv<S>(jf), cv<S>(jk)};
    const S gj[3] = {dot(jv[0], ns), dot(jv[1], ns), dot(jv[2], ns)};
    const S dg[3] = {dt * ce * gj[0], dt * ce * gj[1], dt * ce * gj[2]};
    const V3<S> gA = cross(rs, ns);
    const S g0[6] = {gA.x, gA.y, gA.z, ns.x, ns.y, ns.z};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const V3<S> rxj = cross(rs, jv[j]);
        const S jb[6] = {rxj.x, rxj.y, rxj.z, jv[j].x, jv[j].y, jv[j].z};
#pragma unroll
        for (int i = 0; i < 6; ++i) L.C[j][i] += de * jb[i] + dg[j] * g0[i];
        L.rl[j] += dt * dot(jv[j], Fs);
    }
    L.A00 += de * dot(jv[0], jv[0]) + dg[0] * gj[0];
    L.A01 += de * dot(jv[0], jv[1]) + dg[0] * gj[1];
    L.A02 += de * dot(jv[0], jv[2]) + dg[0] * gj[2];
    L.A11 += de * dot(jv[1], jv[1]) + dg[1] * gj[1];
    L.A12 += de * dot(jv[1], jv[2]) + dg[1] * gj[2];
    L.A22 += de * dot(jv[2], jv[2]) + dg[2] * gj[2];
}

// contact terms of a force F at body-frame point r with normal n and secant eta (all in
// the geometry type R) on a 6x6 body system accumulated in S
template <typename R, typename S>
__device__ __forceinline__ void body_contact(R eta, R c, V3<R> r, V3<R> n, V3<R> F, S dt, S* Q, S* rb)
{
    base_contact_folded(S(eta), S(c), cv<S>(r), cv<S>(n), cv<S>(F), dt, Q, rb);
}

// ------------------------------------------------------------------------------
// one dynamics step of one sample; lane g (0..15) of the sample, leg g >> 2, sub-lane
// g & 3.  R: the geometry type (kinematics, contact detection and law, state); S: the
// system type (mass matrix, bias, contact damping and forces as terms of the implicit
// system, the leg elimination, the sums and the 6x6 solves).  MR / MS: the model in
// both.  uj: the joint target this lane interpolated (joint g & 3 of its leg, lanes 3
// repeat joint 2).  red / sred: this sample's LDS rows.  tau2 receives sum tau^2.
// ------------------------------------------------------------------------------
template <int SCENE, typename R, typename S>
__device__ __forceinline__ void step16(const ModelT<R>& MR, const ModelT<S>& MS, const float* __restrict__ hf, S dt,
                                       S kp, S kd, int g, Base<R>& b, Leg<R>& lg, BoxS<R>& bx, R uj, S* red,
                                       S* sred, R& tau2)
{
    const int leg = g >> 2, sub = g & 3;
    const R dtr = R(dt);
    const R u[3] = {dpp<0x00>(uj), dpp<0x55>(uj), dpp<0xAA>(uj)};
    S tau[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) tau[j] = kp * (S(u[j]) - S(lg.q[j])) - kd * S(lg.qd[j]);
    const S t2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];

    const M33<R> Rm = quat_R(b.qw, b.qx, b.qy, b.qz);
    const V3<R> w = b.w;
    const V3<R> vb = mulT(Rm, b.vw);
    const V3<R> gb = (-MR.g) * v3(Rm.m[6], Rm.m[7], Rm.m[8]);

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
    G.ey = v3(R(0), ca, sa);
    G.d1 = v3(-sf, sa * cf, -ca * cf);
    G.d2 = v3(-s12, sa * c12, -ca * c12);
    G.h = v3((leg < 2) ? MR.hip_x : -MR.hip_x, (leg & 1) ? -MR.hip_y : MR.hip_y, R(0));
    G.pk = G.h + MR.l1 * G.d1;
    G.pf = G.pk + MR.l2 * G.d2;
    G.c1 = G.h + (R(0.5) * MR.l1) * G.d1;
    G.c2 = G.pk + (R(0.5) * MR.l2) * G.d2;

    // the leg's geometry and velocities in the system type
    const V3<S> ex = v3(S(1), S(0), S(0));
    const V3<S> ey = cv<S>(G.ey), d1 = cv<S>(G.d1), d2 = cv<S>(G.d2), h = cv<S>(G.h), pk = cv<S>(G.pk),
                c1 = cv<S>(G.c1), c2 = cv<S>(G.c2);
    const V3<S> ws = cv<S>(w), gbs = cv<S>(gb);
    const S dqa = S(lg.qd[0]), dqf = S(lg.qd[1]), dqk = S(lg.qd[2]);

    // ---- the leg's mass-matrix terms: base block, coupling columns, leg block
    S Q[21];
#pragma unroll
    for (int i = 0; i < 21; ++i) Q[i] = S(0);
    {
        const S r1 = dot(c1, c1), r2 = dot(c2, c2);
        const S cv1[3] = {c1.x, c1.y, c1.z}, cv2[3] = {c2.x, c2.y, c2.z};
        const S d1v[3] = {d1.x, d1.y, d1.z}, d2v[3] = {d2.x, d2.y, d2.z};
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                const S I = (i == j) ? S(1) : S(0);
                Q[s6(i, j)] = MS.k1 * (I - d1v[i] * d1v[j]) + MS.k2 * (I - d2v[i] * d2v[j]) +
                              MS.m1 * (r1 * I - cv1[i] * cv1[j]) + MS.m2 * (r2 * I - cv2[i] * cv2[j]);
            }
        const V3<S> hl = MS.m1 * c1 + MS.m2 * c2;
        Q[s6(0, 4)] = -hl.z; Q[s6(0, 5)] = hl.y;
        Q[s6(1, 3)] = hl.z;  Q[s6(1, 5)] = -hl.x;
        Q[s6(2, 3)] = -hl.y; Q[s6(2, 4)] = hl.x;
    }
    LegSys<S> L;
    {
        const V3<S> ua1 = cross(ex, c1 - h), ua2 = cross(ex, c2 - h);
        const V3<S> uf1 = cross(ey, c1 - h), uf2 = cross(ey, c2 - h);
        const V3<S> uk2 = cross(ey, c2 - pk);
        const V3<S> Pa = MS.m1 * ua1 + MS.m2 * ua2;
        const V3<S> La =
            MS.m1 * cross(c1, ua1) + MS.m2 * cross(c2, ua2) + rod_I(MS.k1, d1, ex) + rod_I(MS.k2, d2, ex);
        const V3<S> Pf = MS.m1 * uf1 + MS.m2 * uf2;
        const V3<S> Lf =
            MS.m1 * cross(c1, uf1) + MS.m2 * cross(c2, uf2) + rod_I(MS.k1, d1, ey) + rod_I(MS.k2, d2, ey);
        const V3<S> Pk = MS.m2 * uk2;
        const V3<S> Lk = MS.m2 * cross(c2, uk2) + rod_I(MS.k2, d2, ey);
        const V3<S> Ls[3] = {La, Lf, Lk}, Ps[3] = {Pa, Pf, Pk};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            L.C[j][0] = Ls[j].x; L.C[j][1] = Ls[j].y; L.C[j][2] = Ls[j].z;
            L.C[j][3] = Ps[j].x; L.C[j][4] = Ps[j].y; L.C[j][5] = Ps[j].z;
        }
        const V3<S> oxa_a = cross(h, ex), oxa_f = cross(h, ey), oxa_k = cross(pk, ey);
        L.A00 = dot(ex, La) + dot(oxa_a, Pa);
        L.A01 = dot(ex, Lf) + dot(oxa_a, Pf);
        L.A02 = dot(ex, Lk) + dot(oxa_a, Pk);
        L.A11 = dot(ey, Lf) + dot(oxa_f, Pf);
        L.A12 = dot(ey, Lk) + dot(oxa_f, Pk);
        L.A22 = dot(ey, Lk) + dot(oxa_k, Pk);
    }

    // ---- bias forces of the leg (zero generalized acceleration, gravity)
    S rb[6];
    {
        const V3<S> w1 = ws + dqa * ex + dqf * ey;
        const V3<S> al1 = dqa * cross(ws, ex) + dqf * cross(ws + dqa * ex, ey);
        const V3<S> ah = cross(ws, cross(ws, h));
        const V3<S> r1 = c1 - h, rk = pk - h;
        const V3<S> ac1 = ah + cross(al1, r1) + cross(w1, cross(w1, r1));
        const V3<S> apk = ah + cross(al1, rk) + cross(w1, cross(w1, rk));
        const V3<S> w2 = w1 + dqk * ey;
        const V3<S> al2 = al1 + dqk * cross(w1, ey);
        const V3<S> r2 = c2 - pk;
        const V3<S> ac2 = apk + cross(al2, r2) + cross(w2, cross(w2, r2));
        const V3<S> F1 = MS.m1 * (ac1 - gbs), F2 = MS.m2 * (ac2 - gbs);
        const V3<S> N1 = rod_I(MS.k1, d1, al1) + cross(w1, rod_I(MS.k1, d1, w1));
        const V3<S> N2 = rod_I(MS.k2, d2, al2) + cross(w2, rod_I(MS.k2, d2, w2));
        const V3<S> Tk = N2 + cross(r2, F2);
        const V3<S> Th = N1 + cross(r1, F1) + N2 + cross(c2 - h, F2);
        const V3<S> Tb = N1 + N2 + cross(c1, F1) + cross(c2, F2);
        const V3<S> Fb = F1 + F2;
        rb[0] = -dt * Tb.x; rb[1] = -dt * Tb.y; rb[2] = -dt * Tb.z;
        rb[3] = -dt * Fb.x; rb[4] = -dt * Fb.y; rb[5] = -dt * Fb.z;
        L.rl[0] = dt * (tau[0] - dot(ex, Th));
        L.rl[1] = dt * (tau[1] - dot(ey, Th));
        L.rl[2] = dt * (tau[2] - dot(ey, Tk));
    }
    L.A00 += dt * kd; L.A11 += dt * kd; L.A22 += dt * kd;

    [[maybe_unused]] BoxFrame<R> bf;
    [[maybe_unused]] S Qb[21], rbx[6];
    const V3<R> zero = v3(R(0), R(0), R(0));
    V3<R> F;
    R eta;
    if constexpr (SCENE == 3) {
        bf.Rb = quat_R(bx.qw, bx.qx, bx.qy, bx.qz);
#pragma unroll
        for (int i = 0; i < 21; ++i) Qb[i] = S(0);
#pragma unroll
        for (int i = 0; i < 6; ++i) rbx[i] = S(0);
    }

    // ---- the leg's foot against terrain and the static or free box.  Each lane lists its
    // foot's contacts (terrain, box) and the wave runs one contact body per listed entry:
    // usually one pass, a second only where a foot touches both.
    {
        const V3<R> pfw = b.p + mul(Rm, G.pf);
        R dT, dB = R(0);
        V3<R> nT, nB = zero;
        const bool hitT = terrain<SCENE>(MR, hf, pfw, MR.foot_r, dT, nT);
        bool hitB = false;
        if constexpr (SCENE == 2) {
            hitB = sphere_aabox(pfw - v3(MR.sb_cx, MR.sb_cy, MR.sb_cz), MR.foot_r, v3(MR.sb_hx, MR.sb_hy, MR.sb_hz),
                                dB, nB);
        }
        if constexpr (SCENE == 3) {
            V3<R> nl = v3(R(0), R(0), R(1));  // left as is when the foot misses the box
            hitB = sphere_aabox(mulT(bf.Rb, pfw - bx.p), MR.foot_r, v3(MR.bx_hx, MR.bx_hy, MR.bx_hz), dB, nl);
            nB = mul(bf.Rb, nl);  // box -> foot (world)
        }
        const int cnt = int(hitT) + int(hitB);
#pragma unroll
        for (int it = 0; it < ((SCENE == 2 || SCENE == 3) ? 2 : 1); ++it) {
            if (!__builtin_amdgcn_ballot_w64(it < cnt)) break;
            const bool isB = (it == 0) ? !hitT : true;  // pass 0: terrain if touched, else the box
            // a lane without a contact in this pass takes a neutral one (zero depth, upward
            // normal, zero weight), so nothing it adds can be non-finite
            const bool on = it < cnt;
            const R wgt = on ? R(1) : R(0);
            const R delta = on ? (isB ? dB : dT) : R(0);
            const V3<R> nw = on ? selv(isB, nB, nT) : v3(R(0), R(0), R(1));
            const V3<R> n = mulT(Rm, nw);
            V3<R> vo = zero;
            [[maybe_unused]] V3<R> pcw;
            if constexpr (SCENE == 3) {
                pcw = pfw - MR.foot_r * nw;
                vo = selv(isB && on, mulT(Rm, box_point_vel(bx, bf, pcw)), zero);
            }
            leg_contact_w(MR, G, vb, w, lg.qd, delta, n, G.pf - MR.foot_r * n, vo, dt, wgt, Q, rb, L, F, eta);
            if constexpr (SCENE == 3) {
                // the box's share in its frame (zero weight for the terrain contact)
                const R wb = isB ? wgt : R(0);
                body_contact(wb * eta, wb * MR.cc, mulT(bf.Rb, pcw - bx.p), mulT(bf.Rb, nw),
                             mulT(bf.Rb, (-wb) * mul(Rm, F)), dt, Qb, rbx);
            }
        }
    }

    // ---- eliminate the leg: W = A_ll^-1 A_l0, y = A_ll^-1 r_l
    const Chol3<S> L3 = chol3(L.A00, L.A01, L.A11, L.A02, L.A12, L.A22);
    S W[3][6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        S x0 = L.C[0][i], x1 = L.C[1][i], x2 = L.C[2][i];
        solve3(L3, x0, x1, x2);
        W[0][i] = x0; W[1][i] = x1; W[2][i] = x2;
    }
    S y0 = L.rl[0], y1 = L.rl[1], y2 = L.rl[2];
    solve3(L3, y0, y1, y2);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
        for (int j = i; j < 6; ++j) Q[s6(i, j)] -= L.C[0][i] * W[0][j] + L.C[1][i] * W[1][j] + L.C[2][i] * W[2][j];
        rb[i] -= L.C[0][i] * y0 + L.C[1][i] * y1 + L.C[2][i] * y2;
    }

    // the leg's terms are the same in its four lanes: only sub-lane 0's copy is summed
    const bool keep = sub == 0;
#pragma unroll
    for (int i = 0; i < 21; ++i) Q[i] = sel(keep, Q[i], S(0));
#pragma unroll
    for (int i = 0; i < 6; ++i) rb[i] = sel(keep, rb[i], S(0));
    if constexpr (SCENE == 3) {
#pragma unroll
        for (int i = 0; i < 21; ++i) Qb[i] = sel(keep, Qb[i], S(0));
#pragma unroll
        for (int i = 0; i < 6; ++i) rbx[i] = sel(keep, rbx[i], S(0));
    }

    // ---- one corner per lane: trunk corner g (g < 8), free-box corner g - 8 (g >= 8)
    if constexpr (SCENE != 3) {
        if (g < 8) {
            const V3<R> rloc = v3((g & 1 ? R(0.5) : R(-0.5)) * MR.tsx, (g & 2 ? R(0.5) : R(-0.5)) * MR.tsy,
                                  (g & 4 ? R(0.5) : R(-0.5)) * MR.tsz);
            const V3<R> pw = b.p + mul(Rm, rloc);
            R delta;
            V3<R> nw;
            if (terrain<SCENE>(MR, hf, pw, R(0), delta, nw)) {
                const V3<R> n = mulT(Rm, nw);
                contact_law(MR, delta, n, vb + cross(w, rloc), F, eta);
                body_contact(eta, MR.cc, rloc, n, F, dt, Q, rb);
            }
            if constexpr (SCENE == 2) {
                if (point_aabox(pw - v3(MR.sb_cx, MR.sb_cy, MR.sb_cz), v3(MR.sb_hx, MR.sb_hy, MR.sb_hz), delta, nw)) {
                    const V3<R> n = mulT(Rm, nw);
                    contact_law(MR, delta, n, vb + cross(w, rloc), F, eta);
                    body_contact(eta, MR.cc, rloc, n, F, dt, Q, rb);
                }
            }
        }
    } else {
        // A corner of body P (the trunk on lanes 0-7, the box on lanes 8-15) against the
        // other body Q (a point inside Q's box, normal out of Q's nearest face) and against
        // the terrain.  The same code serves both roles: each contact adds its terms to the
        // trunk's and the box's 6x6 systems in their own frames, with zero weight where a
        // body is not part of the contact.
        const bool own_trunk = g < 8;
        const int ci = g & 7;
        Pose<R> PT, PB;
        PT.Rt = Rm; PT.p = b.p; PT.vw = b.vw; PT.w = b.w;
        PB.Rt = bf.Rb; PB.p = bx.p; PB.vw = bx.vw; PB.w = bx.w;
        const Pose<R> own = sel_pose(own_trunk, PT, PB), oth = sel_pose(own_trunk, PB, PT);
        const V3<R> th = v3(R(0.5) * MR.tsx, R(0.5) * MR.tsy, R(0.5) * MR.tsz), bh = v3(MR.bx_hx, MR.bx_hy, MR.bx_hz);
        const V3<R> hP = selv(own_trunk, th, bh), hQ = selv(own_trunk, bh, th);
        const V3<R> cl = v3(ci & 1 ? hP.x : -hP.x, ci & 2 ? hP.y : -hP.y, ci & 4 ? hP.z : -hP.z);
        const V3<R> x = own.p + mul(own.Rt, cl);
        const V3<R> lq = mulT(oth.Rt, x - oth.p);
        R dP = R(0), dG;
        V3<R> nlq = zero, nG;
        const bool hitP = point_aabox(lq, hQ, dP, nlq);  // nlq: Q's face normal toward the corner
        const bool hitG = terrain<SCENE>(MR, hf, x, R(0), dG, nG);
        const int cnt = int(hitP) + int(hitG);
        if (__builtin_amdgcn_ballot_w64(cnt > 0)) {
            const V3<R> vP = pose_point_vel(own, x), vQ = pose_point_vel(oth, x);
            const V3<R> nPw = mul(oth.Rt, nlq);
#pragma unroll
            for (int it = 0; it < 2; ++it) {
                if (!__builtin_amdgcn_ballot_w64(it < cnt)) break;
                const bool pair = (it == 0) && hitP;  // pass 0: the pair if touching, else the terrain
                // a lane without a contact in this pass takes a neutral one (zero depth and
                // velocity, zero weight), so nothing it adds can be non-finite
                const bool on = it < cnt;
                const R wgt = on ? R(1) : R(0);
                const R wq = pair ? wgt : R(0);
                const V3<R> n = on ? selv(pair, nPw, nG) : v3(R(0), R(0), R(1));
                contact_law(MR, on ? (pair ? dP : dG) : R(0), n, on ? selv(pair, vP - vQ, vP) : zero, F, eta);
                F = wgt * F;
                eta = wgt * eta;
                // P's side in P's frame (force +F), Q's side in Q's frame (force -F)
                const V3<R> nP = mulT(own.Rt, n), FP = mulT(own.Rt, F);
                const V3<R> FQ = R(-1) * mulT(oth.Rt, F);
                const R cP = wgt * MR.cc, cQ = wq * MR.cc, eQ = wq * eta;
                body_contact(sel(own_trunk, eta, eQ), sel(own_trunk, cP, cQ), selv(own_trunk, cl, lq),
                             selv(own_trunk, nP, nlq), selv(own_trunk, FP, wq * FQ), dt, Q, rb);
                body_contact(sel(own_trunk, eQ, eta), sel(own_trunk, cQ, cP), selv(own_trunk, lq, cl),
                             selv(own_trunk, nlq, nP), selv(own_trunk, wq * FQ, FP), dt, Qb, rbx);
            }
        }
    }

    // ---- sum the trunk (and box) systems and the squared torques over the 16 lanes
    constexpr int NV = n_summed<SCENE>();
    {
        S v[NV];
#pragma unroll
        for (int i = 0; i < 21; ++i) v[i] = Q[i];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[21 + i] = rb[i];
        v[27] = sel(keep, t2, S(0));
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
    tau2 = R(sred[27]);
    if constexpr (SCENE == 3) {
#pragma unroll
        for (int i = 0; i < 21; ++i) Qb[i] = sred[28 + i];
#pragma unroll
        for (int i = 0; i < 6; ++i) rbx[i] = sred[49 + i];
    }

    // ---- the trunk's own terms: inertia, total mass, gyroscopic and gravity bias
    Q[s6(0, 0)] += MS.I0x; Q[s6(1, 1)] += MS.I0y; Q[s6(2, 2)] += MS.I0z;
    Q[s6(3, 3)] += MS.mtot; Q[s6(4, 4)] += MS.mtot; Q[s6(5, 5)] += MS.mtot;
    {
        const V3<S> Iw = v3(MS.I0x * ws.x, MS.I0y * ws.y, MS.I0z * ws.z);
        const V3<S> gy = cross(ws, Iw);
        rb[0] -= dt * gy.x; rb[1] -= dt * gy.y; rb[2] -= dt * gy.z;
        rb[3] += dt * MS.m0 * gbs.x; rb[4] += dt * MS.m0 * gbs.y; rb[5] += dt * MS.m0 * gbs.z;
    }
    if constexpr (SCENE != 3) {
        chol6_solve(Q, rb);  // rb <- trunk increment [d omega; d v_b]
    } else {
        // the box's own terms, then one 6x6 solve per lane: trunk on even lanes, box on
        // odd lanes; neighbours swap their results
        Qb[s6(0, 0)] += MS.bx_Ix; Qb[s6(1, 1)] += MS.bx_Iy; Qb[s6(2, 2)] += MS.bx_Iz;
        Qb[s6(3, 3)] += MS.bx_m; Qb[s6(4, 4)] += MS.bx_m; Qb[s6(5, 5)] += MS.bx_m;
        const V3<S> wbx = cv<S>(bx.w);
        const V3<S> gyb = cross(wbx, v3(MS.bx_Ix * wbx.x, MS.bx_Iy * wbx.y, MS.bx_Iz * wbx.z));
        const V3<S> gl = cv<S>((-MR.g) * v3(bf.Rb.m[6], bf.Rb.m[7], bf.Rb.m[8]));
        rbx[0] -= dt * gyb.x; rbx[1] -= dt * gyb.y; rbx[2] -= dt * gyb.z;
        rbx[3] += dt * MS.bx_m * gl.x; rbx[4] += dt * MS.bx_m * gl.y; rbx[5] += dt * MS.bx_m * gl.z;
        const bool odd = (g & 1) != 0;
        S Qs[21], rs[6];
#pragma unroll
        for (int i = 0; i < 21; ++i) Qs[i] = sel(odd, Qb[i], Q[i]);
#pragma unroll
        for (int i = 0; i < 6; ++i) rs[i] = sel(odd, rbx[i], rb[i]);
        chol6_solve(Qs, rs);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const S other = dpp<0xB1>(rs[i]);  // the neighbour's result (lanes 0<->1, 2<->3)
            rb[i] = sel(odd, other, rs[i]);
            rbx[i] = sel(odd, rs[i], other);
        }
    }

    // ---- back-substitute the leg and integrate (semi-implicit Euler): velocities add the
    // increments in S, positions take dt times the new velocities in R
    S dq[3] = {y0, y1, y2};
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 6; ++i) dq[j] -= W[j][i] * rb[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        lg.qd[j] = R(S(lg.qd[j]) + dq[j]);
        lg.q[j] += dtr * lg.qd[j];
    }
    M33<S> Rs;
#pragma unroll
    for (int i = 0; i < 9; ++i) Rs.m[i] = S(Rm.m[i]);
    b.w = cv<R>(ws + v3(rb[0], rb[1], rb[2]));
    b.vw = cv<R>(cv<S>(b.vw) + mul(Rs, v3(rb[3], rb[4], rb[5])));
    b.p = b.p + dtr * b.vw;
    if constexpr (SCENE != 3) {
        quat_step(b.qw, b.qx, b.qy, b.qz, b.w, dtr);
    } else {
        M33<S> Rbs;
#pragma unroll
        for (int i = 0; i < 9; ++i) Rbs.m[i] = S(bf.Rb.m[i]);
        bx.w = cv<R>(cv<S>(bx.w) + v3(rbx[0], rbx[1], rbx[2]));
        bx.vw = cv<R>(cv<S>(bx.vw) + mul(Rbs, v3(rbx[3], rbx[4], rbx[5])));
        bx.p = bx.p + dtr * bx.vw;
        // one quaternion step per lane: the trunk's on even lanes, the box's on odd lanes
        const bool odd = (g & 1) != 0;
        R q[4] = {sel(odd, bx.qw, b.qw), sel(odd, bx.qx, b.qx), sel(odd, bx.qy, b.qy), sel(odd, bx.qz, b.qz)};
        quat_step(q[0], q[1], q[2], q[3], selv(odd, bx.w, b.w), dtr);
        R o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = dpp<0xB1>(q[i]);
        b.qw = sel(odd, o[0], q[0]); b.qx = sel(odd, o[1], q[1]); b.qy = sel(odd, o[2], q[2]); b.qz = sel(odd, o[3], q[3]);
        bx.qw = sel(odd, q[0], o[0]); bx.qx = sel(odd, q[1], o[1]); bx.qy = sel(odd, q[2], o[2]);
        bx.qz = sel(odd, q[3], o[3]);
    }
}

}  // namespace r16

// ------------------------------------------------------------------------------
// rollout kernel: workgroup of 64 lanes = 4 samples x 16 lanes.  R: geometry and state
// type, S: system type (FP32/FP32, FP64/FP64, or FP32 geometry with the FP64 system).
// LDS: the summation rows [4][NV][kPitch] (NV summed values of the scene) and sums
// [4][kSumPitch] (type S), then the heightfield (scene 1).  eps addressing as in the quad kernel: eps_in[n * eps_sn + d *
// eps_sd] when given, otherwise Philox noise stored to eps_out[d * K + n].  DIRECT: one
// value per control step (the direct representation, whose noise is drawn inside the step
// loop; the `direct` argument equals it); a separate instantiation, so that the knot
// representations carry no per-step sampling code and its registers in their step loop.
// ------------------------------------------------------------------------------
template <int SCENE, typename R, typename S, bool DIRECT>
__global__ __launch_bounds__(64) void rollout16_kernel(ModelT<R> Mr, ModelT<S> Ms, DevParams P,
                                                       const double* __restrict__ gB,
                                                       const float* __restrict__ ghf, const float* __restrict__ mu,
                                                       const float* __restrict__ x0,
                                                       const float* __restrict__ eps_in, int eps_sn, int eps_sd,
                                                       float* __restrict__ eps_out, float* __restrict__ costs,
                                                       float* __restrict__ traj, int direct,
                                                       const int* __restrict__ skip, int* __restrict__ input_status)
{
    // a plain fallback rollout whose proposal the gate took: nothing to do
    if (skip && skip[0]) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    // the model's constants are read from LDS (values in vector registers), which keeps the
    // scalar registers for the kernel's pointers and loop state
    __shared__ ModelT<R> sMr;
    __shared__ ModelT<S> sMs;
    constexpr int NV = r16::n_summed<SCENE>();
    S* red = reinterpret_cast<S*>(lds_raw);
    S* sred = red + r16::kSamples * NV * r16::kPitch;
    float* sHF = reinterpret_cast<float*>(sred + r16::kSamples * r16::kSumPitch);
    if (threadIdx.x == 0) {
        sMr = Mr;
        sMs = Ms;
    }
    if constexpr (SCENE == 1) {
        const int cells = Mr.hf_nx * Mr.hf_ny;
        for (int i = threadIdx.x; i < cells; i += blockDim.x) sHF[i] = ghf[i];
    }
    __syncthreads();
    const ModelT<R>& MR = sMr;
    const ModelT<S>& MS = sMs;

    const int tid = threadIdx.x;
    const int g = tid & 15, grp = tid >> 4;
    const int leg = g >> 2, sub = g & 3;
    const int jl = sub < 3 ? sub : 2;  // this lane's joint of its leg
    const int n = blockIdx.x * r16::kSamples + grp;
    const bool valid = n < P.K;
    const int ns = valid ? n : P.K - 1;
    const int nk = P.nk;
    const R sigma = P.sigma;

    // knots of this lane's joint, theta = mu + sigma eps (sample 0 is the nominal); the
    // direct representation draws one value per step inside the step loop instead
    R th[kMaxKnots];
#pragma unroll
    for (int i = 0; i < kMaxKnots; ++i) {
        th[i] = R(0);
        if (!DIRECT && i < nk) {
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

    // a start state that is not finite: no rollout, every cost +inf, and the flag set
    {
        bool bad = false;
        for (int i = tid; i < P.nx; i += 64) bad |= !(fabsf(x0[i]) <= 3.0e38f);
        const bool any_bad = __builtin_amdgcn_ballot_w64(bad) != 0;
        if (input_status && blockIdx.x == 0 && tid == 0) input_status[0] = any_bad ? 1 : 0;
        if (any_bad) {
            if (valid && g == 0) costs[n] = __int_as_float(0x7f800000);
            return;
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

    S* my_red = red + grp * NV * r16::kPitch;
    S* my_sum = sred + grp * r16::kSumPitch;
    const S dt = P.dt, kp = P.kp, kd = P.kd;
    R L = R(0);
    for (int k = 0; k < P.H; ++k) {
        R uj = R(0);
        if constexpr (DIRECT) {
            // value k of this lane's joint (nk == H): theta = mu + sigma eps
            const int d = (3 * leg + jl) * nk + k;
            R e;
            if (eps_in) {
                e = eps_in[(size_t)ns * eps_sn + (size_t)d * eps_sd];
            } else {
                e = gauss_elem<R>(P, (uint32_t)ns, (uint32_t)d);
                if (valid && sub < 3 && eps_out) eps_out[(size_t)d * P.K + n] = (float)e;
            }
            uj = R(mu[d]) + (ns ? sigma * e : R(0));
        } else {
#pragma unroll
            for (int i = 0; i < kMaxKnots; ++i)
                if (i < nk) uj += R(gB[k * nk + i]) * th[i];
        }
        R tau2;
        r16::step16<SCENE, R, S>(MR, MS, sHF, dt, kp, kd, g, b, lg, bx, uj, my_red, my_sum, tau2);
        round_state(b, lg);
        if constexpr (SCENE == 3) round_box(bx);
        L += R(dt) * stage_cost<SCENE>(P, b, bx, tau2);
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

template <typename S>
size_t lds_bytes(int scene, int hf_cells)
{
    const size_t nv = scene == 3 ? 55 : 28;  // n_summed<scene>()
    size_t b = sizeof(S) * ((size_t)kSamples * nv * kPitch + (size_t)kSamples * kSumPitch);
    if (scene == 1) b += sizeof(float) * (size_t)hf_cells;
    return b;
}

template <typename R, typename S>
hipError_t launch_t(const ModelT<R>& Mr, const ModelT<S>& Ms, const DevParams& P, const RolloutArgs& a,
                    hipStream_t st)
{
    const int blocks = (P.K + kSamples - 1) / kSamples;
    const size_t lds = lds_bytes<S>(Mr.scene, Mr.hf_nx * Mr.hf_ny);
    if (lds > 65536) return hipErrorInvalidValue;
#define MPPI_LAUNCH_R16_D(SC, D)                                                                               \
    hipLaunchKernelGGL((rollout16_kernel<SC, R, S, D>), dim3(blocks), dim3(64), lds, st, Mr, Ms, P, a.B, a.hf,     \
                       a.mu, a.x0, a.eps_in, a.eps_sn, a.eps_sd, a.eps_out, a.costs, a.traj, a.direct, a.skip,     \
                       a.input_status)
#define MPPI_LAUNCH_R16(SC)          \
    if (a.direct)                    \
        MPPI_LAUNCH_R16_D(SC, true); \
    else                             \
        MPPI_LAUNCH_R16_D(SC, false)
    switch (Mr.scene) {
    case 0: MPPI_LAUNCH_R16(0); break;
    case 1: MPPI_LAUNCH_R16(1); break;
    case 2: MPPI_LAUNCH_R16(2); break;
    case 3: MPPI_LAUNCH_R16(3); break;
    default: return hipErrorInvalidValue;
    }
#undef MPPI_LAUNCH_R16
#undef MPPI_LAUNCH_R16_D
    return hipGetLastError();
}

}  // namespace r16

bool rollout16_fits(int arith, int scene, int hf_cells)
{
    const size_t b = arith == 1 ? r16::lds_bytes<float>(scene, hf_cells) : r16::lds_bytes<double>(scene, hf_cells);
    return b <= 65536;
}

// arith: 0 FP64, 1 FP32, 2 FP32 geometry with the FP64 implicit system
hipError_t launch_rollout16(const DevModelF& Mf, const DevModelD& Md, int arith, const DevParams& P,
                            const RolloutArgs& a, hipStream_t st)
{
    if (arith == 1) return r16::launch_t(Mf, Mf, P, a, st);
    if (arith == 2) return r16::launch_t(Mf, Md, P, a, st);
    return r16::launch_t(Md, Md, P, a, st);
}

}  // namespace mppi
