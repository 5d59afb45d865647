/*
 * Oracle for whole-body MPPI -- plain FP64 C.  TEST INFRASTRUCTURE ONLY (tests,
 * smoke check, CPU baseline); the product library never links or calls it.
 *
 * What it follows:
 *   - MPPI weights and mean update: Eq. 1 and Eq. 2 (Sec. II-B), loop structure of
 *     Algorithm 1 (one knot vector per sample, simulated over the horizon while the
 *     running cost is summed; then weights, mean update, first control, shift).
 *   - Controls as a cubic spline through evenly spaced knots, tracked by joint PD
 *     (Sec. III-B, Fig. "system overview"; PD tracking Sec. IV-A).
 *   - The paper simulates with MuJoCo (Sec. III-A); here the simulator is replaced by
 *     floating-base rigid-body dynamics with penalty contact, written from textbook
 *     definitions: the mass matrix is sum_b J_b^T I_b J_b over bodies, the bias is the
 *     projected Newton-Euler wrench sum_b J_b^T W_b (Kane's form), contacts are
 *     spring-damper normal forces with tanh-smoothed Coulomb friction, and one step is
 *     (M + dt D) dv = dt f with D = -df/dv (damping treated implicitly).
 *   - Walk cost of Eq. 3 in simplified form; box-push cost of Eq. 4 with squared
 *     distances and the robot's goal at the box centre (Sec. IV-D).
 * Everything is written for clarity, not speed: dense 18x18 matrices, dense Jacobians.
 */
#include "mppi_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* small vector helpers                                                 */
/* ------------------------------------------------------------------ */
static void cross3(const double a[3], const double b[3], double o[3])
{
    double t0 = a[1] * b[2] - a[2] * b[1];
    double t1 = a[2] * b[0] - a[0] * b[2];
    double t2 = a[0] * b[1] - a[1] * b[0];
    o[0] = t0; o[1] = t1; o[2] = t2;
}
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void matvec3(const double R[9], const double a[3], double o[3])
{
    double t0 = R[0] * a[0] + R[1] * a[1] + R[2] * a[2];
    double t1 = R[3] * a[0] + R[4] * a[1] + R[5] * a[2];
    double t2 = R[6] * a[0] + R[7] * a[1] + R[8] * a[2];
    o[0] = t0; o[1] = t1; o[2] = t2;
}
static void matTvec3(const double R[9], const double a[3], double o[3])
{
    double t0 = R[0] * a[0] + R[3] * a[1] + R[6] * a[2];
    double t1 = R[1] * a[0] + R[4] * a[1] + R[7] * a[2];
    double t2 = R[2] * a[0] + R[5] * a[1] + R[8] * a[2];
    o[0] = t0; o[1] = t1; o[2] = t2;
}
static void matmul3(const double A[9], const double B[9], double C[9])
{
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            T[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
    memcpy(C, T, sizeof(T));
}
static void quat_to_mat(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}
static void quat_mul(const double a[4], const double b[4], double o[4])
{
    double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}
/* quaternion of the rotation by vector phi (axis * angle) */
static void quat_exp(const double phi[3], double o[4])
{
    double a = sqrt(dot3(phi, phi)) * 0.5;
    double s = (a > 0) ? sin(a) / a : 1.0;
    o[0] = cos(a); o[1] = 0.5 * s * phi[0]; o[2] = 0.5 * s * phi[1]; o[3] = 0.5 * s * phi[2];
}
/* rotation matrix about unit axis by angle (Rodrigues) */
static void axis_angle(const double a[3], double ang, double R[9])
{
    double c = cos(ang), s = sin(ang), C = 1 - c;
    double x = a[0], y = a[1], z = a[2];
    R[0] = c + x * x * C;     R[1] = x * y * C - z * s; R[2] = x * z * C + y * s;
    R[3] = y * x * C + z * s; R[4] = c + y * y * C;     R[5] = y * z * C - x * s;
    R[6] = z * x * C - y * s; R[7] = z * y * C + x * s; R[8] = c + z * z * C;
}

/* ------------------------------------------------------------------ */
/* robot description as a generic kinematic tree                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int parent[ORC_NB];
    double axis[ORC_NB][3];     /* joint axis in the body's own frame */
    double offset[ORC_NB][3];   /* joint position in the parent frame */
    double mass[ORC_NB];
    double com[ORC_NB][3];      /* centre of mass in body frame */
    double inertia[ORC_NB][3];  /* principal inertia about the CoM, body axes */
} tree_t;

static void build_tree(const orc_model *m, tree_t *t)
{
    memset(t, 0, sizeof(*t));
    const double sx = m->trunk_size[0], sy = m->trunk_size[1], sz = m->trunk_size[2];
    t->parent[0] = -1;
    t->mass[0] = m->trunk_mass;
    t->inertia[0][0] = m->trunk_mass * (sy * sy + sz * sz) / 12.0;
    t->inertia[0][1] = m->trunk_mass * (sx * sx + sz * sz) / 12.0;
    t->inertia[0][2] = m->trunk_mass * (sx * sx + sy * sy) / 12.0;
    for (int l = 0; l < 4; ++l) {
        /* legs FL, FR, RL, RR: front has +x, left has +y */
        double hx = (l < 2) ? m->hip_x : -m->hip_x;
        double hy = (l % 2 == 0) ? m->hip_y : -m->hip_y;
        int a = 1 + 3 * l, f = a + 1, kn = a + 2;
        t->parent[a] = 0;  t->offset[a][0] = hx; t->offset[a][1] = hy; t->axis[a][0] = 1;
        t->parent[f] = a;  t->axis[f][1] = 1;
        t->parent[kn] = f; t->offset[kn][2] = -m->thigh_len; t->axis[kn][1] = 1;
        t->mass[f] = m->thigh_mass; t->com[f][2] = -0.5 * m->thigh_len;
        t->inertia[f][0] = t->inertia[f][1] = m->thigh_mass * m->thigh_len * m->thigh_len / 12.0;
        t->mass[kn] = m->calf_mass; t->com[kn][2] = -0.5 * m->calf_len;
        t->inertia[kn][0] = t->inertia[kn][1] = m->calf_mass * m->calf_len * m->calf_len / 12.0;
    }
}

typedef struct {
    double R[ORC_NB][9];
    double p[ORC_NB][3];     /* body origin (joint point) in world */
    double c[ORC_NB][3];     /* body CoM in world */
    double a[ORC_NB][3];     /* joint axis in world (bodies >= 1) */
    double Iw[ORC_NB][9];    /* inertia about CoM, world axes */
} fk_t;

static void fk_compute(const orc_model *m, const tree_t *t, const double *q, fk_t *k)
{
    quat_to_mat(q + 3, k->R[0]);
    for (int i = 0; i < 3; ++i) k->p[0][i] = q[i];
    for (int b = 1; b < ORC_NB; ++b) {
        int P = t->parent[b];
        double Rj[9], off[3];
        axis_angle(t->axis[b], q[7 + b - 1], Rj);
        matmul3(k->R[P], Rj, k->R[b]);
        matvec3(k->R[P], t->offset[b], off);
        for (int i = 0; i < 3; ++i) k->p[b][i] = k->p[P][i] + off[i];
        matvec3(k->R[P], t->axis[b], k->a[b]);
    }
    for (int b = 0; b < ORC_NB; ++b) {
        double cw[3];
        matvec3(k->R[b], t->com[b], cw);
        for (int i = 0; i < 3; ++i) k->c[b][i] = k->p[b][i] + cw[i];
        /* Iw = R diag(I) R^T */
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0;
                for (int l = 0; l < 3; ++l) s += k->R[b][3 * i + l] * t->inertia[b][l] * k->R[b][3 * j + l];
                k->Iw[b][3 * i + j] = s;
            }
    }
    (void)m;
}

static int is_ancestor_or_self(const tree_t *t, int j, int b)
{
    while (b >= 0) {
        if (b == j) return 1;
        b = t->parent[b];
    }
    return 0;
}

/* linear-velocity Jacobian of world point x fixed on body b: 3 x 18, row-major */
static void jac_point(const tree_t *t, const fk_t *k, int b, const double x[3], double J[3 * ORC_NV])
{
    memset(J, 0, sizeof(double) * 3 * ORC_NV);
    double r[3] = {x[0] - k->p[0][0], x[1] - k->p[0][1], x[2] - k->p[0][2]};
    for (int i = 0; i < 3; ++i) J[i * ORC_NV + i] = 1.0;
    for (int e = 0; e < 3; ++e) {
        double ew[3] = {k->R[0][e], k->R[0][3 + e], k->R[0][6 + e]}, col[3];
        cross3(ew, r, col);
        for (int i = 0; i < 3; ++i) J[i * ORC_NV + 3 + e] = col[i];
    }
    for (int jb = 1; jb < ORC_NB; ++jb) {
        if (!is_ancestor_or_self(t, jb, b)) continue;
        double rr[3] = {x[0] - k->p[jb][0], x[1] - k->p[jb][1], x[2] - k->p[jb][2]}, col[3];
        cross3(k->a[jb], rr, col);
        for (int i = 0; i < 3; ++i) J[i * ORC_NV + 5 + jb] = col[i];
    }
}
/* angular-velocity Jacobian of body b: 3 x 18 */
static void jac_rot(const tree_t *t, const fk_t *k, int b, double J[3 * ORC_NV])
{
    memset(J, 0, sizeof(double) * 3 * ORC_NV);
    for (int e = 0; e < 3; ++e)
        for (int i = 0; i < 3; ++i) J[i * ORC_NV + 3 + e] = k->R[0][3 * i + e];
    for (int jb = 1; jb < ORC_NB; ++jb) {
        if (!is_ancestor_or_self(t, jb, b)) continue;
        for (int i = 0; i < 3; ++i) J[i * ORC_NV + 5 + jb] = k->a[jb][i];
    }
}

static void mass_matrix_k(const tree_t *t, const fk_t *k, double *M)
{
    memset(M, 0, sizeof(double) * ORC_NV * ORC_NV);
    double Jv[3 * ORC_NV], Jw[3 * ORC_NV];
    for (int b = 0; b < ORC_NB; ++b) {
        if (t->mass[b] == 0) continue;
        jac_point(t, k, b, k->c[b], Jv);
        jac_rot(t, k, b, Jw);
        for (int i = 0; i < ORC_NV; ++i)
            for (int j = 0; j < ORC_NV; ++j) {
                double s = 0;
                for (int r = 0; r < 3; ++r) s += t->mass[b] * Jv[r * ORC_NV + i] * Jv[r * ORC_NV + j];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) s += Jw[r * ORC_NV + i] * k->Iw[b][3 * r + c] * Jw[c * ORC_NV + j];
                M[i * ORC_NV + j] += s;
            }
    }
}

/* bias b(q,v): the generalized force that produces zero generalized acceleration,
   with gravity; computed as sum_b J_b^T [m (a_c - g); I alpha + w x I w] where a_c and
   alpha are body accelerations at zero generalized acceleration (classical mechanics). */
static void bias_k(const orc_model *m, const tree_t *t, const fk_t *k, const double *v, double *bias)
{
    double w[ORC_NB][3], al[ORC_NB][3], ao[ORC_NB][3];  /* angular vel, angular acc, acc of body origin */
    /* base: world omega = R omega_b; at zero generalized acceleration the base origin
       does not accelerate and alpha = d/dt(R omega_b) = R (omega_b x omega_b) = 0 */
    matvec3(k->R[0], v + 3, w[0]);
    for (int i = 0; i < 3; ++i) { al[0][i] = 0; ao[0][i] = 0; }
    for (int b = 1; b < ORC_NB; ++b) {
        int P = t->parent[b];
        double qd = v[5 + b];
        double r[3] = {k->p[b][0] - k->p[P][0], k->p[b][1] - k->p[P][1], k->p[b][2] - k->p[P][2]};
        double t1[3], t2[3], t3[3];
        /* acceleration of the joint point as a point of the parent */
        cross3(al[P], r, t1);
        cross3(w[P], r, t2);
        cross3(w[P], t2, t3);
        for (int i = 0; i < 3; ++i) ao[b][i] = ao[P][i] + t1[i] + t3[i];
        double aq[3] = {k->a[b][0] * qd, k->a[b][1] * qd, k->a[b][2] * qd};
        cross3(w[P], aq, t1);   /* the axis turns with the parent */
        for (int i = 0; i < 3; ++i) { w[b][i] = w[P][i] + aq[i]; al[b][i] = al[P][i] + t1[i]; }
    }
    memset(bias, 0, sizeof(double) * ORC_NV);
    double g[3] = {0, 0, -m->gravity};
    double Jv[3 * ORC_NV], Jw[3 * ORC_NV];
    for (int b = 0; b < ORC_NB; ++b) {
        if (t->mass[b] == 0) continue;
        double r[3] = {k->c[b][0] - k->p[b][0], k->c[b][1] - k->p[b][1], k->c[b][2] - k->p[b][2]};
        double t1[3], t2[3], t3[3], ac[3], F[3], N[3], Iw_w[3], Ia[3];
        cross3(al[b], r, t1);
        cross3(w[b], r, t2);
        cross3(w[b], t2, t3);
        for (int i = 0; i < 3; ++i) ac[i] = ao[b][i] + t1[i] + t3[i];
        for (int i = 0; i < 3; ++i) F[i] = t->mass[b] * (ac[i] - g[i]);
        matvec3(k->Iw[b], w[b], Iw_w);
        matvec3(k->Iw[b], al[b], Ia);
        cross3(w[b], Iw_w, t1);
        for (int i = 0; i < 3; ++i) N[i] = Ia[i] + t1[i];
        jac_point(t, k, b, k->c[b], Jv);
        jac_rot(t, k, b, Jw);
        for (int j = 0; j < ORC_NV; ++j)
            for (int r2 = 0; r2 < 3; ++r2) bias[j] += Jv[r2 * ORC_NV + j] * F[r2] + Jw[r2 * ORC_NV + j] * N[r2];
    }
}

/* dense Cholesky solve of SPD A (n x n, row-major, overwritten) */
static int chol_solve(int n, double *A, double *b)
{
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0)) return -1;
        double d = sqrt(s);
        A[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / d;
        }
    }
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= A[i * n + k] * b[k];
        b[i] = s / A[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= A[k * n + i] * b[k];
        b[i] = s / A[i * n + i];
    }
    return 0;
}

int orc_nx(const orc_model *m) { return m->scene == ORC_SCENE_FREE_BOX ? ORC_NX_BOX : ORC_NX; }

/* ------------------------------------------------------------------ */
/* public rigid-body entry points                                       */
/* ------------------------------------------------------------------ */
void orc_fk(const orc_model *m, const double *q, double *R, double *pos, double *com)
{
    tree_t t; fk_t k;
    build_tree(m, &t);
    fk_compute(m, &t, q, &k);
    for (int b = 0; b < ORC_NB; ++b) {
        if (R) memcpy(R + 9 * b, k.R[b], sizeof(double) * 9);
        if (pos) memcpy(pos + 3 * b, k.p[b], sizeof(double) * 3);
        if (com) memcpy(com + 3 * b, k.c[b], sizeof(double) * 3);
    }
}

static void foot_center(const orc_model *m, const fk_t *k, int leg, double out[3])
{
    int b = 3 + 3 * leg;
    double loc[3] = {0, 0, -m->calf_len}, w[3];
    matvec3(k->R[b], loc, w);
    for (int i = 0; i < 3; ++i) out[i] = k->p[b][i] + w[i];
}

void orc_foot_positions(const orc_model *m, const double *q, double *feet)
{
    tree_t t; fk_t k;
    build_tree(m, &t);
    fk_compute(m, &t, q, &k);
    for (int l = 0; l < 4; ++l) foot_center(m, &k, l, feet + 3 * l);
}

void orc_mass_matrix(const orc_model *m, const double *q, double *M)
{
    tree_t t; fk_t k;
    build_tree(m, &t);
    fk_compute(m, &t, q, &k);
    mass_matrix_k(&t, &k, M);
}

void orc_bias(const orc_model *m, const double *q, const double *v, double *b)
{
    tree_t t; fk_t k;
    build_tree(m, &t);
    fk_compute(m, &t, q, &k);
    bias_k(m, &t, &k, v, b);
}

double orc_kinetic_energy(const orc_model *m, const double *q, const double *v)
{
    double M[ORC_NV * ORC_NV];
    orc_mass_matrix(m, q, M);
    double T = 0;
    for (int i = 0; i < ORC_NV; ++i)
        for (int j = 0; j < ORC_NV; ++j) T += 0.5 * v[i] * M[i * ORC_NV + j] * v[j];
    return T;
}

/* move along generalized velocity v for time t: p += t v_w, quat <- quat (x) exp(t w_b), q_j += t v_j */
void orc_retract(const double *q, const double *v, double t, double *qo)
{
    double phi[3] = {t * v[3], t * v[4], t * v[5]}, dq[4], nq[4];
    for (int i = 0; i < 3; ++i) qo[i] = q[i] + t * v[i];
    quat_exp(phi, dq);
    quat_mul(q + 3, dq, nq);
    for (int i = 0; i < 4; ++i) qo[3 + i] = nq[i];
    for (int j = 0; j < 12; ++j) qo[7 + j] = q[7 + j] + t * v[6 + j];
}

/* kinetic energy from body velocities obtained by central finite differences of the
   forward kinematics along v (independent of the Jacobians used above) */
double orc_kinetic_energy_fd(const orc_model *m, const double *q, const double *v, double eps)
{
    tree_t t; fk_t kp, km;
    double qp[ORC_NQ], qm[ORC_NQ];
    build_tree(m, &t);
    orc_retract(q, v, eps, qp);
    orc_retract(q, v, -eps, qm);
    fk_compute(m, &t, qp, &kp);
    fk_compute(m, &t, qm, &km);
    tree_t *tt = &t;
    fk_t k0;
    fk_compute(m, &t, q, &k0);
    double T = 0;
    for (int b = 0; b < ORC_NB; ++b) {
        if (tt->mass[b] == 0) continue;
        double vc[3];
        for (int i = 0; i < 3; ++i) vc[i] = (kp.c[b][i] - km.c[b][i]) / (2 * eps);
        /* skew part of R(+eps) R(-eps)^T = 2 eps [w x] + O(eps^3) */
        double A[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0;
                for (int l = 0; l < 3; ++l) s += kp.R[b][3 * i + l] * km.R[b][3 * j + l];
                A[3 * i + j] = s;
            }
        double w[3] = {(A[7] - A[5]) / (4 * eps), (A[2] - A[6]) / (4 * eps), (A[3] - A[1]) / (4 * eps)};
        double Iw[3];
        matvec3(k0.Iw[b], w, Iw);
        T += 0.5 * tt->mass[b] * dot3(vc, vc) + 0.5 * dot3(w, Iw);
    }
    return T;
}

double orc_potential_energy(const orc_model *m, const double *q)
{
    tree_t t; fk_t k;
    build_tree(m, &t);
    fk_compute(m, &t, q, &k);
    double V = 0;
    for (int b = 0; b < ORC_NB; ++b) V += t.mass[b] * m->gravity * k.c[b][2];
    return V;
}

void orc_momentum(const orc_model *m, const double *q, const double *v, double *P, double *Lo)
{
    tree_t t; fk_t k;
    build_tree(m, &t);
    fk_compute(m, &t, q, &k);
    double Jv[3 * ORC_NV], Jw[3 * ORC_NV];
    for (int i = 0; i < 3; ++i) P[i] = Lo[i] = 0;
    for (int b = 0; b < ORC_NB; ++b) {
        if (t.mass[b] == 0) continue;
        jac_point(&t, &k, b, k.c[b], Jv);
        jac_rot(&t, &k, b, Jw);
        double vc[3] = {0, 0, 0}, w[3] = {0, 0, 0}, Iw[3], mv[3], cxmv[3];
        for (int r = 0; r < 3; ++r)
            for (int j = 0; j < ORC_NV; ++j) { vc[r] += Jv[r * ORC_NV + j] * v[j]; w[r] += Jw[r * ORC_NV + j] * v[j]; }
        matvec3(k.Iw[b], w, Iw);
        for (int i = 0; i < 3; ++i) mv[i] = t.mass[b] * vc[i];
        cross3(k.c[b], mv, cxmv);
        for (int i = 0; i < 3; ++i) { P[i] += mv[i]; Lo[i] += cxmv[i] + Iw[i]; }
    }
}

void orc_accel(const orc_model *m, const double *q, const double *v, const double *tau_gen, double *vdot)
{
    double M[ORC_NV * ORC_NV], b[ORC_NV];
    orc_mass_matrix(m, q, M);
    orc_bias(m, q, v, b);
    for (int i = 0; i < ORC_NV; ++i) vdot[i] = tau_gen[i] - b[i];
    chol_solve(ORC_NV, M, vdot);
}

/* time derivative of the configuration for generalized velocity v */
static void qdot_of(const double *q, const double *v, double *qd)
{
    for (int i = 0; i < 3; ++i) qd[i] = v[i];
    double wq[4] = {0, v[3], v[4], v[5]}, o[4];
    quat_mul(q + 3, wq, o);
    for (int i = 0; i < 4; ++i) qd[3 + i] = 0.5 * o[i];
    for (int j = 0; j < 12; ++j) qd[7 + j] = v[6 + j];
}

/* classical RK4 on the continuous contact-free dynamics; with spring != 0 the joint
   torques are kp (target - q) (conservative springs), otherwise tau_gen is constant */
void orc_rk4(const orc_model *m, double *q, double *v, const double *tau_gen, double dt, int nsteps, int spring,
             const double *kp_target, double kp)
{
    double kq[4][ORC_NQ], kv[4][ORC_NV], qs[ORC_NQ], vs[ORC_NV], tg[ORC_NV];
    for (int s = 0; s < nsteps; ++s) {
        for (int st = 0; st < 4; ++st) {
            double h = (st == 0) ? 0 : (st == 3 ? dt : 0.5 * dt);
            for (int i = 0; i < ORC_NQ; ++i) qs[i] = q[i] + (st ? h * kq[st - 1][i] : 0);
            for (int i = 0; i < ORC_NV; ++i) vs[i] = v[i] + (st ? h * kv[st - 1][i] : 0);
            for (int i = 0; i < ORC_NV; ++i) tg[i] = tau_gen ? tau_gen[i] : 0;
            if (spring)
                for (int j = 0; j < 12; ++j) tg[6 + j] += kp * (kp_target[j] - qs[7 + j]);
            qdot_of(qs, vs, kq[st]);
            orc_accel(m, qs, vs, tg, kv[st]);
        }
        for (int i = 0; i < ORC_NQ; ++i) q[i] += dt / 6 * (kq[0][i] + 2 * kq[1][i] + 2 * kq[2][i] + kq[3][i]);
        for (int i = 0; i < ORC_NV; ++i) v[i] += dt / 6 * (kv[0][i] + 2 * kv[1][i] + 2 * kv[2][i] + kv[3][i]);
    }
}

/* ------------------------------------------------------------------ */
/* contact                                                              */
/* ------------------------------------------------------------------ */
/* Terrain query for a sphere of radius r centred at c (r = 0 for a point).
   Flat ground is z = 0.  The heightfield is bilinear on a regular grid, clamped to the
   edge value outside it (zero slope there); its normal comes from the bilinear gradient
   and the depth is the vertical gap scaled by n_z. */
static int terrain(const orc_model *m, const double c[3], double r, double *delta, double n[3])
{
    double h = 0, gx = 0, gy = 0;
    if (m->scene == ORC_SCENE_HEIGHTFIELD) {
        int nx = m->hf_nx, ny = m->hf_ny;
        double fx = (c[0] - m->hf_x0) / m->hf_cell, fy = (c[1] - m->hf_y0) / m->hf_cell;
        int inx = 1, iny = 1;
        if (fx < 0) { fx = 0; inx = 0; }
        if (fx > nx - 1) { fx = nx - 1; inx = 0; }
        if (fy < 0) { fy = 0; iny = 0; }
        if (fy > ny - 1) { fy = ny - 1; iny = 0; }
        int i0 = (int)floor(fx), j0 = (int)floor(fy);
        if (i0 > nx - 2) i0 = nx - 2;
        if (j0 > ny - 2) j0 = ny - 2;
        double tx = fx - i0, ty = fy - j0;
        double h00 = m->hf[j0 * nx + i0], h10 = m->hf[j0 * nx + i0 + 1];
        double h01 = m->hf[(j0 + 1) * nx + i0], h11 = m->hf[(j0 + 1) * nx + i0 + 1];
        h = (1 - ty) * ((1 - tx) * h00 + tx * h10) + ty * ((1 - tx) * h01 + tx * h11);
        if (inx) gx = ((1 - ty) * (h10 - h00) + ty * (h11 - h01)) / m->hf_cell;
        if (iny) gy = ((1 - tx) * (h01 - h00) + tx * (h11 - h10)) / m->hf_cell;
    }
    double nn = sqrt(gx * gx + gy * gy + 1.0);
    n[0] = -gx / nn; n[1] = -gy / nn; n[2] = 1.0 / nn;
    *delta = (h + r - c[2]) * n[2];
    return *delta > 0;
}

/* sphere (centre c, radius r) against an oriented box (centre p, rotation R, half sizes h).
   n points from the box toward the sphere. */
static int sphere_box(const double c[3], double r, const double p[3], const double R[9], const double h[3],
                      double *delta, double n[3])
{
    double d[3] = {c[0] - p[0], c[1] - p[1], c[2] - p[2]}, cl[3];
    matTvec3(R, d, cl);
    int inside = fabs(cl[0]) <= h[0] && fabs(cl[1]) <= h[1] && fabs(cl[2]) <= h[2];
    double nl[3] = {0, 0, 0};
    if (!inside) {
        double qn[3], e[3];
        for (int i = 0; i < 3; ++i) {
            qn[i] = cl[i] < -h[i] ? -h[i] : (cl[i] > h[i] ? h[i] : cl[i]);
            e[i] = cl[i] - qn[i];
        }
        double dist = sqrt(dot3(e, e));
        if (dist >= r) return 0;
        *delta = r - dist;
        for (int i = 0; i < 3; ++i) nl[i] = e[i] / dist;
    } else {
        int best = 0;
        double depth = h[0] - fabs(cl[0]);
        for (int i = 1; i < 3; ++i)
            if (h[i] - fabs(cl[i]) < depth) { depth = h[i] - fabs(cl[i]); best = i; }
        nl[best] = cl[best] >= 0 ? 1.0 : -1.0;
        *delta = r + depth;
    }
    matvec3(R, nl, n);
    return 1;
}

/* point x inside an oriented box: depth of the shallowest face and its outward normal */
static int point_box(const double x[3], const double p[3], const double R[9], const double h[3],
                     double *delta, double n[3])
{
    double d[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]}, cl[3];
    matTvec3(R, d, cl);
    if (!(fabs(cl[0]) < h[0] && fabs(cl[1]) < h[1] && fabs(cl[2]) < h[2])) return 0;
    int best = 0;
    double depth = h[0] - fabs(cl[0]);
    for (int i = 1; i < 3; ++i)
        if (h[i] - fabs(cl[i]) < depth) { depth = h[i] - fabs(cl[i]); best = i; }
    double nl[3] = {0, 0, 0};
    nl[best] = cl[best] >= 0 ? 1.0 : -1.0;
    matvec3(R, nl, n);
    *delta = depth;
    return 1;
}

/* Penalty contact: a linear spring-damper along the normal while the pair overlaps,
     Fn = k delta - c v_n   (delta > 0),
   and tanh-smoothed Coulomb friction  F_t = -mu max(Fn, 0) tanh(s) t,  s = |v_t| / v_s.
   The damper acts for the whole overlap (it may pull while the bodies separate), so
   the normal law stays linear where the implicit step linearises it; a clamp at
   Fn >= 0 makes feet chatter on and off at dt = 0.01-0.02 s.  Friction enters as a
   viscous force with the secant coefficient mu Fn tanh(s) / (s v_s) taken at the start
   of the step: D = c n n^T + mu Fn tanh(s)/(s v_s) (I - n n^T), which stays stable when
   the foot slides (the tangent slope sech^2(s) vanishes there and the friction force
   would reverse the sliding velocity in one step).  Returns 0 when not overlapping. */
static int contact_law(const orc_model *m, double delta, const double n[3], const double vrel[3], double F[3],
                       double D[9])
{
    if (!(delta > 0)) return 0;
    double vn = dot3(n, vrel);
    double Fn = m->k * delta - m->c * vn;
    double Fp = Fn > 0 ? Fn : 0.0;
    double vt[3] = {vrel[0] - vn * n[0], vrel[1] - vn * n[1], vrel[2] - vn * n[2]};
    double s = sqrt(dot3(vt, vt)) / m->vs;
    double phi = (s < 1e-4) ? 1 - s * s / 3 : tanh(s) / s;     /* tanh(s)/s */
    double eta = m->mu * Fp / m->vs * phi;                      /* secant viscosity */
    for (int i = 0; i < 3; ++i) F[i] = Fn * n[i] - eta * vt[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double nn = n[i] * n[j];
            D[3 * i + j] = m->c * nn + eta * ((i == j ? 1.0 : 0.0) - nn);
        }
    return 1;
}

typedef struct {
    const orc_model *m;
    const tree_t *t;
    const fk_t *k;
    const double *v;       /* robot generalized velocity */
    double Rb[9];          /* free box */
    const double *pb, *vb, *wb;
    double *f, *D;         /* robot generalized force / damping (18, 18x18) */
    double *fbox, *Dbox;   /* box (6, 6x6) */
    double Ftot_robot[3], Ftot_box[3];
    int n_active;
} cstate_t;

#define BODY_NONE (-1)
#define BODY_BOX (-2)

static void box_jac(const cstate_t *s, const double x[3], double J[18])
{
    /* world velocity of box point x = v + (R w_b) x (x - p) ; columns [v(3), w_b(3)] */
    memset(J, 0, sizeof(double) * 18);
    double r[3] = {x[0] - s->pb[0], x[1] - s->pb[1], x[2] - s->pb[2]};
    for (int i = 0; i < 3; ++i) J[i * 6 + i] = 1.0;
    for (int e = 0; e < 3; ++e) {
        double ew[3] = {s->Rb[e], s->Rb[3 + e], s->Rb[6 + e]}, col[3];
        cross3(ew, r, col);
        for (int i = 0; i < 3; ++i) J[i * 6 + 3 + e] = col[i];
    }
}

static void point_velocity(const cstate_t *s, int body, const double x[3], double vel[3])
{
    vel[0] = vel[1] = vel[2] = 0;
    if (body == BODY_NONE) return;
    if (body == BODY_BOX) {
        double J[18];
        box_jac(s, x, J);
        double vv[6] = {s->vb[0], s->vb[1], s->vb[2], s->wb[0], s->wb[1], s->wb[2]};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 6; ++j) vel[i] += J[i * 6 + j] * vv[j];
        return;
    }
    double J[3 * ORC_NV];
    jac_point(s->t, s->k, body, x, J);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < ORC_NV; ++j) vel[i] += J[i * ORC_NV + j] * s->v[j];
}

/* apply force sgn*F at point x of body, add J^T Dc J to its damping block */
static void apply_to_body(cstate_t *s, int body, const double x[3], const double F[3], double sgn, const double Dc[9])
{
    if (body == BODY_NONE) return;
    if (body == BODY_BOX) {
        double J[18];
        box_jac(s, x, J);
        for (int j = 0; j < 6; ++j)
            for (int r = 0; r < 3; ++r) s->fbox[j] += sgn * J[r * 6 + j] * F[r];
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double acc = 0;
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) acc += J[r * 6 + i] * Dc[3 * r + c] * J[c * 6 + j];
                s->Dbox[i * 6 + j] += acc;
            }
        for (int i = 0; i < 3; ++i) s->Ftot_box[i] += sgn * F[i];
        return;
    }
    double J[3 * ORC_NV];
    jac_point(s->t, s->k, body, x, J);
    for (int j = 0; j < ORC_NV; ++j)
        for (int r = 0; r < 3; ++r) s->f[j] += sgn * J[r * ORC_NV + j] * F[r];
    for (int i = 0; i < ORC_NV; ++i)
        for (int j = 0; j < ORC_NV; ++j) {
            double acc = 0;
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) acc += J[r * ORC_NV + i] * Dc[3 * r + c] * J[c * ORC_NV + j];
            s->D[i * ORC_NV + j] += acc;
        }
    for (int i = 0; i < 3; ++i) s->Ftot_robot[i] += sgn * F[i];
}

/* one contact pair: body A receives +F at pc, body B receives -F; n points from B to A */
static void pair(cstate_t *s, int A, int B, const double pc[3], const double n[3], double delta)
{
    double va[3], vbv[3], vrel[3], F[3], Dc[9];
    point_velocity(s, A, pc, va);
    point_velocity(s, B, pc, vbv);
    for (int i = 0; i < 3; ++i) vrel[i] = va[i] - vbv[i];
    if (!contact_law(s->m, delta, n, vrel, F, Dc)) return;
    s->n_active++;
    apply_to_body(s, A, pc, F, 1.0, Dc);
    apply_to_body(s, B, pc, F, -1.0, Dc);
}

static void trunk_corner(const orc_model *m, const fk_t *k, int i, double out[3])
{
    double loc[3] = {(i & 1 ? 0.5 : -0.5) * m->trunk_size[0], (i & 2 ? 0.5 : -0.5) * m->trunk_size[1],
                     (i & 4 ? 0.5 : -0.5) * m->trunk_size[2]}, w[3];
    matvec3(k->R[0], loc, w);
    for (int j = 0; j < 3; ++j) out[j] = k->p[0][j] + w[j];
}

static void box_corner(const cstate_t *s, const double h[3], int i, double out[3])
{
    double loc[3] = {(i & 1 ? 1 : -1) * h[0], (i & 2 ? 1 : -1) * h[1], (i & 4 ? 1 : -1) * h[2]}, w[3];
    matvec3(s->Rb, loc, w);
    for (int j = 0; j < 3; ++j) out[j] = s->pb[j] + w[j];
}

static void all_contacts(cstate_t *s)
{
    const orc_model *m = s->m;
    const fk_t *k = s->k;
    double c[3], n[3], pc[3], delta;
    const double I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    /* feet (spheres on the calves) and trunk corners against the terrain */
    for (int l = 0; l < 4; ++l) {
        foot_center(m, k, l, c);
        if (terrain(m, c, m->foot_r, &delta, n)) {
            for (int i = 0; i < 3; ++i) pc[i] = c[i] - m->foot_r * n[i];
            pair(s, 3 + 3 * l, BODY_NONE, pc, n, delta);
        }
    }
    for (int i = 0; i < 8; ++i) {
        trunk_corner(m, k, i, c);
        if (terrain(m, c, 0.0, &delta, n)) pair(s, 0, BODY_NONE, c, n, delta);
    }
    if (m->scene == ORC_SCENE_STATIC_BOX) {
        for (int l = 0; l < 4; ++l) {
            foot_center(m, k, l, c);
            if (sphere_box(c, m->foot_r, m->sbox_center, I3, m->sbox_half, &delta, n)) {
                for (int i = 0; i < 3; ++i) pc[i] = c[i] - m->foot_r * n[i];
                pair(s, 3 + 3 * l, BODY_NONE, pc, n, delta);
            }
        }
        for (int i = 0; i < 8; ++i) {
            trunk_corner(m, k, i, c);
            if (point_box(c, m->sbox_center, I3, m->sbox_half, &delta, n)) pair(s, 0, BODY_NONE, c, n, delta);
        }
    }
    if (m->scene == ORC_SCENE_FREE_BOX) {
        for (int l = 0; l < 4; ++l) {
            foot_center(m, k, l, c);
            if (sphere_box(c, m->foot_r, s->pb, s->Rb, m->box_half, &delta, n)) {
                for (int i = 0; i < 3; ++i) pc[i] = c[i] - m->foot_r * n[i];
                pair(s, 3 + 3 * l, BODY_BOX, pc, n, delta);
            }
        }
        for (int i = 0; i < 8; ++i) {
            trunk_corner(m, k, i, c);
            if (point_box(c, s->pb, s->Rb, m->box_half, &delta, n)) pair(s, 0, BODY_BOX, c, n, delta);
        }
        double th[3] = {0.5 * m->trunk_size[0], 0.5 * m->trunk_size[1], 0.5 * m->trunk_size[2]};
        for (int i = 0; i < 8; ++i) {
            box_corner(s, m->box_half, i, c);
            if (point_box(c, k->p[0], k->R[0], th, &delta, n)) pair(s, BODY_BOX, 0, c, n, delta);
        }
        for (int i = 0; i < 8; ++i) {
            box_corner(s, m->box_half, i, c);
            if (terrain(m, c, 0.0, &delta, n)) pair(s, BODY_BOX, BODY_NONE, c, n, delta);
        }
    }
}

static void integrate_base(double dt, const double *p, const double *quat, const double *vw, const double *wb,
                           double *po, double *quato)
{
    double phi[3] = {dt * wb[0], dt * wb[1], dt * wb[2]}, dq[4], nq[4];
    for (int i = 0; i < 3; ++i) po[i] = p[i] + dt * vw[i];
    quat_exp(phi, dq);
    quat_mul(quat, dq, nq);
    double nrm = sqrt(nq[0] * nq[0] + nq[1] * nq[1] + nq[2] * nq[2] + nq[3] * nq[3]);
    for (int i = 0; i < 4; ++i) quato[i] = nq[i] / nrm;
}

static void contact_setup(const orc_model *m, const tree_t *t, const fk_t *k, const double *x, cstate_t *s,
                          double *f, double *D, double *fbox, double *Dbox)
{
    memset(s, 0, sizeof(*s));
    s->m = m; s->t = t; s->k = k; s->v = x + ORC_NQ;
    s->f = f; s->D = D; s->fbox = fbox; s->Dbox = Dbox;
    if (m->scene == ORC_SCENE_FREE_BOX) {
        s->pb = x + ORC_NX; s->vb = x + ORC_NX + 7; s->wb = x + ORC_NX + 10;
        quat_to_mat(x + ORC_NX + 3, s->Rb);
    }
}

int orc_step(const orc_model *m, const double *x, const double *u, double kp, double kd, double dt, double *xo,
             double *tau_out)
{
    tree_t t; fk_t k;
    build_tree(m, &t);
    const double *q = x, *v = x + ORC_NQ;
    fk_compute(m, &t, q, &k);
    double M[ORC_NV * ORC_NV], b[ORC_NV], f[ORC_NV], D[ORC_NV * ORC_NV];
    double fbox[6] = {0}, Dbox[36] = {0};
    mass_matrix_k(&t, &k, M);
    bias_k(m, &t, &k, v, b);
    double tau[12];
    for (int j = 0; j < 12; ++j) tau[j] = kp * (u[j] - q[7 + j]) - kd * v[6 + j];
    for (int i = 0; i < ORC_NV; ++i) f[i] = -b[i];
    for (int j = 0; j < 12; ++j) f[6 + j] += tau[j];
    memset(D, 0, sizeof(D));
    for (int j = 0; j < 12; ++j) D[(6 + j) * ORC_NV + 6 + j] = kd;
    cstate_t s;
    contact_setup(m, &t, &k, x, &s, f, D, fbox, Dbox);
    all_contacts(&s);
    double A[ORC_NV * ORC_NV], dv[ORC_NV];
    for (int i = 0; i < ORC_NV * ORC_NV; ++i) A[i] = M[i] + dt * D[i];
    for (int i = 0; i < ORC_NV; ++i) dv[i] = dt * f[i];
    int rc = chol_solve(ORC_NV, A, dv);
    double vn[ORC_NV];
    for (int i = 0; i < ORC_NV; ++i) vn[i] = v[i] + dv[i];
    integrate_base(dt, q, q + 3, vn, vn + 3, xo, xo + 3);
    for (int j = 0; j < 12; ++j) xo[7 + j] = q[7 + j] + dt * vn[6 + j];
    memcpy(xo + ORC_NQ, vn, sizeof(vn));
    if (m->scene == ORC_SCENE_FREE_BOX) {
        const double *xb = x + ORC_NX;
        double mb = m->box_mass, sx = 2 * m->box_half[0], sy = 2 * m->box_half[1], sz = 2 * m->box_half[2];
        double Ib[3] = {mb * (sy * sy + sz * sz) / 12, mb * (sx * sx + sz * sz) / 12, mb * (sx * sx + sy * sy) / 12};
        double Ab[36], dvb[6];
        /* box: M = diag(m, m, m, Ib), bias = [m g e_z ; w x I w] */
        const double *wb = xb + 10;
        double Iw[3] = {Ib[0] * wb[0], Ib[1] * wb[1], Ib[2] * wb[2]}, gyro[3];
        cross3(wb, Iw, gyro);
        double bb[6] = {0, 0, mb * m->gravity, gyro[0], gyro[1], gyro[2]};
        for (int i = 0; i < 36; ++i) Ab[i] = dt * Dbox[i];
        for (int i = 0; i < 3; ++i) { Ab[i * 6 + i] += mb; Ab[(3 + i) * 6 + 3 + i] += Ib[i]; }
        for (int i = 0; i < 6; ++i) dvb[i] = dt * (fbox[i] - bb[i]);
        if (chol_solve(6, Ab, dvb)) rc = -1;
        double vbn[6];
        for (int i = 0; i < 6; ++i) vbn[i] = xb[7 + i] + dvb[i];
        integrate_base(dt, xb, xb + 3, vbn, vbn + 3, xo + ORC_NX, xo + ORC_NX + 3);
        memcpy(xo + ORC_NX + 7, vbn, sizeof(vbn));
    }
    if (tau_out) memcpy(tau_out, tau, sizeof(tau));
    return rc;
}

/* the linear system of one step, A dv = dt f (robot part), for diagnostics and tests */
int orc_step_system(const orc_model *m, const double *x, const double *u, double kp, double kd, double dt,
                    double *A_out, double *rhs_out)
{
    tree_t t; fk_t k;
    build_tree(m, &t);
    const double *q = x, *v = x + ORC_NQ;
    fk_compute(m, &t, q, &k);
    double M[ORC_NV * ORC_NV], b[ORC_NV], f[ORC_NV], D[ORC_NV * ORC_NV];
    double fbox[6] = {0}, Dbox[36] = {0};
    mass_matrix_k(&t, &k, M);
    bias_k(m, &t, &k, v, b);
    for (int i = 0; i < ORC_NV; ++i) f[i] = -b[i];
    for (int j = 0; j < 12; ++j) f[6 + j] += kp * (u[j] - q[7 + j]) - kd * v[6 + j];
    memset(D, 0, sizeof(D));
    for (int j = 0; j < 12; ++j) D[(6 + j) * ORC_NV + 6 + j] = kd;
    cstate_t s;
    contact_setup(m, &t, &k, x, &s, f, D, fbox, Dbox);
    all_contacts(&s);
    for (int i = 0; i < ORC_NV * ORC_NV; ++i) A_out[i] = M[i] + dt * D[i];
    for (int i = 0; i < ORC_NV; ++i) rhs_out[i] = dt * f[i];
    return s.n_active;
}

int orc_step_system_box(const orc_model *m, const double *x, const double *u, double kp, double kd, double dt,
                        double *A_out, double *rhs_out)
{
    (void)u; (void)kp; (void)kd;
    if (m->scene != ORC_SCENE_FREE_BOX) return -1;
    tree_t t; fk_t k;
    build_tree(m, &t);
    fk_compute(m, &t, x, &k);
    double f[ORC_NV] = {0}, D[ORC_NV * ORC_NV] = {0}, fbox[6] = {0}, Dbox[36] = {0};
    cstate_t s;
    contact_setup(m, &t, &k, x, &s, f, D, fbox, Dbox);
    all_contacts(&s);
    const double *xb = x + ORC_NX, *wb = xb + 10;
    double mb = m->box_mass, sx = 2 * m->box_half[0], sy = 2 * m->box_half[1], sz = 2 * m->box_half[2];
    double Ib[3] = {mb * (sy * sy + sz * sz) / 12, mb * (sx * sx + sz * sz) / 12, mb * (sx * sx + sy * sy) / 12};
    double Iw[3] = {Ib[0] * wb[0], Ib[1] * wb[1], Ib[2] * wb[2]}, gyro[3];
    cross3(wb, Iw, gyro);
    double bb[6] = {0, 0, mb * m->gravity, gyro[0], gyro[1], gyro[2]};
    for (int i = 0; i < 36; ++i) A_out[i] = dt * Dbox[i];
    for (int i = 0; i < 3; ++i) { A_out[i * 6 + i] += mb; A_out[(3 + i) * 6 + 3 + i] += Ib[i]; }
    for (int i = 0; i < 6; ++i) rhs_out[i] = dt * (fbox[i] - bb[i]);
    return s.n_active;
}

void orc_contact_total(const orc_model *m, const double *x, double *F_robot, double *F_box, int *n_active)
{
    tree_t t; fk_t k;
    build_tree(m, &t);
    fk_compute(m, &t, x, &k);
    double f[ORC_NV] = {0}, D[ORC_NV * ORC_NV] = {0}, fbox[6] = {0}, Dbox[36] = {0};
    cstate_t s;
    contact_setup(m, &t, &k, x, &s, f, D, fbox, Dbox);
    all_contacts(&s);
    for (int i = 0; i < 3; ++i) { F_robot[i] = s.Ftot_robot[i]; F_box[i] = s.Ftot_box[i]; }
    *n_active = s.n_active;
}

int orc_terrain(const orc_model *m, const double *c, double r, double *delta, double *n)
{
    return terrain(m, c, r, delta, n);
}

int orc_sphere_box(const double *c, double r, const double *p, const double *quat, const double *h, double *delta,
                   double *n)
{
    double R[9];
    quat_to_mat(quat, R);
    return sphere_box(c, r, p, R, h, delta, n);
}

int orc_point_box(const double *x, const double *p, const double *quat, const double *h, double *delta, double *n)
{
    double R[9];
    quat_to_mat(quat, R);
    return point_box(x, p, R, h, delta, n);
}

int orc_contact_law(const orc_model *m, double delta, const double *n, const double *vrel, double *F, double *D)
{
    return contact_law(m, delta, n, vrel, F, D);
}

/* ------------------------------------------------------------------ */
/* counter-based Gaussian sampler                                       */
/* ------------------------------------------------------------------ */
/* Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw (SC'11): ten rounds of
   two 32x32->64 multiplies with the Weyl-sequence key schedule. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Noise for sample n, dimension d (d = joint * nk + knot): counter (d/4, n, step,
   instance), key = seed; 24-bit uniforms (x >> 8 + 1/2) / 2^24 and Box-Muller on the
   pairs (0,1), (2,3). */
static double u24(uint32_t x) { return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0); }

void orc_philox_raw(const orc_params *p, uint32_t step, uint32_t *raw)
{
    int D = 12 * p->nk, nb = (D + 3) / 4;
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    for (int n = 0; n < p->K; ++n)
        for (int c = 0; c < nb; ++c) {
            uint32_t ctr[4] = {(uint32_t)c, (uint32_t)n, step, p->instance};
            orc_philox4x32_10(ctr, key, raw + (size_t)n * nb * 4 + 4 * c);
        }
}

void orc_sample_eps(const orc_params *p, uint32_t step, double *eps)
{
    int D = 12 * p->nk, nb = (D + 3) / 4;
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    const double two_pi = 6.283185307179586476925286766559;
    for (int n = 0; n < p->K; ++n)
        for (int c = 0; c < nb; ++c) {
            uint32_t ctr[4] = {(uint32_t)c, (uint32_t)n, step, p->instance}, o[4];
            orc_philox4x32_10(ctr, key, o);
            double g[4];
            for (int h = 0; h < 2; ++h) {
                double r = sqrt(-2.0 * log(u24(o[2 * h])));
                double a = two_pi * u24(o[2 * h + 1]);
                g[2 * h] = r * cos(a);
                g[2 * h + 1] = r * sin(a);
            }
            for (int i = 0; i < 4; ++i)
                if (4 * c + i < D) eps[(size_t)n * D + 4 * c + i] = g[i];
        }
}

/* ------------------------------------------------------------------ */
/* spline (Sec. III-B)                                                  */
/* ------------------------------------------------------------------ */
/* Not-a-knot cubic spline through nk knots evenly spaced on [0, T]: solve directly for
   the 4(nk-1) segment polynomial coefficients from interpolation, C1 and C2 continuity
   and the not-a-knot conditions (C3 continuity at the second and second-to-last knots).
   With 3 knots the spline is the interpolating parabola and with 2 knots the line. */
static int gauss_solve(int n, double *A, double *b)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0) return -1;
        if (piv != c) {
            for (int j = 0; j < n; ++j) { double t = A[c * n + j]; A[c * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int j = r + 1; j < n; ++j) s -= A[r * n + j] * b[j];
        b[r] = s / A[r * n + r];
    }
    return 0;
}

static void spline_coeffs(int nk, double T, const double *y, double *coef /* 4(nk-1) */)
{
    int ns = nk - 1, n = 4 * ns;
    double hk = T / ns;
    double *A = calloc((size_t)n * n, sizeof(double));
    double *b = calloc((size_t)n, sizeof(double));
    int row = 0;
    for (int s = 0; s < ns; ++s) {     /* interpolation at both ends of each segment */
        A[row * n + 4 * s] = 1; b[row++] = y[s];
        for (int p = 0; p < 4; ++p) A[row * n + 4 * s + p] = pow(hk, p);
        b[row++] = y[s + 1];
    }
    for (int s = 0; s + 1 < ns; ++s) { /* C1, C2 at interior knots */
        A[row * n + 4 * s + 1] = 1; A[row * n + 4 * s + 2] = 2 * hk; A[row * n + 4 * s + 3] = 3 * hk * hk;
        A[row * n + 4 * (s + 1) + 1] = -1; row++;
        A[row * n + 4 * s + 2] = 2; A[row * n + 4 * s + 3] = 6 * hk;
        A[row * n + 4 * (s + 1) + 2] = -2; row++;
    }
    if (ns == 1) {
        A[row * n + 2] = 1; row++;
        A[row * n + 3] = 1; row++;
    } else if (ns == 2) {
        A[row * n + 3] = 1; row++;
        A[row * n + 7] = 1; row++;
    } else {
        A[row * n + 3] = 1; A[row * n + 7] = -1; row++;
        A[row * n + 4 * (ns - 2) + 3] = 1; A[row * n + 4 * (ns - 1) + 3] = -1; row++;
    }
    gauss_solve(n, A, b);
    memcpy(coef, b, sizeof(double) * n);
    free(A); free(b);
}

void orc_spline_eval(int nk, double T, const double *knots, double t, double *out)
{
    int ns = nk - 1;
    double hk = T / ns;
    double *coef = malloc(sizeof(double) * 4 * ns);
    spline_coeffs(nk, T, knots, coef);
    int s = (int)floor(t / hk);
    if (s < 0) s = 0;
    if (s > ns - 1) s = ns - 1;
    double tau = t - s * hk;
    *out = coef[4 * s] + tau * (coef[4 * s + 1] + tau * (coef[4 * s + 2] + tau * coef[4 * s + 3]));
    free(coef);
}

/* Lower-order interpolations of the same knots (Sec. III-B): the segment is the knot
   interval containing t (the last interval for t at or past the horizon end). */
void orc_interp_eval(int basis, int nk, double T, const double *knots, double t, double *out)
{
    if (basis == 0) {
        orc_spline_eval(nk, T, knots, t, out);
        return;
    }
    if (basis == 3) {           /* direct: one value per control step, knot i applies on
                                   [i dt, (i + 1) dt) with dt = T / nk, the last one held */
        int s = (int)floor(t / (T / nk) + 1e-9);
        if (s < 0) s = 0;
        if (s > nk - 1) s = nk - 1;
        *out = knots[s];
        return;
    }
    double hk = T / (nk - 1);
    if (basis == 2) {           /* zeroth order: the knot at the start of the interval; a time
                                   within 1e-9 of an interval of a knot time counts as on it */
        int s = (int)floor(t / hk + 1e-9);
        if (s < 0) s = 0;
        if (s > nk - 1) s = nk - 1;
        *out = knots[s];
        return;
    }
    int s = (int)floor(t / hk); /* linear */
    if (s < 0) s = 0;
    if (s > nk - 2) s = nk - 2;
    double a = (t - s * hk) / hk;
    *out = (1 - a) * knots[s] + a * knots[s + 1];
}

void orc_basis_matrix(int basis, int nk, int H, double dt, double *B)
{
    double T = H * dt;
    double *e = calloc(nk, sizeof(double));
    for (int j = 0; j < nk; ++j) {
        memset(e, 0, sizeof(double) * nk);
        e[j] = 1;
        for (int k = 0; k < H; ++k) orc_interp_eval(basis, nk, T, e, k * dt, &B[k * nk + j]);
    }
    free(e);
}

void orc_spline_basis(int nk, int H, double dt, double *B) { orc_basis_matrix(0, nk, H, dt, B); }

/* warm-start shift: new knot j = old interpolant at t_j + dt, held at the horizon end
   (knot times t_j = j T / (nk - 1); direct values sit at t_j = j dt) */
void orc_shift_matrix_b(int basis, int nk, int H, double dt, double *S)
{
    double T = H * dt;
    double *e = calloc(nk, sizeof(double));
    for (int j = 0; j < nk; ++j) {
        memset(e, 0, sizeof(double) * nk);
        e[j] = 1;
        for (int i = 0; i < nk; ++i) {
            double t = (basis == 3 ? i * dt : i * T / (nk - 1)) + dt;
            if (t > T) t = T;
            orc_interp_eval(basis, nk, T, e, t, &S[i * nk + j]);
        }
    }
    free(e);
}

void orc_shift_matrix(int nk, int H, double dt, double *S) { orc_shift_matrix_b(0, nk, H, dt, S); }

/* ------------------------------------------------------------------ */
/* cost, rollout, MPPI                                                  */
/* ------------------------------------------------------------------ */
/* running cost: height, uprightness (R_zz), forward velocity, torque; the box-push
   scene replaces the velocity term by the distance to the box and adds the box's
   squared distance to the goal (xy only) */
double orc_stage_cost(const orc_model *m, const orc_params *p, const double *x, const double *tau)
{
    double z = x[2], qx = x[4], qy = x[5];
    double Rzz = 1 - 2 * (qx * qx + qy * qy);
    double t2 = 0;
    for (int j = 0; j < 12; ++j) t2 += tau[j] * tau[j];
    double l = p->w_h * (z - p->h_ref) * (z - p->h_ref) + p->w_o * (1 - Rzz * Rzz) + p->w_tau * t2;
    if (m->scene == ORC_SCENE_FREE_BOX) {
        double bx = x[ORC_NX], by = x[ORC_NX + 1];
        double dx = x[0] - bx, dy = x[1] - by, gx = bx - p->goal[0], gy = by - p->goal[1];
        l += p->w_reach * (dx * dx + dy * dy) + p->w_box * (gx * gx + gy * gy);
    } else {
        double vx = x[ORC_NQ];
        l += p->w_v * (vx - p->v_ref) * (vx - p->v_ref);
    }
    return l;
}

static int all_finite(const double *x, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

static double rollout_with_basis(const orc_model *m, const orc_params *p, const double *B, const double *x0,
                                 const double *theta, double *traj)
{
    int nx = orc_nx(m), nk = p->nk;
    double x[ORC_NX_BOX], xn[ORC_NX_BOX], u[12], tau[12];
    memcpy(x, x0, sizeof(double) * nx);
    if (traj) memcpy(traj, x0, sizeof(double) * nx);
    double L = 0;
    for (int k = 0; k < p->H; ++k) {
        for (int j = 0; j < 12; ++j) {
            double s = 0;
            for (int i = 0; i < nk; ++i) s += B[k * nk + i] * theta[j * nk + i];
            u[j] = s;
        }
        int rc = orc_step(m, x, u, p->kp, p->kd, p->dt, xn, tau);
        L += p->dt * orc_stage_cost(m, p, xn, tau);
        if (traj) memcpy(traj + (size_t)(k + 1) * nx, xn, sizeof(double) * nx);
        if (rc || !all_finite(xn, nx) || !isfinite(L)) {
            if (traj)
                for (int kk = k + 1; kk <= p->H; ++kk)
                    for (int i = 0; i < nx; ++i) traj[(size_t)kk * nx + i] = NAN;
            return INFINITY;
        }
        memcpy(x, xn, sizeof(double) * nx);
    }
    return L;
}

double orc_rollout(const orc_model *m, const orc_params *p, const double *x0, const double *theta, double *traj)
{
    double *B = malloc(sizeof(double) * p->H * p->nk);
    orc_basis_matrix(p->basis, p->nk, p->H, p->dt, B);
    double L = rollout_with_basis(m, p, B, x0, theta, traj);
    free(B);
    return L;
}

/* theta_0 = mu (the nominal), theta_n = mu + sigma eps_n for n >= 1 */
void orc_rollout_batch(const orc_model *m, const orc_params *p, const double *x0, const double *mu,
                       const double *eps, double *costs, double *traj, int nthreads)
{
    int D = 12 * p->nk, nx = orc_nx(m);
    double *B = malloc(sizeof(double) * p->H * p->nk);
    orc_basis_matrix(p->basis, p->nk, p->H, p->dt, B);
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int n = 0; n < p->K; ++n) {
        double *theta = malloc(sizeof(double) * D);
        for (int d = 0; d < D; ++d) theta[d] = mu[d] + (n ? p->sigma * eps[(size_t)n * D + d] : 0.0);
        costs[n] = rollout_with_basis(m, p, B, x0, theta, traj ? traj + (size_t)n * (p->H + 1) * nx : NULL);
        free(theta);
    }
    (void)nthreads;
    free(B);
}

/* Eq. 1: w_n = exp(-(L_n - L_min)/lambda) / sum; non-finite costs get zero weight.
   Returns 1 if no cost is finite (all weights zero). */
int orc_weights(int K, double lambda, const double *costs, double *w)
{
    double Lmin = INFINITY;
    for (int n = 0; n < K; ++n)
        if (isfinite(costs[n]) && costs[n] < Lmin) Lmin = costs[n];
    if (!isfinite(Lmin)) {
        for (int n = 0; n < K; ++n) w[n] = 0;
        return 1;
    }
    double s = 0;
    for (int n = 0; n < K; ++n) {
        w[n] = isfinite(costs[n]) ? exp(-(costs[n] - Lmin) / lambda) : 0.0;
        s += w[n];
    }
    for (int n = 0; n < K; ++n) w[n] /= s;
    return 0;
}

/* Eq. 2 applied to the knots: mu' = sum_n w_n theta_n */
int orc_update(const orc_params *p, const double *costs, const double *mu, const double *eps, double *mu_out,
               double *w_out)
{
    int K = p->K, D = 12 * p->nk;
    double *w = malloc(sizeof(double) * K);
    int rc = orc_weights(K, p->lambda, costs, w);
    if (rc) {
        memcpy(mu_out, mu, sizeof(double) * D);
    } else {
        for (int d = 0; d < D; ++d) {
            double s = 0;
            for (int n = 0; n < K; ++n) {
                double th = mu[d] + (n ? p->sigma * eps[(size_t)n * D + d] : 0.0);
                s += w[n] * th;
            }
            mu_out[d] = s;
        }
    }
    if (w_out) memcpy(w_out, w, sizeof(double) * K);
    free(w);
    return rc;
}

/* first control u = spline(mu', 0) and warm start mu <- S mu' (Algorithm 1, last steps) */
void orc_shift(const orc_params *p, const double *mu_prime, double *mu_out, double *u0)
{
    int nk = p->nk;
    double T = p->H * p->dt;
    double *S = malloc(sizeof(double) * nk * nk);
    orc_shift_matrix_b(p->basis, nk, p->H, p->dt, S);
    for (int j = 0; j < 12; ++j) {
        if (u0) orc_interp_eval(p->basis, nk, T, mu_prime + j * nk, 0.0, &u0[j]);
        for (int i = 0; i < nk; ++i) {
            double s = 0;
            for (int l = 0; l < nk; ++l) s += S[i * nk + l] * mu_prime[j * nk + l];
            mu_out[j * nk + i] = s;
        }
    }
    free(S);
}

int orc_mppi_step(const orc_model *m, const orc_params *p, uint32_t step, const double *x0, double *mu,
                  double *u0, double *costs, int nthreads)
{
    int K = p->K, D = 12 * p->nk;
    double *eps = malloc(sizeof(double) * (size_t)K * D);
    double *L = costs ? costs : malloc(sizeof(double) * K);
    double *mup = malloc(sizeof(double) * D);
    orc_sample_eps(p, step, eps);
    orc_rollout_batch(m, p, x0, mu, eps, L, NULL, nthreads);
    int rc = orc_update(p, L, mu, eps, mup, NULL);
    orc_shift(p, mup, mu, u0);
    free(eps);
    free(mup);
    if (!costs) free(L);
    return rc;
}

/* Learned-proposal step (Sec. V-B names richer sampling distributions as future work; the
   network-given proposal is the reading of this library).  With Kp samples around the
   proposal: theta_0 = c (proposal mean), theta_1 = mu (shifted nominal), and
   theta_n = c + sd * eps_n for 2 <= n < Kp, eps from the same counters as a plain step.
   With gate 0, when L(c) is finite and L(c) <= L(mu) the Eq. 1-2 update runs over these
   Kp samples, otherwise the step falls back to a plain step with K samples around mu;
   gate 2 does the same with the least cost over the samples other than mu in place of
   L(c); gate 1 always takes the Kp samples.  *accepted reports which branch ran; costs_p (Kp)
   and costs (K, fallback only) are optional outputs. */
int orc_mppi_step_proposal(const orc_model *m, const orc_params *p, uint32_t step, const double *x0, double *mu,
                           const double *center, const double *sd, int Kp, int gate, double *u0, double *costs_p,
                           double *costs, int *accepted, int nthreads)
{
    int D = 12 * p->nk, nx = orc_nx(m);
    orc_params q = *p;
    q.K = Kp;
    double *eps = malloc(sizeof(double) * (size_t)Kp * D);
    double *L = malloc(sizeof(double) * Kp);
    double *theta = malloc(sizeof(double) * (size_t)Kp * D);
    double *B = malloc(sizeof(double) * p->H * p->nk);
    orc_sample_eps(&q, step, eps);
    orc_basis_matrix(p->basis, p->nk, p->H, p->dt, B);
    for (int n = 0; n < Kp; ++n)
        for (int d = 0; d < D; ++d)
            theta[(size_t)n * D + d] = n == 0 ? center[d] : n == 1 ? mu[d] : center[d] + sd[d] * eps[(size_t)n * D + d];
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int n = 0; n < Kp; ++n) L[n] = rollout_with_basis(m, p, B, x0, theta + (size_t)n * D, NULL);
    (void)nthreads;
    (void)nx;
    if (costs_p) memcpy(costs_p, L, sizeof(double) * Kp);
    /* gate 0: the centre's cost against the nominal's; gate 2: the least cost over the
       proposal's samples other than the nominal; gate 1: always the proposal */
    double Lg = L[0];
    if (gate == 2) {
        Lg = INFINITY;
        for (int n = 0; n < Kp; ++n)
            if (n != 1 && isfinite(L[n]) && L[n] < Lg) Lg = L[n];
    }
    int acc = gate == 1 || (Kp >= 2 && isfinite(Lg) && Lg <= L[1]);
    if (accepted) *accepted = acc;
    int rc;
    if (acc) {
        double *w = malloc(sizeof(double) * Kp), *mup = malloc(sizeof(double) * D);
        rc = orc_weights(Kp, p->lambda, L, w);
        for (int d = 0; d < D; ++d) {
            double s = 0;
            for (int n = 0; n < Kp; ++n) s += w[n] * theta[(size_t)n * D + d];
            mup[d] = s;
        }
        orc_shift(p, mup, mu, u0);
        free(w);
        free(mup);
    } else {
        rc = orc_mppi_step(m, p, step, x0, mu, u0, costs, nthreads);
    }
    free(eps); free(L); free(theta); free(B);
    return rc;
}
