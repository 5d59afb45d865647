/*
 * Oracle for the learned sampling proposal: a plain FP64 multilayer perceptron
 * 40 -> 512 -> 512 -> 512 -> 512 -> 144 with SiLU activations, its Gaussian negative
 * log-likelihood loss, the gradient by reverse-mode differentiation written out layer by
 * layer, and the Adam update (Kingma and Ba, 2015).  TEST INFRASTRUCTURE ONLY.
 *
 * The paper names sampling from more sophisticated distributions as future work
 * (Sec. V-B) and cites learning an offline sampling distribution (Sec. II-B); the
 * network maps (state, command) to a mean and log standard deviation for each knot.
 *
 * Parameter layout (flat): for each layer l, W_l (fan_in x fan_out, row-major, W[i][o])
 * followed by b_l (fan_out).  With `bf16` set, weights and the inputs of every layer are
 * rounded to bfloat16 (round to nearest even) and the sums of products are kept in
 * double: the rounding points of a BF16-operand / wide-accumulator kernel.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "mppi_oracle.h"

#define NL 5
static const int DIMS[NL + 1] = {40, 512, 512, 512, 512, 144};

int orc_mlp_n_params(void)
{
    int n = 0;
    for (int l = 0; l < NL; ++l) n += DIMS[l] * DIMS[l + 1] + DIMS[l + 1];
    return n;
}

static double bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return f;  /* inf / nan unchanged */
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return f;
}

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double dsilu(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

/* forward for a batch; Z (pre-activations) and A (layer inputs) optionally kept:
   A[l] has B x DIMS[l] entries (A[0] = X), Z[l] has B x DIMS[l+1] */
static void forward(const double *P, int B, const double *X, double *out, int bf, double **A, double **Z)
{
    const double *in = X;
    double *buf_in = NULL;
    int off = 0;
    for (int l = 0; l < NL; ++l) {
        int fi = DIMS[l], fo = DIMS[l + 1];
        const double *W = P + off, *b = P + off + fi * fo;
        double *z = malloc(sizeof(double) * B * fo);
        for (int r = 0; r < B; ++r)
            for (int o = 0; o < fo; ++o) {
                double s = b[o];
                for (int i = 0; i < fi; ++i) {
                    double a = in[r * fi + i], w = W[i * fo + o];
                    if (bf) { a = bf16(a); w = bf16(w); }
                    s += a * w;
                }
                z[r * fo + o] = s;
            }
        if (A) {
            A[l] = malloc(sizeof(double) * B * fi);
            memcpy(A[l], in, sizeof(double) * B * fi);
        }
        if (Z) {
            Z[l] = malloc(sizeof(double) * B * fo);
            memcpy(Z[l], z, sizeof(double) * B * fo);
        }
        off += fi * fo + fo;
        if (l < NL - 1) {
            for (int k = 0; k < B * fo; ++k) z[k] = silu(z[k]);
            free(buf_in);
            buf_in = z;
            in = z;
        } else {
            memcpy(out, z, sizeof(double) * B * fo);
            free(z);
        }
    }
    free(buf_in);
}

void orc_mlp_forward(const double *P, int B, const double *X, double *out, int bf)
{
    forward(P, B, X, out, bf, NULL, NULL);
}

/* Gaussian NLL averaged over batch and the 72 outputs:
     L = mean( (y - m)^2 / (2 e^{2s}) + s ),   out = [m (72), s (72)]
   log-std s is used as produced (the caller clamps it when sampling). */
double orc_mlp_loss(const double *P, int B, const double *X, const double *Y, int bf)
{
    double *out = malloc(sizeof(double) * B * 144);
    forward(P, B, X, out, bf, NULL, NULL);
    double L = 0;
    for (int r = 0; r < B; ++r)
        for (int d = 0; d < 72; ++d) {
            double m = out[r * 144 + d], s = out[r * 144 + 72 + d], e = Y[r * 72 + d] - m;
            L += 0.5 * e * e * exp(-2 * s) + s;
        }
    free(out);
    return L / (B * 72.0);
}

/* gradient of the loss with respect to all parameters (reverse mode, layer by layer) */
double orc_mlp_grad(const double *P, int B, const double *X, const double *Y, double *G, int bf)
{
    double *A[NL], *Z[NL];
    double *out = malloc(sizeof(double) * B * 144);
    forward(P, B, X, out, bf, A, Z);
    double L = 0;
    double *dz = malloc(sizeof(double) * B * 144);
    const double inv = 1.0 / (B * 72.0);
    for (int r = 0; r < B; ++r)
        for (int d = 0; d < 72; ++d) {
            double m = out[r * 144 + d], s = out[r * 144 + 72 + d], e = Y[r * 72 + d] - m;
            double q = e * e * exp(-2 * s);
            L += 0.5 * q + s;
            dz[r * 144 + d] = -e * exp(-2 * s) * inv;
            dz[r * 144 + 72 + d] = (1.0 - q) * inv;
        }
    int offs[NL], off = 0;
    for (int l = 0; l < NL; ++l) {
        offs[l] = off;
        off += DIMS[l] * DIMS[l + 1] + DIMS[l + 1];
    }
    memset(G, 0, sizeof(double) * off);
    for (int l = NL - 1; l >= 0; --l) {
        int fi = DIMS[l], fo = DIMS[l + 1];
        const double *W = P + offs[l];
        double *gW = G + offs[l], *gb = G + offs[l] + fi * fo;
        for (int r = 0; r < B; ++r)
            for (int o = 0; o < fo; ++o) {
                double g = dz[r * fo + o];
                gb[o] += g;
                if (bf) g = bf16(g);
                for (int i = 0; i < fi; ++i) {
                    double a = A[l][r * fi + i];
                    if (bf) a = bf16(a);
                    gW[i * fo + o] += a * g;
                }
            }
        if (l > 0) {
            double *da = malloc(sizeof(double) * B * fi);
            for (int r = 0; r < B; ++r)
                for (int i = 0; i < fi; ++i) {
                    double s = 0;
                    for (int o = 0; o < fo; ++o) {
                        double w = W[i * fo + o], g = dz[r * fo + o];
                        if (bf) { w = bf16(w); g = bf16(g); }
                        s += g * w;
                    }
                    /* A[l] = silu(Z[l-1]) */
                    da[r * fi + i] = s * dsilu(Z[l - 1][r * fi + i]);
                }
            free(dz);
            dz = da;
        }
    }
    free(dz);
    for (int l = 0; l < NL; ++l) { free(A[l]); free(Z[l]); }
    free(out);
    return L * inv;
}

/* Adam with bias correction; t is the 1-based step number */
void orc_adam(double *P, double *m, double *v, const double *G, int n, int t, double lr, double b1, double b2,
              double eps)
{
    double c1 = 1 - pow(b1, t), c2 = 1 - pow(b2, t);
    for (int i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1 - b1) * G[i];
        v[i] = b2 * v[i] + (1 - b2) * G[i] * G[i];
        P[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* Network input: the robot state with the base xy taken relative to the episode origin,
   followed by the 3-dim command (forward, lateral, yaw-rate references), standardised
   with the dataset statistics. */
void orc_policy_features(const double *x, const double *cmd, const double *origin, const double *in_mean,
                         const double *in_std, double *feat)
{
    double f[40];
    for (int i = 0; i < 37; ++i) f[i] = x[i];
    f[0] -= origin[0];
    f[1] -= origin[1];
    for (int i = 0; i < 3; ++i) f[37 + i] = cmd[i];
    for (int i = 0; i < 40; ++i) feat[i] = (f[i] - in_mean[i]) / in_std[i];
}

/* Network output -> sampling distribution of a controller with nk knots per joint.
   out = [standardised means (12 x 6, joint-major), standardised log-stds (12 x 6)].
   Means are de-standardised (m = y sigma_y + mean_y) and log-stds shifted by log sigma_y;
   both are resampled from the 6-knot spline to nk knots evenly spaced over the same
   horizon (the knot times are at the same fractions of the horizon, so the map does not
   depend on H dt); the log-std is clamped to [log 0.02, log sigma_max]. */
void orc_policy_head(const double *out, const double *out_mean, const double *out_std, int nk, double sigma_max,
                     double *center, double *sd)
{
    const double lo = log(0.02), hi = log(sigma_max);
    for (int j = 0; j < 12; ++j) {
        double m6[6], s6[6];
        for (int k = 0; k < 6; ++k) {
            int d = j * 6 + k;
            m6[k] = out[d] * out_std[d] + out_mean[d];
            s6[k] = out[72 + d] + log(out_std[d]);
        }
        for (int i = 0; i < nk; ++i) {
            double t = (double)i / (nk - 1), m, s;
            if (nk == 6) {
                m = m6[i];
                s = s6[i];
            } else {
                orc_spline_eval(6, 1.0, m6, t, &m);
                orc_spline_eval(6, 1.0, s6, t, &s);
            }
            if (s < lo) s = lo;
            if (s > hi) s = hi;
            center[j * nk + i] = m;
            sd[j * nk + i] = exp(s);
        }
    }
}
