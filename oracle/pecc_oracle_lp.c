/*
 * pecc_oracle_lp.c -- plain FP64 CPU oracle for the learned proposal that
 * chooses which circles the solution-space exploring step of SED relocates
 * (the perturbation of Sec. 5, Alg. 5, here a relocation of 5 % of the
 * circles chosen by a small network instead of a shift of every circle).
 * The network is not part of the paper; the definitions below are the
 * project's, written out plainly.
 *
 * TEST INFRASTRUCTURE ONLY.  Like pecc_oracle.c this file is the independent
 * checker of the HIP library; only the test suite, the smoke entry point and
 * the CPU-baseline leg of the benchmark load it, and it shares no code with
 * the GPU path.  Build with -O2 -ffp-contract=off.
 *
 * Contents
 *   oracle_bf16_round   round-to-nearest-even of FP32 to BF16
 *   oracle_features     8 local features of a candidate (circle i, point q)
 *   oracle_mlp_forward  8 -> 64 -> 64 -> 1 network, erf GELU, FP64
 *   oracle_mlp_grad     mean binary cross-entropy on the logits and its
 *                       gradient by the chain rule, FP64
 *   oracle_adam         one Adam step (Kingma & Ba), FP64
 *   oracle_propose      top-k distinct circles by score and their relocation
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const double kPi = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* BF16: keep the upper 16 bits of the FP32 pattern after adding half an     */
/* ulp of the result, with ties going to the even result.  Infinities pass   */
/* through; NaN stays NaN.                                                   */
/* ------------------------------------------------------------------------ */
static float bf16_of(float w)
{
    if (w != w) return w;                             /* nan stays nan */
    uint32_t u;
    memcpy(&u, &w, 4);
    uint32_t keep_even = (u >> 16) & 1u;              /* infinities round to themselves */
    u += 0x7fffu + keep_even;
    u &= 0xffff0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

void oracle_bf16_round(int64_t count, const float *in, float *out)
{
    for (int64_t i = 0; i < count; ++i) out[i] = bf16_of(in[i]);
}

/* ------------------------------------------------------------------------ */
/* Features of one candidate: a circle i of the current layout and a point   */
/* q uniform in the disk of radius R - 1 where i would be moved.  Four       */
/* quantities, each taken once around i at its own centre c_i (j != i) and   */
/* once around q (again over j != i, i.e. with i already lifted out):        */
/*   e      overlap energy of a unit circle there: sum_j max(0, 2 - l)^2 +   */
/*          max(0, rho + 1 - R)^2, entered as log10(e + 1e-20) / 20 + 1      */
/*   near   number of j with l^2 < 2.3^2 (the neighbor cutoff)               */
/*   gap    (R - 1 - rho) / R                                                */
/*   dens   number of j with l^2 < 4^2, divided by 16 pi                     */
/* Output per candidate: [e, near, gap, dens] at c_i then at q.              */
/* Distances use FP64 on the FP32 coordinates, dx*dx + dy*dy, both compares  */
/* strict.                                                                   */
/* ------------------------------------------------------------------------ */
static void features_at(int n, const float *xy, double R, int skip, double px, double py,
                        double *f)
{
    double e = 0.0;
    int near = 0, dens = 0;
    for (int j = 0; j < n; ++j) {
        if (j == skip) continue;
        double dx = px - (double)xy[2 * j];
        double dy = py - (double)xy[2 * j + 1];
        double l2 = dx * dx + dy * dy;
        if (l2 < 4.0) {
            double d = 2.0 - sqrt(l2);
            e += d * d;
        }
        if (l2 < 5.29) ++near;
        if (l2 < 16.0) ++dens;
    }
    double rho = sqrt(px * px + py * py);
    double d0 = rho + 1.0 - R;
    if (d0 > 0.0) e += d0 * d0;
    f[0] = log10(e + 1e-20) / 20.0 + 1.0;
    f[1] = (double)near;
    f[2] = (R - 1.0 - rho) / R;
    f[3] = (double)dens / (16.0 * kPi);
}

/* Returns 0, or -1 when a candidate names a circle outside [0, n). */
int oracle_features(int n, const float *xy, double R, int ncand, const int32_t *cand_circle,
                    const float *cand_dest, double *feat)
{
    for (int c = 0; c < ncand; ++c) {
        int i = cand_circle[c];
        if (i < 0 || i >= n) return -1;
        features_at(n, xy, R, i, (double)xy[2 * i], (double)xy[2 * i + 1], feat + 8 * c);
        features_at(n, xy, R, i, (double)cand_dest[2 * c], (double)cand_dest[2 * c + 1],
                    feat + 8 * c + 4);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The network.  Parameters in one flat vector of 4801 values:               */
/*   W1 [64][8]  at 0      b1 [64] at 512                                    */
/*   W2 [64][64] at 576    b2 [64] at 4672                                   */
/*   W3 [64]     at 4736   b3      at 4800                                   */
/* a1 = W1 x + b1, h1 = gelu(a1), a2 = W2 h1 + b2, h2 = gelu(a2),            */
/* z = W3 . h2 + b3, gelu(t) = t Phi(t) = t (1 + erf(t / sqrt 2)) / 2.       */
/* With round_bf16 set, the three weight matrices enter as their BF16        */
/* roundings (of the parameter taken as FP32); biases are used as given.     */
/* ------------------------------------------------------------------------ */
enum { NIN = 8, NH = 64, OW1 = 0, OB1 = 512, OW2 = 576, OB2 = 4672, OW3 = 4736, OB3 = 4800,
       NPARAM = 4801 };

static double gelu(double t) { return 0.5 * t * (1.0 + erf(t / sqrt(2.0))); }

static double gelu_prime(double t)
{
    double Phi = 0.5 * (1.0 + erf(t / sqrt(2.0)));
    double phi = exp(-0.5 * t * t) / sqrt(2.0 * kPi);
    return Phi + t * phi;
}

static void effective_params(const double *params, int round_bf16, double *w)
{
    for (int k = 0; k < NPARAM; ++k) {
        int is_weight = (k < OB1) || (k >= OW2 && k < OB2) || (k >= OW3 && k < OB3);
        w[k] = (round_bf16 && is_weight) ? (double)bf16_of((float)params[k]) : params[k];
    }
}

/* One row forward; keeps the pre-activations for the backward pass. */
static double forward_row(const double *w, const double *x, double *a1, double *h1, double *a2,
                          double *h2)
{
    for (int j = 0; j < NH; ++j) {
        double s = w[OB1 + j];
        for (int k = 0; k < NIN; ++k) s += w[OW1 + j * NIN + k] * x[k];
        a1[j] = s;
        h1[j] = gelu(s);
    }
    for (int j = 0; j < NH; ++j) {
        double s = w[OB2 + j];
        for (int k = 0; k < NH; ++k) s += w[OW2 + j * NH + k] * h1[k];
        a2[j] = s;
        h2[j] = gelu(s);
    }
    double z = w[OB3];
    for (int j = 0; j < NH; ++j) z += w[OW3 + j] * h2[j];
    return z;
}

void oracle_mlp_forward(const double *params, int round_bf16, int64_t rows, const double *x,
                        double *z)
{
    double w[NPARAM], a1[NH], h1[NH], a2[NH], h2[NH];
    effective_params(params, round_bf16, w);
    for (int64_t r = 0; r < rows; ++r) z[r] = forward_row(w, x + NIN * r, a1, h1, a2, h2);
}

/* Loss: mean over rows of the binary cross-entropy of sigmoid(z) against the
 * label y in {0, 1}, written on the logit as max(z, 0) - z y + log(1 + e^-|z|).
 * grad receives d loss / d params (with respect to the weights as used, i.e.
 * the BF16 roundings when round_bf16 is set).  Returns the loss. */
double oracle_mlp_grad(const double *params, int round_bf16, int64_t rows, const double *x,
                       const double *y, double *grad)
{
    double w[NPARAM], a1[NH], h1[NH], a2[NH], h2[NH], d2[NH], d1[NH];
    effective_params(params, round_bf16, w);
    memset(grad, 0, sizeof(double) * NPARAM);
    double loss = 0.0;
    if (rows <= 0) return 0.0;
    for (int64_t r = 0; r < rows; ++r) {
        const double *xr = x + NIN * r;
        double z = forward_row(w, xr, a1, h1, a2, h2);
        loss += fmax(z, 0.0) - z * y[r] + log1p(exp(-fabs(z)));
        double dz = (1.0 / (1.0 + exp(-z)) - y[r]) / (double)rows;
        /* output layer */
        grad[OB3] += dz;
        for (int j = 0; j < NH; ++j) {
            grad[OW3 + j] += dz * h2[j];
            d2[j] = dz * w[OW3 + j] * gelu_prime(a2[j]);
        }
        /* hidden layer 2 */
        for (int j = 0; j < NH; ++j) {
            grad[OB2 + j] += d2[j];
            for (int k = 0; k < NH; ++k) grad[OW2 + j * NH + k] += d2[j] * h1[k];
        }
        for (int k = 0; k < NH; ++k) {
            double s = 0.0;
            for (int j = 0; j < NH; ++j) s += w[OW2 + j * NH + k] * d2[j];
            d1[k] = s * gelu_prime(a1[k]);     /* s = d loss / d h1[k] */
        }
        /* hidden layer 1 */
        for (int j = 0; j < NH; ++j) {
            grad[OB1 + j] += d1[j];
            for (int k = 0; k < NIN; ++k) grad[OW1 + j * NIN + k] += d1[j] * xr[k];
        }
    }
    return loss / (double)rows;
}

/* ------------------------------------------------------------------------ */
/* Adam, step number t >= 1: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,   */
/* p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).              */
/* ------------------------------------------------------------------------ */
void oracle_adam(int count, double *p, double *m, double *v, const double *g, int t, double lr,
                 double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)t);
    double c2 = 1.0 - pow(b2, (double)t);
    for (int k = 0; k < count; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * g[k];
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
        p[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Proposal: choose up to k distinct circles among the candidates.           */
/* Each circle that some candidate names is represented by its best           */
/* candidate: highest score, the lowest candidate index among equal scores.  */
/* Circles are ranked by that score (high first), equal scores by the lower  */
/* candidate index, and the first k are taken.  Without scores (NULL), or    */
/* when any score is NaN, every score counts as equal: the choice is then    */
/* the first k distinct circles in candidate order, a uniform random subset  */
/* because the candidates are drawn uniformly.                               */
/* selected[] receives the chosen candidate indices in rank order; xy_out    */
/* (nullable) is xy with each chosen circle moved to its candidate's point.  */
/* Returns the number chosen.                                                */
/* ------------------------------------------------------------------------ */
int oracle_propose(int n, const float *xy, int ncand, const int32_t *cand_circle,
                   const float *cand_dest, const float *scores, int k, int32_t *selected,
                   float *xy_out)
{
    int use_scores = scores != NULL;
    for (int c = 0; use_scores && c < ncand; ++c)
        if (scores[c] != scores[c]) use_scores = 0;
    int *best = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) best[i] = -1;
    for (int c = 0; c < ncand; ++c) {
        int i = cand_circle[c];
        if (i < 0 || i >= n) continue;
        if (best[i] < 0) { best[i] = c; continue; }
        if (use_scores && scores[c] > scores[best[i]]) best[i] = c;
    }
    if (xy_out) memcpy(xy_out, xy, sizeof(float) * 2 * (size_t)n);
    int taken = 0;
    for (; taken < k; ++taken) {
        /* the remaining best-ranked circle: a plain selection scan */
        int pick = -1;
        for (int i = 0; i < n; ++i) {
            int c = best[i];
            if (c < 0) continue;
            if (pick < 0) { pick = i; continue; }
            int cp = best[pick];
            float sc = use_scores ? scores[c] : 0.0f, sp = use_scores ? scores[cp] : 0.0f;
            if (sc > sp || (sc == sp && c < cp)) pick = i;
        }
        if (pick < 0) break;
        int c = best[pick];
        selected[taken] = c;
        if (xy_out) {
            xy_out[2 * pick] = cand_dest[2 * c];
            xy_out[2 * pick + 1] = cand_dest[2 * c + 1];
        }
        best[pick] = -1;
    }
    free(best);
    return taken;
}
