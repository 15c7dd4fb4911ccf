/*
 * pecc_oracle_part.c -- plain CPU oracle for the k-batch partitions of the
 * geometric batch optimization (Sec. 4.1: sector, annulus, fence, random),
 * the batch descent of Alg. 1 with the batches visited one after another,
 * and the adaptive neighbor maintenance ANM (Sec. 4.3, Alg. 3).
 *
 * TEST INFRASTRUCTURE ONLY, like the other oracle files: only the test
 * suite, the smoke entry point and the CPU-baseline leg of the benchmark
 * load it; it shares no code with the GPU path.  Build with -O2
 * -ffp-contract=off.
 *
 * Partitions (Sec. 4.1): the circles are sorted by a key and cut into k
 * consecutive runs; batch p holds floor(n/k) + [p < n mod k] circles, so
 * every size is floor(n/k) or ceil(n/k) and the larger batches come first.
 * The order is a strict total order (equal keys: lower index first) and
 * the rank of circle i is the number of circles that precede it.
 *   sector   the polar angle atan2(y, x) in (-pi, pi], ascending.  The
 *            arctan(y/x) of the text cannot tell opposite quadrants apart,
 *            so the full angle is used.  It is compared exactly, without
 *            evaluating an angle: the classes y < 0, (y = 0, x >= 0),
 *            y > 0, (y = 0, x < 0) come in this order, and inside the
 *            first and third class a precedes b iff x_a y_b - y_a x_b > 0
 *            (products of FP32 values are exact in FP64, and the sign of
 *            their rounded difference is the exact sign);
 *   annulus  x^2 + y^2 in FP64 (the distance's square: same order);
 *   fence    x;
 *   random   word 0 of Philox4x64-10 at counter (i, instance, 0, 2^62),
 *            key (seed, 0): a uniformly random order, hence random batches
 *            of the same sizes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "pecc_oracle_types.h"

enum { PART_SECTOR = 0, PART_ANNULUS = 1, PART_FENCE = 2, PART_RANDOM = 3 };

void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double oracle_energy_grad(int n, const double *xy, double R, double rad,
                          double *e_pair, double *e_cont, double *grad);
double oracle_batch_energy_grad(int n, const double *xy, double R, double rad,
                                const int32_t *mask, double *grad);
void oracle_two_loop(int dim, int k, const double *S, const double *Y,
                     const double *g, double *r);

static int angle_class(double x, double y)
{
    if (y < 0.0) return 0;
    if (y > 0.0) return 2;
    return x < 0.0 ? 3 : 1;
}

/* Does circle a come before circle b in the order of `kind`? */
static int precedes(int kind, const float *xy, const uint64_t *rnd, int a, int b)
{
    const double xa = xy[2 * a], ya = xy[2 * a + 1], xb = xy[2 * b], yb = xy[2 * b + 1];
    int c = 0;   /* -1: a first, 1: b first, 0: equal keys */
    if (kind == PART_SECTOR) {
        const int ca = angle_class(xa, ya), cb = angle_class(xb, yb);
        if (ca != cb) {
            c = ca < cb ? -1 : 1;
        } else if (ca == 0 || ca == 2) {
            const double p = xa * yb, q = ya * xb;
            const double cross = p - q;
            c = cross > 0.0 ? -1 : (cross < 0.0 ? 1 : 0);
        }
    } else if (kind == PART_ANNULUS) {
        const double ra = xa * xa + ya * ya, rb = xb * xb + yb * yb;
        c = ra < rb ? -1 : (ra > rb ? 1 : 0);
    } else if (kind == PART_FENCE) {
        c = xa < xb ? -1 : (xa > xb ? 1 : 0);
    } else {
        c = rnd[a] < rnd[b] ? -1 : (rnd[a] > rnd[b] ? 1 : 0);
    }
    return c < 0 || (c == 0 && a < b);
}

/* Batch of the circle of rank r: batches of floor(n/k) + [p < n mod k]. */
static int batch_of_rank(int r, int n, int k)
{
    const int q = n / k, rem = n % k;
    const int big = rem * (q + 1);
    return r < big ? r / (q + 1) : rem + (r - big) / q;
}

/* batch_of[i] in [0, k) for the partition `kind` of one instance (index
 * `instance` within its batch, used by the random kind only).  Returns 0,
 * or -2 for an invalid kind or k. */
int oracle_partition(int n, const float *xy, int kind, int k, uint64_t seed, int32_t instance,
                     int32_t *batch_of)
{
    if (k < 1 || kind < 0 || kind > 3) return -2;
    uint64_t *rnd = NULL;
    if (kind == PART_RANDOM) {
        rnd = malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
        if (!rnd) return -1;
        const uint64_t key[2] = { seed, 0 };
        for (int i = 0; i < n; ++i) {
            const uint64_t ctr[4] = { (uint64_t)(uint32_t)i, (uint64_t)(uint32_t)instance, 0,
                                      1ULL << 62 };
            uint64_t w[4];
            oracle_philox4x64(ctr, key, w);
            rnd[i] = w[0];
        }
    }
    for (int i = 0; i < n; ++i) {
        int rank = 0;
        for (int j = 0; j < n; ++j)
            if (j != i && precedes(kind, xy, rnd, j, i)) ++rank;
        batch_of[i] = batch_of_rank(rank, n, k);
    }
    free(rnd);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Neighbor structure Gamma (Sec. 4.3) at FP64 positions: for every circle,  */
/* the ascending list of j != i with (x_i - x_j)^2 + (y_i - y_j)^2 < l_cut^2. */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    int *row;    /* n + 1 */
    int *col;
    int64_t cap;
} gamma_set;

static int gamma_build(gamma_set *G, int n, const double *xy, double lcut)
{
    const double c2 = lcut * lcut;
    int64_t cnt = 0;
    for (int pass = 0; pass < 2; ++pass) {
        cnt = 0;
        for (int i = 0; i < n; ++i) {
            if (pass == 1) G->row[i] = (int)cnt;
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                const double dx = xy[2 * i] - xy[2 * j], dy = xy[2 * i + 1] - xy[2 * j + 1];
                const double a = dx * dx, b = dy * dy;
                if (a + b < c2) {
                    if (pass == 1) G->col[cnt] = j;
                    ++cnt;
                }
            }
        }
        if (pass == 0 && cnt > G->cap) {
            free(G->col);
            G->col = malloc(sizeof(int) * (size_t)(cnt > 0 ? cnt : 1));
            if (!G->col) return -1;
            G->cap = cnt;
        }
    }
    G->row[n] = (int)cnt;
    G->n = n;
    return 0;
}

static int gamma_equal(const gamma_set *a, const gamma_set *b)
{
    if (a->row[a->n] != b->row[b->n]) return 0;
    for (int i = 0; i <= a->n; ++i)
        if (a->row[i] != b->row[i]) return 0;
    for (int t = 0; t < a->row[a->n]; ++t)
        if (a->col[t] != b->col[t]) return 0;
    return 1;
}

/* E over Gamma: the pair terms of Eq. 5 only for pairs listed in Gamma,
 * summed as the brute-force energy sums them (i ascending, then j > i
 * ascending; containment after the pairs).  grad (nullable, 2n). */
static double gamma_energy_grad(const gamma_set *G, const double *xy, double R, double rad,
                                double *grad)
{
    const int n = G->n;
    double sp = 0.0, sc = 0.0;
    const double two_r = 2.0 * rad;
    if (grad) memset(grad, 0, sizeof(double) * 2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        const double xi = xy[2 * i], yi = xy[2 * i + 1];
        for (int t = G->row[i]; t < G->row[i + 1]; ++t) {
            const int j = G->col[t];
            if (j <= i) continue;
            const double dx = xi - xy[2 * j];
            const double dy = yi - xy[2 * j + 1];
            const double l2 = dx * dx + dy * dy;
            if (l2 < two_r * two_r) {
                const double l = sqrt(l2);
                const double d = two_r - l;
                sp += d * d;
                if (grad && l > 0.0) {
                    const double k = -2.0 * d / l;
                    grad[2 * i] += k * dx;
                    grad[2 * i + 1] += k * dy;
                    grad[2 * j] -= k * dx;
                    grad[2 * j + 1] -= k * dy;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) {
        const double x = xy[2 * i], y = xy[2 * i + 1];
        const double rho = sqrt(x * x + y * y);
        const double d0 = rho + rad - R;
        if (d0 > 0.0) {
            sc += d0 * d0;
            if (grad && rho > 0.0) {
                grad[2 * i] += 2.0 * d0 * x / rho;
                grad[2 * i + 1] += 2.0 * d0 * y / rho;
            }
        }
    }
    return sp + sc;
}

/* Batch energy of Eq. 7 over Gamma (the reformulation of Sec. 4.3): for i
 * in B_p, j in Gamma(i) ascending, the pair counts when j is outside B_p
 * or j < i; the gradient keeps dE/dc_i of the members. */
static double gamma_batch_energy_grad(const gamma_set *G, const double *xy, double R, double rad,
                                      const int32_t *mask, double *grad)
{
    const int n = G->n;
    double e = 0.0;
    const double two_r = 2.0 * rad;
    if (grad) memset(grad, 0, sizeof(double) * 2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        if (!mask[i]) continue;
        const double xi = xy[2 * i], yi = xy[2 * i + 1];
        for (int t = G->row[i]; t < G->row[i + 1]; ++t) {
            const int j = G->col[t];
            const double dx = xi - xy[2 * j];
            const double dy = yi - xy[2 * j + 1];
            const double l2 = dx * dx + dy * dy;
            if (!(l2 < two_r * two_r)) continue;
            const double l = sqrt(l2);
            const double d = two_r - l;
            if (!mask[j] || j < i) e += d * d;
            if (grad && l > 0.0) {
                const double k = -2.0 * d / l;
                grad[2 * i] += k * dx;
                grad[2 * i + 1] += k * dy;
            }
        }
        const double rho = sqrt(xi * xi + yi * yi);
        const double d0 = rho + rad - R;
        if (d0 > 0.0) {
            e += d0 * d0;
            if (grad && rho > 0.0) {
                grad[2 * i] += 2.0 * d0 * xi / rho;
                grad[2 * i + 1] += 2.0 * d0 * yi / rho;
            }
        }
    }
    return e;
}

/* Energy over Gamma of a layout (test hook): Gamma is built at `ref` with
 * l_cut, the energy is evaluated at xy. */
double oracle_gamma_energy(int n, const double *ref, const double *xy, double R, double lcut)
{
    gamma_set G = { 0, malloc(sizeof(int) * (size_t)(n + 1)), NULL, 0 };
    if (!G.row || gamma_build(&G, n, ref, lcut) != 0) {
        free(G.row); free(G.col);
        return NAN;
    }
    const double e = gamma_energy_grad(&G, xy, R, 1.0, NULL);
    free(G.row); free(G.col);
    return e;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 with the batches of a given partition visited in order p = 0..k-1  */
/* (each visit sees the positions the earlier visits left), the limited-     */
/* memory reading of Eq. 8-11 per batch, and either exact energies (every    */
/* pair) or energies over Gamma maintained by ANM (Alg. 3).                  */
/*                                                                          */
/* Outer iteration t:                                                       */
/*   stop tests on the current layout, in this order: non-finite E,         */
/*     E < e_feasible, (t > 0) the sum over batches of ||g(x_p)||_2 of the  */
/*     previous outer iteration <= g_tol, relative decrease of E over the   */
/*     last ftol_window outer iterations below ftol, (t > 0) every visit of */
/*     the previous outer iteration stalled, t >= max_outer;                */
/*   for every non-empty batch p: g(x_p) (Eq. 7) at the current positions,  */
/*     p = -H_p g (two-loop over the batch's own history, reset to -g when   */
/*     not a descent direction), alpha0 = 1 with history, 1/max(1,||g||)    */
/*     without, halve alpha until E(x_p + alpha p) <= E(x_p) + c1 alpha g'p  */
/*     (max_halvings; a visit that fails leaves the batch where it was),    */
/*     keep (s, y) when s'y > eps_curv y'y, y from two gradients under the  */
/*     same positions of the other batches;                                 */
/*   ANM (Alg. 3): cnt += 1; once cnt >= len the neighbor structure Gamma'  */
/*     of the current layout is built: Gamma' != Gamma gives cnt = 0,       */
/*     len = 1, Gamma = Gamma'; otherwise cnt = 0, len = 2 len.  Gamma is   */
/*     built at the start with cnt = 0, len = 1;                            */
/*   E of the new layout (over Gamma when ANM is on).                       */
/* dense = 1 replaces the limited-memory history by the paper's dense        */
/* inverse-Hessian approximation H_p of every batch (Eq. 8-11): H_p = I at    */
/* the start, p = -H_p g, and after an accepted step with s'y > eps_curv y'y */
/* (u = s, v = y, beta = v'u)                                               */
/*   H_p <- (I - u v'/beta) H_p (I - v u'/beta) + u u'/beta,                */
/* evaluated as H - (w u' + u w')/beta + (v'w/beta^2 + 1/beta) u u' with     */
/* w = H v (the same matrix, H symmetric).  A direction that is not a       */
/* descent direction resets H_p to I; alpha0 = 1 once H_p has been updated, */
/* 1/max(1,||g||) before.                                                   */
/* xy (2n) is updated in place; trace (nullable, max_outer + 1) gets E at   */
/* the top of every outer iteration, xtrace (nullable, (max_outer + 1) 2n)  */
/* the positions there.                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t max_outer;
    int32_t anm;          /* 0: exact energies over every pair; 1: over Gamma, ANM */
    double lcut;          /* l_cut of Gamma (4 in the paper)                 */
    int32_t dense;        /* 1: dense H_p per batch (Eq. 11) instead of L-BFGS */
    int32_t pad;
} oracle_seq_params;

typedef struct {
    int32_t status;
    int32_t outer;
    int32_t visits;
    int32_t evals;
    int32_t stalled_visits;
    int32_t anm_checks;   /* Gamma' built and compared                      */
    int32_t anm_changes;  /* ... and found different                        */
    int32_t pad;
    double E;
    double gsum;
} oracle_seq_result;

enum { SQ_RUNNING = 0, SQ_FEASIBLE = 1, SQ_STATIONARY = 2, SQ_CONVERGED = 3,
       SQ_STALLED = 4, SQ_MAX_ITER = 5, SQ_NONFINITE = 6 };

static double dotp(int d, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < d; ++i) s += a[i] * b[i];
    return s;
}

/* H <- H - (w u' + u w')/beta + (v'w/beta^2 + 1/beta) u u', w = H v: the
 * product form of Eq. 11 multiplied out for a symmetric H (d x d, row-major). */
void oracle_bfgs_update(int d, double *H, const double *u, const double *v)
{
    double *w = malloc(sizeof(double) * (size_t)(d > 0 ? d : 1));
    if (!w) return;
    double beta = 0.0, vw = 0.0;
    for (int r = 0; r < d; ++r) {
        double acc = 0.0;
        for (int c = 0; c < d; ++c) acc += H[(size_t)r * d + c] * v[c];
        w[r] = acc;
        beta += v[r] * u[r];
    }
    for (int r = 0; r < d; ++r) vw += v[r] * w[r];
    const double a = vw / (beta * beta) + 1.0 / beta;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            H[(size_t)r * d + c] += -(w[r] * u[c] + u[r] * w[c]) / beta + a * u[r] * u[c];
    free(w);
}

static void set_identity(int d, double *H)
{
    memset(H, 0, sizeof(double) * (size_t)d * d);
    for (int r = 0; r < d; ++r) H[(size_t)r * d + r] = 1.0;
}

int oracle_gbo_seq_descend(int n, double *xy, double R, const oracle_params *P,
                           const int32_t *batch_of, int k, const oracle_seq_params *Q,
                           oracle_seq_result *res, double *trace, double *xtrace)
{
    const int m = P->m;
    if (k < 1 || m < 1 || m > 64) return -2;
    for (int i = 0; i < n; ++i)
        if (batch_of[i] < 0 || batch_of[i] >= k) return -2;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *mask = calloc(nn, sizeof(int32_t));
    int *cnt = calloc((size_t)k, sizeof(int)), *start = calloc((size_t)k + 1, sizeof(int));
    int *member = malloc(sizeof(int) * nn), *kh = calloc((size_t)k, sizeof(int));
    double **Sh = calloc((size_t)k, sizeof(double *)), **Yh = calloc((size_t)k, sizeof(double *));
    double *g = malloc(sizeof(double) * 2 * nn), *gt = malloc(sizeof(double) * 2 * nn);
    double *bg = malloc(sizeof(double) * 2 * nn), *bp = malloc(sizeof(double) * 2 * nn);
    double *bs = malloc(sizeof(double) * 2 * nn), *by = malloc(sizeof(double) * 2 * nn);
    double *bx0 = malloc(sizeof(double) * 2 * nn);
    const int W = P->ftol_window > 0 ? P->ftol_window : 1;
    double *ehist = calloc((size_t)W + 1, sizeof(double));
    gamma_set G = { 0, malloc(sizeof(int) * (nn + 1)), NULL, 0 };
    gamma_set G2 = { 0, malloc(sizeof(int) * (nn + 1)), NULL, 0 };
    int rc = 0;
    if (!mask || !cnt || !start || !member || !kh || !Sh || !Yh || !g || !gt || !bg || !bp ||
        !bs || !by || !bx0 || !ehist || !G.row || !G2.row) {
        rc = -1;
        goto done;
    }
    for (int i = 0; i < n; ++i) ++cnt[batch_of[i]];
    for (int p = 0; p < k; ++p) start[p + 1] = start[p] + cnt[p];
    {
        int *fill = calloc((size_t)k, sizeof(int));
        if (!fill) { rc = -1; goto done; }
        for (int i = 0; i < n; ++i) member[start[batch_of[i]] + fill[batch_of[i]]++] = i;
        free(fill);
    }
    for (int p = 0; p < k; ++p) {
        const size_t dim = 2 * (size_t)(cnt[p] > 0 ? cnt[p] : 1);
        if (Q->dense) {
            /* Sh[p] holds H_p (dim x dim); Yh[p] is unused */
            Sh[p] = malloc(sizeof(double) * dim * dim);
            Yh[p] = malloc(sizeof(double));
            if (Sh[p]) set_identity((int)dim, Sh[p]);
        } else {
            Sh[p] = calloc((size_t)m * dim, sizeof(double));
            Yh[p] = calloc((size_t)m * dim, sizeof(double));
        }
        if (!Sh[p] || !Yh[p]) { rc = -1; goto done; }
    }
    int anm_cnt = 0, anm_len = 1, checks = 0, changes = 0;
    if (Q->anm && gamma_build(&G, n, xy, Q->lcut) != 0) { rc = -1; goto done; }
#define TOTAL_E(X) (Q->anm ? gamma_energy_grad(&G, (X), R, P->rad, NULL) \
                           : oracle_energy_grad(n, (X), R, P->rad, NULL, NULL, NULL))
#define BATCH_EG(X, GR) (Q->anm ? gamma_batch_energy_grad(&G, (X), R, P->rad, mask, (GR)) \
                                : oracle_batch_energy_grad(n, (X), R, P->rad, mask, (GR)))
    int visits = 0, evals = 0, stalled = 0, t = 0, status = SQ_RUNNING;
    int stalled_prev = 0, visited_prev = 0;
    double E = TOTAL_E(xy);
    double gsum_prev = -1.0;
    for (t = 0;; ++t) {
        if (trace) trace[t] = E;
        if (xtrace) memcpy(xtrace + (size_t)t * 2 * n, xy, sizeof(double) * 2 * (size_t)n);
        if (!isfinite(E)) { status = SQ_NONFINITE; break; }
        if (E < P->e_feasible) { status = SQ_FEASIBLE; break; }
        if (t > 0 && gsum_prev <= P->g_tol) { status = SQ_STATIONARY; break; }
        if (P->ftol > 0.0 && t >= W) {
            const double e_old = ehist[(t - W) % (W + 1)];
            if (e_old - E <= P->ftol * e_old) { status = SQ_CONVERGED; break; }
        }
        ehist[t % (W + 1)] = E;
        if (t > 0 && visited_prev > 0 && stalled_prev == visited_prev) { status = SQ_STALLED; break; }
        if (t >= Q->max_outer) { status = SQ_MAX_ITER; break; }
        double gsum = 0.0;
        stalled_prev = 0;
        visited_prev = 0;
        for (int p = 0; p < k; ++p) {
            const int np = cnt[p];
            if (np == 0) continue;
            const int *mem = member + start[p];
            const int dim = 2 * np;
            ++visits;
            ++visited_prev;
            for (int q = 0; q < np; ++q) mask[mem[q]] = 1;
            const double Ep = BATCH_EG(xy, g);
            ++evals;
            for (int q = 0; q < np; ++q) {
                bg[2 * q] = g[2 * mem[q]];
                bg[2 * q + 1] = g[2 * mem[q] + 1];
                bx0[2 * q] = xy[2 * mem[q]];
                bx0[2 * q + 1] = xy[2 * mem[q] + 1];
            }
            const double gn = sqrt(dotp(dim, bg, bg));
            gsum += gn;
            if (Q->dense) {
                const double *H = Sh[p];
                for (int r = 0; r < dim; ++r) {
                    double acc = 0.0;
                    for (int c = 0; c < dim; ++c) acc += H[(size_t)r * dim + c] * bg[c];
                    bp[r] = -acc;
                }
            } else {
                oracle_two_loop(dim, kh[p], Sh[p], Yh[p], bg, bp);
                for (int d = 0; d < dim; ++d) bp[d] = -bp[d];
            }
            double gp = dotp(dim, bg, bp);
            if (kh[p] > 0 && !(gp < 0.0)) {
                kh[p] = 0;
                if (Q->dense) set_identity(dim, Sh[p]);
                for (int d = 0; d < dim; ++d) bp[d] = -bg[d];
                gp = dotp(dim, bg, bp);
            }
            double alpha = kh[p] > 0 ? 1.0 : 1.0 / (gn > 1.0 ? gn : 1.0);
            int accepted = 0;
            for (int h = 0; h <= P->max_halvings; ++h) {
                for (int q = 0; q < np; ++q) {
                    xy[2 * mem[q]] = bx0[2 * q] + alpha * bp[2 * q];
                    xy[2 * mem[q] + 1] = bx0[2 * q + 1] + alpha * bp[2 * q + 1];
                }
                const double Et = BATCH_EG(xy, gt);
                ++evals;
                if (Et <= Ep + P->c1 * alpha * gp) { accepted = 1; break; }
                alpha *= 0.5;
            }
            if (accepted) {
                double sy = 0.0, yy = 0.0;
                for (int q = 0; q < np; ++q) {
                    for (int c = 0; c < 2; ++c) {
                        const int d = 2 * q + c;
                        bs[d] = xy[2 * mem[q] + c] - bx0[d];
                        by[d] = gt[2 * mem[q] + c] - bg[d];
                        sy += bs[d] * by[d];
                        yy += by[d] * by[d];
                    }
                }
                if (sy > P->eps_curv * yy) {
                    if (Q->dense) {
                        oracle_bfgs_update(dim, Sh[p], bs, by);
                        if (kh[p] < m) ++kh[p];
                    } else {
                        if (kh[p] == m) {
                            memmove(Sh[p], Sh[p] + dim, sizeof(double) * (size_t)(m - 1) * dim);
                            memmove(Yh[p], Yh[p] + dim, sizeof(double) * (size_t)(m - 1) * dim);
                            kh[p] = m - 1;
                        }
                        memcpy(Sh[p] + (size_t)kh[p] * dim, bs, sizeof(double) * dim);
                        memcpy(Yh[p] + (size_t)kh[p] * dim, by, sizeof(double) * dim);
                        ++kh[p];
                    }
                }
            } else {
                for (int q = 0; q < np; ++q) {
                    xy[2 * mem[q]] = bx0[2 * q];
                    xy[2 * mem[q] + 1] = bx0[2 * q + 1];
                }
                ++stalled;
                ++stalled_prev;
            }
            for (int q = 0; q < np; ++q) mask[mem[q]] = 0;
        }
        gsum_prev = gsum;
        if (Q->anm) {
            if (++anm_cnt >= anm_len) {
                if (gamma_build(&G2, n, xy, Q->lcut) != 0) { rc = -1; goto done; }
                ++checks;
                if (!gamma_equal(&G, &G2)) {
                    gamma_set tmp = G; G = G2; G2 = tmp;
                    anm_cnt = 0;
                    anm_len = 1;
                    ++changes;
                } else {
                    anm_cnt = 0;
                    anm_len *= 2;
                }
            }
        }
        E = TOTAL_E(xy);
    }
#undef TOTAL_E
#undef BATCH_EG
    res->status = status;
    res->outer = t;
    res->visits = visits;
    res->evals = evals;
    res->stalled_visits = stalled;
    res->anm_checks = checks;
    res->anm_changes = changes;
    res->pad = 0;
    res->E = E;
    res->gsum = gsum_prev;
done:
    if (Sh) for (int p = 0; p < k; ++p) free(Sh[p]);
    if (Yh) for (int p = 0; p < k; ++p) free(Yh[p]);
    free(Sh); free(Yh); free(mask); free(cnt); free(start); free(member); free(kh);
    free(g); free(gt); free(bg); free(bp); free(bs); free(by); free(bx0); free(ehist);
    free(G.row); free(G.col); free(G2.row); free(G2.col);
    return rc;
}
