/*
 * pecc_oracle.c -- plain FP64 CPU oracle for the penalty-energy descent of
 * Zhou, He, Zheng & Li, "Geometric Batch Optimization for the Packing Equal
 * Circles in a Circle Problem on Large Scale" (arXiv 2303.02650).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent checker of the HIP
 * library.  Only the test suite, the smoke entry point and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU path and includes nothing from it.
 *
 * Everything is brute force and FP64: every pair i<j is enumerated, no cell
 * grid, no neighbor list, no blocking.  Build with -O2 -ffp-contract=off so
 * that no multiply-add is fused (the neighbor predicate must round exactly
 * like the GPU's, see oracle_neighbors).
 *
 * Sections of the paper followed:
 *   Sec. 3.1, Eq. 1-2   problem (feasibility)
 *   Def. 3.1 (Eq. 3)    overlap distances d_ij, d_i0
 *   Def. 3.2 (Eq. 5)    elastic energy E = sum_{i<j} d_ij^2 + sum_i d_i0^2
 *   Sec. 4.1, Eq. 7     batch energy E(x_p)
 *   Sec. 4.1, Eq. 8-11  quasi-Newton step, BFGS inverse update
 *   Sec. 4.1, Alg. 1    batch descent loop and its stop rule
 *   Sec. 4.3            neighbor set Gamma(i) = { j != i : l_ij < l_cut }
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "pecc_oracle_types.h"

/* ------------------------------------------------------------------------ */
/* Energy and gradient: Def. 3.1 and Def. 3.2, written out pair by pair.     */
/*                                                                           */
/* rad is the circle radius (1 for the paper's unit circles; a value         */
/* 1+mu describes circles inflated by a contact margin mu).  Overlap of i,j  */
/* is d = max(0, 2 rad - l), container overlap d0 = max(0, rho + rad - R).   */
/* d(d^2)/dc_i = 2 d * (-(c_i - c_j)/l); at l = 0 the pair adds (2rad)^2 to  */
/* E and nothing to g (0 lies in the generalized gradient there).            */
/* Returns E; e_pair / e_cont (nullable) get the two sums; grad (nullable,   */
/* length 2n, interleaved like x) receives dE/dx.                            */
/* ------------------------------------------------------------------------ */
static int all_finite_d(int n, const double *xy)
{
    for (int i = 0; i < 2 * n; ++i)
        if (!isfinite(xy[i])) return 0;
    return 1;
}

static int all_finite_f(int n, const float *xy)
{
    for (int i = 0; i < 2 * n; ++i)
        if (!isfinite(xy[i])) return 0;
    return 1;
}

/* E is a sum over every circle (Eq. 5), so a circle without a finite
 * position leaves it undefined: E, its parts and g are then NaN. */
double oracle_energy_grad(int n, const double *xy, double R, double rad,
                          double *e_pair, double *e_cont, double *grad)
{
    double sp = 0.0, sc = 0.0;
    const double two_r = 2.0 * rad;
    if (!all_finite_d(n, xy)) {
        if (grad) for (int i = 0; i < 2 * n; ++i) grad[i] = NAN;
        if (e_pair) *e_pair = NAN;
        if (e_cont) *e_cont = NAN;
        return NAN;
    }
    if (grad) memset(grad, 0, sizeof(double) * 2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        const double xi = xy[2 * i], yi = xy[2 * i + 1];
        for (int j = i + 1; j < n; ++j) {
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
    if (e_pair) *e_pair = sp;
    if (e_cont) *e_cont = sc;
    return sp + sc;
}

/* Batch energy of Eq. 7: circles i with mask[i] != 0 form B_p.
 *   E(x_p) = sum_{i in B_p} sum_{j != i} d_ij^2 [j not in B_p or j < i]
 *          + sum_{i in B_p} d_i0^2
 * grad (nullable, 2n) receives dE(x_p)/dx restricted to B_p (zero outside). */
double oracle_batch_energy_grad(int n, const double *xy, double R, double rad,
                                const int32_t *mask, double *grad)
{
    double e = 0.0;
    const double two_r = 2.0 * rad;
    if (grad) memset(grad, 0, sizeof(double) * 2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        if (!mask[i]) continue;
        const double xi = xy[2 * i], yi = xy[2 * i + 1];
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = xi - xy[2 * j];
            const double dy = yi - xy[2 * j + 1];
            const double l2 = dx * dx + dy * dy;
            if (!(l2 < two_r * two_r)) continue;
            const double l = sqrt(l2);
            const double d = two_r - l;
            if (!mask[j] || j < i) e += d * d;
            if (grad && l > 0.0) {
                /* only the derivative with respect to c_i is kept: pairs
                 * inside B_p are visited from both ends, pairs leaving B_p
                 * once, and both give exactly dE/dc_i. */
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

/* ------------------------------------------------------------------------ */
/* Neighbor set Gamma(i) of Sec. 4.3 with l_cut = cutoff, as the half set of */
/* pairs i < j.  The predicate is evaluated in FP64 on FP32 coordinates:     */
/*   dx = (double)x_i - (double)x_j;  dy likewise;                           */
/*   pair  <=>  dx*dx + dy*dy < cutoff*cutoff   (strict, no fused mult-add)  */
/* Pairs come out ordered by i, then j.  Returns the number of pairs; only   */
/* the first cap are stored.                                                 */
/* ------------------------------------------------------------------------ */
int64_t oracle_neighbors(int n, const float *xy, double cutoff,
                         int32_t *pi, int32_t *pj, int64_t cap)
{
    const double c2 = cutoff * cutoff;
    int64_t cnt = 0;
    for (int i = 0; i < n; ++i) {
        const double xi = (double)xy[2 * i], yi = (double)xy[2 * i + 1];
        for (int j = i + 1; j < n; ++j) {
            const double dx = xi - (double)xy[2 * j];
            const double dy = yi - (double)xy[2 * j + 1];
            const double a = dx * dx;
            const double b = dy * dy;
            if (a + b < c2) {
                if (cnt < cap) { pi[cnt] = i; pj[cnt] = j; }
                ++cnt;
            }
        }
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Limited-memory inverse-Hessian product r = H g.  H is what the BFGS       */
/* inverse update of Eq. 10-11 gives when applied to the k stored pairs      */
/* (u = s, v = y), oldest first, starting from H0 = gamma I with gamma =     */
/* s^T y / y^T y of the newest pair.  Computed by the standard two-loop      */
/* recursion (Nocedal & Wright, Numerical Optimization, Alg. 7.4), which     */
/* equals the dense product without forming H.  S and Y hold k rows of       */
/* length dim, oldest first.  k = 0 gives r = g.                             */
/* ------------------------------------------------------------------------ */
void oracle_two_loop(int dim, int k, const double *S, const double *Y,
                     const double *g, double *r)
{
    double alpha[64];
    double rho[64];
    for (int d = 0; d < dim; ++d) r[d] = g[d];
    if (k <= 0) return;
    for (int i = 0; i < k; ++i) {
        double sy = 0.0;
        for (int d = 0; d < dim; ++d) sy += S[(size_t)i * dim + d] * Y[(size_t)i * dim + d];
        rho[i] = 1.0 / sy;
    }
    for (int i = k - 1; i >= 0; --i) {
        double a = 0.0;
        for (int d = 0; d < dim; ++d) a += S[(size_t)i * dim + d] * r[d];
        a *= rho[i];
        alpha[i] = a;
        for (int d = 0; d < dim; ++d) r[d] -= a * Y[(size_t)i * dim + d];
    }
    {
        double sy = 0.0, yy = 0.0;
        const double *s = S + (size_t)(k - 1) * dim, *y = Y + (size_t)(k - 1) * dim;
        for (int d = 0; d < dim; ++d) { sy += s[d] * y[d]; yy += y[d] * y[d]; }
        const double gamma = sy / yy;
        for (int d = 0; d < dim; ++d) r[d] *= gamma;
    }
    for (int i = 0; i < k; ++i) {
        double b = 0.0;
        for (int d = 0; d < dim; ++d) b += Y[(size_t)i * dim + d] * r[d];
        b *= rho[i];
        for (int d = 0; d < dim; ++d) r[d] += S[(size_t)i * dim + d] * (alpha[i] - b);
    }
}

/* ------------------------------------------------------------------------ */
/* Descent parameters and outcome (the oracle's own definitions).            */
/* ------------------------------------------------------------------------ */
enum { OR_RUNNING = 0, OR_FEASIBLE = 1, OR_STATIONARY = 2, OR_CONVERGED = 3,
       OR_STALLED = 4, OR_MAX_ITER = 5, OR_NONFINITE = 6 };

typedef double (*energy_fn)(void *ctx, const double *x, double *g);

typedef struct { int n; double R; double rad; } whole_ctx;

static double whole_energy(void *c, const double *x, double *g)
{
    const whole_ctx *w = (const whole_ctx *)c;
    return oracle_energy_grad(w->n, x, w->R, w->rad, NULL, NULL, g);
}

static double dot(int d, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < d; ++i) s += a[i] * b[i];
    return s;
}

/* State of one L-BFGS minimisation in FP64. */
typedef struct {
    int dim, m, k;
    double *S, *Y;   /* m rows each, oldest first */
    double *x, *g, *p, *xt, *gt, *ehist;
    double E;
} lbfgs_state;

static int lbfgs_alloc(lbfgs_state *st, int dim, int m, int hist_len)
{
    memset(st, 0, sizeof(*st));
    st->dim = dim; st->m = m; st->k = 0;
    st->S = calloc((size_t)m * dim, sizeof(double));
    st->Y = calloc((size_t)m * dim, sizeof(double));
    st->g = calloc(dim, sizeof(double));
    st->p = calloc(dim, sizeof(double));
    st->xt = calloc(dim, sizeof(double));
    st->gt = calloc(dim, sizeof(double));
    st->ehist = calloc(hist_len > 0 ? hist_len : 1, sizeof(double));
    return st->S && st->Y && st->g && st->p && st->xt && st->gt && st->ehist;
}

static void lbfgs_free(lbfgs_state *st)
{
    free(st->S); free(st->Y); free(st->g); free(st->p); free(st->xt);
    free(st->gt); free(st->ehist);
}

/* ------------------------------------------------------------------------ */
/* Whole-instance L-BFGS descent (Alg. 1 with k = 1 and the limited-memory  */
/* reading of Eq. 8-11).  One iteration:                                     */
/*   stop tests on the current point, in this order: non-finite E,          */
/*     E < e_feasible, ||g||_2 <= g_tol, relative decrease over the last     */
/*     ftol_window iterations below ftol, iteration budget spent;            */
/*   p = -H g (two-loop), reset to -g when it is not a descent direction;    */
/*   alpha0 = 1 with history, 1/max(1,||g||) without;                        */
/*   halve alpha until E(x+alpha p) <= E + c1 alpha g^T p (max_halvings);    */
/*   x <- x + alpha p; keep (s,y) when s^T y > eps_curv y^T y, at most m.    */
/* xy (2n) is updated in place.  trace (nullable, max_iter+1) gets E at the  */
/* start of every iteration.                                                 */
/* ------------------------------------------------------------------------ */
static int run_descent(int dim, double *x, const oracle_params *P, energy_fn f,
                       void *ctx, oracle_result *res, double *trace)
{
    lbfgs_state st;
    const int W = P->ftol_window > 0 ? P->ftol_window : 1;
    if (!lbfgs_alloc(&st, dim, P->m, W + 1)) { lbfgs_free(&st); return -1; }
    double *cand_s = calloc(dim, sizeof(double));
    double *cand_y = calloc(dim, sizeof(double));
    if (!cand_s || !cand_y) { free(cand_s); free(cand_y); lbfgs_free(&st); return -1; }
    st.x = x;
    int evals = 0, resets = 0, it = 0, status = OR_RUNNING;
    st.E = f(ctx, x, st.g);
    ++evals;
    for (it = 0;; ++it) {
        const double gn = sqrt(dot(dim, st.g, st.g));
        if (trace) trace[it] = st.E;
        if (!isfinite(st.E) || !isfinite(gn)) { status = OR_NONFINITE; break; }
        if (st.E < P->e_feasible) { status = OR_FEASIBLE; break; }
        if (gn <= P->g_tol) { status = OR_STATIONARY; break; }
        if (P->ftol > 0.0 && it >= W) {
            const double e_old = st.ehist[(it - W) % (W + 1)];
            if (e_old - st.E <= P->ftol * e_old) { status = OR_CONVERGED; break; }
        }
        st.ehist[it % (W + 1)] = st.E;
        if (it >= P->max_iter) { status = OR_MAX_ITER; break; }

        /* direction */
        double *p = st.p, *g = st.g, *xt = st.xt, *gt = st.gt;
        oracle_two_loop(dim, st.k, st.S, st.Y, g, p);
        for (int d = 0; d < dim; ++d) p[d] = -p[d];
        double gp = dot(dim, g, p);
        if (st.k > 0 && !(gp < 0.0)) {
            st.k = 0;
            ++resets;
            for (int d = 0; d < dim; ++d) p[d] = -g[d];
            gp = dot(dim, g, p);
        }
        /* backtracking line search (reading of Eq. 9) */
        double alpha = st.k > 0 ? 1.0 : 1.0 / (gn > 1.0 ? gn : 1.0);
        int accepted = 0;
        double Et = 0.0;
        for (int h = 0; h <= P->max_halvings; ++h) {
            for (int d = 0; d < dim; ++d) xt[d] = x[d] + alpha * p[d];
            Et = f(ctx, xt, gt);
            ++evals;
            if (Et <= st.E + P->c1 * alpha * gp) { accepted = 1; break; }
            alpha *= 0.5;
        }
        if (!accepted) { status = OR_STALLED; break; }
        /* curvature pair (Eq. 10: u = s, v = y) */
        double sy = 0.0, yy = 0.0;
        for (int d = 0; d < dim; ++d) {
            cand_s[d] = xt[d] - x[d];
            cand_y[d] = gt[d] - g[d];
            sy += cand_s[d] * cand_y[d];
            yy += cand_y[d] * cand_y[d];
        }
        if (sy > P->eps_curv * yy) {
            if (st.k == st.m) {
                memmove(st.S, st.S + dim, sizeof(double) * (size_t)(st.m - 1) * dim);
                memmove(st.Y, st.Y + dim, sizeof(double) * (size_t)(st.m - 1) * dim);
                st.k = st.m - 1;
            }
            memcpy(st.S + (size_t)st.k * dim, cand_s, sizeof(double) * dim);
            memcpy(st.Y + (size_t)st.k * dim, cand_y, sizeof(double) * dim);
            ++st.k;
        }
        memcpy(x, xt, sizeof(double) * dim);
        memcpy(g, gt, sizeof(double) * dim);
        st.E = Et;
    }
    res->status = status;
    res->iters = it;
    res->evals = evals;
    res->resets = resets;
    res->E = st.E;
    res->gnorm = sqrt(dot(dim, st.g, st.g));
    free(cand_s); free(cand_y);
    lbfgs_free(&st);
    return 0;
}

int oracle_descend(int n, double *xy, double R, const oracle_params *P,
                   oracle_result *res, double *trace)
{
    whole_ctx c = { n, R, P->rad };
    if (P->m < 1 || P->m > 64) return -2;
    return run_descent(2 * n, xy, P, whole_energy, &c, res, trace);
}

/* ------------------------------------------------------------------------ */
/* Container adjustment (Sec. 4.2, Eq. 12, Alg. 2).  The radius joins the    */
/* variables, z = [x_1, y_1, ..., x_n, y_n, R], and the energy gets a        */
/* penalty that pulls the container in:                                      */
/*   U(z, lambda) = sum_{i<j} d_ij^2 + sum_i d_i0^2 + lambda R^2,            */
/*   d_i0 = max(0, rho_i + rad - R),  dU/dR = -2 sum_i d_i0 + 2 lambda R.    */
/* Alg. 2: lambda starts at lambda0 (1e-4) and is halved after each of        */
/* `rounds` (35) minimisations of U; each minimisation is a fresh L-BFGS     */
/* descent with the readings of run_descent (no FEASIBLE stop: U > 0).       */
/* ------------------------------------------------------------------------ */
typedef struct { int n; double rad; double lambda; } adj_ctx;

static double adj_energy(void *c, const double *z, double *g)
{
    const adj_ctx *a = (const adj_ctx *)c;
    const int n = a->n;
    const double R = z[2 * n];
    double U = oracle_energy_grad(n, z, R, a->rad, NULL, NULL, g);
    double sum_d0 = 0.0;
    for (int i = 0; i < n; ++i) {
        const double rho = sqrt(z[2 * i] * z[2 * i] + z[2 * i + 1] * z[2 * i + 1]);
        const double d0 = rho + a->rad - R;
        if (d0 > 0.0) sum_d0 += d0;
    }
    U += a->lambda * R * R;
    if (g) g[2 * n] = -2.0 * sum_d0 + 2.0 * a->lambda * R;
    return U;
}

/* U and its gradient (2n + 1 entries) at z, for tests. */
double oracle_container_energy(int n, const double *z, double rad, double lambda, double *g)
{
    adj_ctx c = { n, rad, lambda };
    return adj_energy(&c, z, g);
}

typedef struct {
    int32_t rounds;       /* minimisations run                                */
    int32_t iters;        /* accepted iterations over all rounds              */
    int32_t evals;        /* energy evaluations over all rounds               */
    int32_t last_status;  /* status of the last round's descent               */
    double R;             /* final radius                                     */
    double E;             /* E of the final layout at the final radius        */
} oracle_adjust_result;

int oracle_adjust_container(int n, double *xy, double *R, const oracle_params *P,
                            double lambda0, int rounds, oracle_adjust_result *res)
{
    if (P->m < 1 || P->m > 64 || rounds < 0) return -2;
    double *z = malloc(sizeof(double) * (size_t)(2 * n + 1));
    if (!z) return -1;
    memcpy(z, xy, sizeof(double) * 2 * (size_t)n);
    z[2 * n] = *R;
    oracle_params Q = *P;
    Q.e_feasible = 0.0;                      /* U is positive: no feasible stop */
    double lambda = lambda0;
    memset(res, 0, sizeof(*res));
    for (int t = 0; t < rounds; ++t) {
        adj_ctx c = { n, P->rad, lambda };
        oracle_result r;
        int rc = run_descent(2 * n + 1, z, &Q, adj_energy, &c, &r, NULL);
        if (rc != 0) { free(z); return rc; }
        res->iters += r.iters;
        res->evals += r.evals;
        res->last_status = r.status;
        res->rounds = t + 1;
        if (r.status == OR_NONFINITE) break;
        lambda *= 0.5;
    }
    memcpy(xy, z, sizeof(double) * 2 * (size_t)n);
    *R = z[2 * n];
    res->R = *R;
    res->E = oracle_energy_grad(n, xy, *R, P->rad, NULL, NULL, NULL);
    free(z);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* FP64 feasibility check (Eq. 1-2 through Eq. 5 with unit circles).         */
/* out[0] = E, out[1] = max_{i<j} d_ij, out[2] = max_i d_i0 (both >= 0),     */
/* returns 1 if E < tol.  Positions are FP32, promoted exactly.  A non-      */
/* finite coordinate makes all three NaN and the layout infeasible.          */
/* ------------------------------------------------------------------------ */
int oracle_verify(int n, const float *xy, double R, double tol, double *out)
{
    double sp = 0.0, sc = 0.0, mp = 0.0, mc = 0.0;
    if (!all_finite_f(n, xy)) {
        out[0] = out[1] = out[2] = NAN;
        return 0;
    }
    for (int i = 0; i < n; ++i) {
        const double xi = (double)xy[2 * i], yi = (double)xy[2 * i + 1];
        for (int j = i + 1; j < n; ++j) {
            const double dx = xi - (double)xy[2 * j];
            const double dy = yi - (double)xy[2 * j + 1];
            const double l2 = dx * dx + dy * dy;
            if (l2 < 4.0) {
                const double d = 2.0 - sqrt(l2);
                sp += d * d;
                if (d > mp) mp = d;
            }
        }
        const double rho = sqrt(xi * xi + yi * yi);
        const double d0 = rho + 1.0 - R;
        if (d0 > 0.0) {
            sc += d0 * d0;
            if (d0 > mc) mc = d0;
        }
    }
    out[0] = sp + sc;
    out[1] = mp;
    out[2] = mc;
    return (sp + sc) < tol ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Geometric batch descent (Alg. 1) with the limited-memory reading of      */
/* Eq. 8-11, the batch energy of Eq. 7 and a 2D grid-block partition.       */
/*                                                                           */
/* Partition (the first step of Alg. 1), fixed for the whole descent: block  */
/* S = 2R / blocks over [-R, R]^2; circle i goes to block (bx, by) with      */
/* bx = clamp(floor((x_i + R) / S), 0, blocks-1) (likewise by), batch id     */
/* p = by * blocks + bx, colour (bx mod 2) + 2 (by mod 2).  Batches are       */
/* visited colour by colour (0..3), in increasing p inside a colour.  With   */
/* jacobi = 1 every batch of a colour sees the others' positions as they     */
/* were when the colour started (the GPU runs them concurrently); with       */
/* jacobi = 0 it sees the latest ones (sequential order).                    */
/*                                                                           */
/* A visit is one quasi-Newton iteration on E(x_p) (Eq. 7) with the other   */
/* circles fixed: gradient, direction from the batch's own (s, y) history,  */
/* backtracking sufficient decrease, curvature pair under the same fixed     */
/* environment.  The pairs are all pairs (brute force), so no step length   */
/* is limited by anything but the line search.  A visit whose line search   */
/* fails leaves the batch unchanged.                                         */
/*                                                                           */
/* Outer iteration of Alg. 1: stop tests at its top: non-finite              */
/* E, E < e_feasible, sum over batches of ||g(x_p)||_2 of the previous outer */
/* iteration <= g_tol, relative decrease of E over ftol_window outer        */
/* iterations <= ftol, max_outer reached.                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t blocks;
    int32_t max_outer;
    int32_t jacobi;
    int32_t pad;
} oracle_gbo_params;

typedef struct {
    int32_t status;
    int32_t outer;
    int32_t visits;
    int32_t evals;
    int32_t stalled_visits;
    int32_t pad;
    double E;
    double gsum;
} oracle_gbo_result;

int oracle_gbo_batches(int n, const double *xy, double R, int blocks, int32_t *batch_of,
                       int32_t *colour_of)
{
    const double S = 2.0 * R / blocks;
    for (int i = 0; i < n; ++i) {
        double tx = floor((xy[2 * i] + R) / S), ty = floor((xy[2 * i + 1] + R) / S);
        int bx = tx < 0 ? 0 : (tx > blocks - 1 ? blocks - 1 : (int)tx);
        int by = ty < 0 ? 0 : (ty > blocks - 1 ? blocks - 1 : (int)ty);
        if (tx != tx) bx = 0;
        if (ty != ty) by = 0;
        batch_of[i] = by * blocks + bx;
        colour_of[i] = (bx & 1) + 2 * (by & 1);
    }
    return blocks * blocks;
}

int oracle_gbo_descend(int n, double *xy, double R, const oracle_params *P,
                       const oracle_gbo_params *G, oracle_gbo_result *res, double *trace)
{
    const int nb = G->blocks * G->blocks, m = P->m;
    if (G->blocks < 1 || m < 1 || m > 64) return -2;
    int32_t *batch_of = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t *colour_of = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t *mask = calloc(n > 0 ? n : 1, sizeof(int32_t));
    int *cnt = calloc(nb, sizeof(int)), *start = calloc(nb + 1, sizeof(int));
    int *member = malloc(sizeof(int) * (n > 0 ? n : 1));
    int *kh = calloc(nb, sizeof(int));
    double **Sh = calloc(nb, sizeof(double *)), **Yh = calloc(nb, sizeof(double *));
    double *snap = malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    double *env = malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    double *nx = malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    double *g = malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    double *gt = malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    double *bg = malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    double *bp = malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    double *bs = malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    double *by = malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    double *bx0 = malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    const int W = P->ftol_window > 0 ? P->ftol_window : 1;
    double *ehist = calloc(W + 1, sizeof(double));
    int rc = 0;
    if (!batch_of || !colour_of || !mask || !cnt || !start || !member || !kh || !Sh || !Yh ||
        !snap || !env || !nx || !g || !gt || !bg || !bp || !bs || !by || !bx0 || !ehist) {
        rc = -1;
        goto done;
    }
    oracle_gbo_batches(n, xy, R, G->blocks, batch_of, colour_of);
    for (int i = 0; i < n; ++i) ++cnt[batch_of[i]];
    for (int p = 0; p < nb; ++p) start[p + 1] = start[p] + cnt[p];
    {
        int *fill = calloc(nb, sizeof(int));
        if (!fill) { rc = -1; goto done; }
        for (int i = 0; i < n; ++i) member[start[batch_of[i]] + fill[batch_of[i]]++] = i;
        free(fill);
    }
    for (int p = 0; p < nb; ++p) {
        const int dim = 2 * cnt[p];
        Sh[p] = calloc((size_t)m * (dim > 0 ? dim : 1), sizeof(double));
        Yh[p] = calloc((size_t)m * (dim > 0 ? dim : 1), sizeof(double));
        if (!Sh[p] || !Yh[p]) { rc = -1; goto done; }
    }
    int visits = 0, evals = 0, stalled = 0, t = 0, status = OR_RUNNING;
    double E = oracle_energy_grad(n, xy, R, P->rad, NULL, NULL, NULL);
    double gsum_prev = -1.0, gsum = 0.0;
    for (t = 0;; ++t) {
        if (trace) trace[t] = E;
        if (!isfinite(E)) { status = OR_NONFINITE; break; }
        if (E < P->e_feasible) { status = OR_FEASIBLE; break; }
        if (t > 0 && gsum_prev <= P->g_tol) { status = OR_STATIONARY; break; }
        if (P->ftol > 0.0 && t >= W) {
            const double e_old = ehist[(t - W) % (W + 1)];
            if (e_old - E <= P->ftol * e_old) { status = OR_CONVERGED; break; }
        }
        ehist[t % (W + 1)] = E;
        if (t >= G->max_outer) { status = OR_MAX_ITER; break; }
        gsum = 0.0;
        for (int c = 0; c < 4; ++c) {
            memcpy(snap, xy, sizeof(double) * 2 * n);
            memcpy(nx, xy, sizeof(double) * 2 * n);
            for (int p = 0; p < nb; ++p) {
                const int np = cnt[p];
                if (np == 0) continue;
                const int *mem = member + start[p];
                if (colour_of[mem[0]] != c) continue;
                const int dim = 2 * np;
                ++visits;
                /* environment: other circles at the colour's start (jacobi) or now */
                memcpy(env, G->jacobi ? snap : nx, sizeof(double) * 2 * n);
                for (int q = 0; q < np; ++q) {
                    env[2 * mem[q]] = xy[2 * mem[q]];
                    env[2 * mem[q] + 1] = xy[2 * mem[q] + 1];
                    mask[mem[q]] = 1;
                }
                const double Ep = oracle_batch_energy_grad(n, env, R, P->rad, mask, g);
                ++evals;
                double gn2 = 0.0;
                for (int q = 0; q < np; ++q) {
                    bg[2 * q] = g[2 * mem[q]];
                    bg[2 * q + 1] = g[2 * mem[q] + 1];
                    bx0[2 * q] = env[2 * mem[q]];
                    bx0[2 * q + 1] = env[2 * mem[q] + 1];
                }
                for (int d = 0; d < dim; ++d) gn2 += bg[d] * bg[d];
                const double gn = sqrt(gn2);
                gsum += gn;
                oracle_two_loop(dim, kh[p], Sh[p], Yh[p], bg, bp);
                for (int d = 0; d < dim; ++d) bp[d] = -bp[d];
                double gp = dot(dim, bg, bp);
                if (kh[p] > 0 && !(gp < 0.0)) {
                    kh[p] = 0;
                    for (int d = 0; d < dim; ++d) bp[d] = -bg[d];
                    gp = dot(dim, bg, bp);
                }
                double alpha = kh[p] > 0 ? 1.0 : 1.0 / (gn > 1.0 ? gn : 1.0);
                int accepted = 0;
                double Et = 0.0;
                for (int h = 0; h <= P->max_halvings; ++h) {
                    for (int q = 0; q < np; ++q) {
                        env[2 * mem[q]] = bx0[2 * q] + alpha * bp[2 * q];
                        env[2 * mem[q] + 1] = bx0[2 * q + 1] + alpha * bp[2 * q + 1];
                    }
                    Et = oracle_batch_energy_grad(n, env, R, P->rad, mask, gt);
                    ++evals;
                    if (Et <= Ep + P->c1 * alpha * gp) { accepted = 1; break; }
                    alpha *= 0.5;
                }
                if (accepted) {
                    double sy = 0.0, yy = 0.0;
                    for (int q = 0; q < np; ++q) {
                        for (int k = 0; k < 2; ++k) {
                            const int d = 2 * q + k;
                            bs[d] = env[2 * mem[q] + k] - bx0[d];
                            by[d] = gt[2 * mem[q] + k] - bg[d];
                            sy += bs[d] * by[d];
                            yy += by[d] * by[d];
                        }
                    }
                    if (sy > P->eps_curv * yy) {
                        if (kh[p] == m) {
                            memmove(Sh[p], Sh[p] + dim, sizeof(double) * (size_t)(m - 1) * dim);
                            memmove(Yh[p], Yh[p] + dim, sizeof(double) * (size_t)(m - 1) * dim);
                            kh[p] = m - 1;
                        }
                        memcpy(Sh[p] + (size_t)kh[p] * dim, bs, sizeof(double) * dim);
                        memcpy(Yh[p] + (size_t)kh[p] * dim, by, sizeof(double) * dim);
                        ++kh[p];
                    }
                    for (int q = 0; q < np; ++q) {
                        nx[2 * mem[q]] = env[2 * mem[q]];
                        nx[2 * mem[q] + 1] = env[2 * mem[q] + 1];
                    }
                } else {
                    ++stalled;
                }
                for (int q = 0; q < np; ++q) mask[mem[q]] = 0;
                if (!G->jacobi) memcpy(xy, nx, sizeof(double) * 2 * n);
            }
            memcpy(xy, nx, sizeof(double) * 2 * n);
        }
        gsum_prev = gsum;
        E = oracle_energy_grad(n, xy, R, P->rad, NULL, NULL, NULL);
    }
    res->status = status;
    res->outer = t;
    res->visits = visits;
    res->evals = evals;
    res->stalled_visits = stalled;
    res->E = E;
    res->gsum = gsum_prev;
done:
    if (Sh) for (int p = 0; p < nb; ++p) free(Sh[p]);
    if (Yh) for (int p = 0; p < nb; ++p) free(Yh[p]);
    free(Sh); free(Yh); free(batch_of); free(colour_of); free(mask); free(cnt); free(start);
    free(member); free(kh); free(snap); free(env); free(nx); free(g); free(gt);
    free(bg); free(bp); free(bs); free(by); free(bx0); free(ehist);
    return rc;
}
