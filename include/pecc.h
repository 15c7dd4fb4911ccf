/*
 * pecc.h -- C ABI of the MI355X (gfx950) penalty-energy descent for packing
 * equal circles in a circle (PECC), after Zhou, He, Zheng & Li, "Geometric
 * Batch Optimization for the Packing Equal Circles in a Circle Problem on
 * Large Scale" (arXiv 2303.02650).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Array arguments are DEVICE pointers to caller-owned memory unless the
 *    comment says "host".  The library never allocates device memory; where
 *    a call needs scratch space the caller passes a workspace sized by the
 *    matching *_workspace_size query.
 *  * Calls are asynchronous and ordered on the given stream; they return
 *    after enqueueing.  Nothing is read back to the host.
 *  * A batch holds B independent instances ("packed" layout).  Instance b
 *    owns circles offset[b] .. offset[b+1]-1; positions are interleaved
 *    float pairs xy[2*i], xy[2*i+1] (the solution vector x of Def. 3.2).
 *    Circle indices in neighbor lists are global over the batch; pairs never
 *    cross instances.  Container centre is the origin (Sec. 3.1).
 *  * Every instance must satisfy 0 <= n_b <= PECC_MAX_N and R_b > 0.
 *    Instances with n_b = 0 are allowed and produce empty results.
 *  * Return value: PECC_OK or a negative PECC_ERR_* code describing an
 *    argument or launch problem; pecc_last_error() gives a message for the
 *    calling thread.  Per-instance numerical outcomes (non-finite input, a
 *    line search that cannot decrease E, ...) are reported in result
 *    structs, never as return codes.  Device-side argument problems that
 *    the host cannot see (n_b > PECC_MAX_N, decreasing offsets) make the
 *    affected instance report PECC_STATUS_BAD_INSTANCE or an empty result.
 */
#ifndef PECC_H
#define PECC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PECC_OK             0
#define PECC_ERR_INVALID   -1  /* null pointer, bad size or parameter        */
#define PECC_ERR_WORKSPACE -2  /* workspace pointer null or too small         */
#define PECC_ERR_HIP       -3  /* a HIP launch or query failed                 */

#define PECC_MAX_N        1024 /* circles per instance                        */
#define PECC_MAX_M          10 /* L-BFGS memory                               */

/* Outcome of one descent (pecc_descent_result.status). */
#define PECC_STATUS_RUNNING      0
#define PECC_STATUS_FEASIBLE     1  /* FP64 E (unit circles) < e_feasible     */
#define PECC_STATUS_STATIONARY   2  /* ||g||_2 <= g_tol                        */
#define PECC_STATUS_CONVERGED    3  /* relative decrease over ftol_window < ftol */
#define PECC_STATUS_STALLED      4  /* no step length passed the line search    */
#define PECC_STATUS_MAX_ITER     5  /* iteration budget spent                  */
#define PECC_STATUS_NONFINITE    6  /* E or g not finite                       */
#define PECC_STATUS_BAD_INSTANCE 7  /* n_b outside [0, PECC_MAX_N]             */

/* A batch of instances.  Host struct holding device pointers. */
typedef struct pecc_instances {
    int32_t        num_instances; /* B >= 1                                     */
    int32_t        max_n;         /* host: an upper bound of every n_b (<= PECC_MAX_N) */
    int64_t        total_n;       /* host: offset[B]                            */
    const int32_t *offset;        /* device [B+1], offset[0] = 0, non-decreasing */
    const float   *R;             /* device [B], container radius (FP32 copy)   */
    const double  *R64;           /* device [B] FP64 radius, or NULL: (double)R  */
} pecc_instances;

/* Thread-local description of the last error on the calling host thread. */
const char *pecc_last_error(void);

/* Library version string. */
const char *pecc_version(void);

/* ------------------------------------------------------------------------
 * Neighbor lists.  Gamma(i) = { j != i : l_ij < l_cut } (Sec. 4.3), built
 * from a uniform cell grid (counting sort of circles into square cells of
 * side >= cutoff over [-R, R]^2; clamped cell coordinates) instead of the
 * paper's scan line.  The predicate is evaluated in FP64 on the FP32
 * positions, without fused multiply-add:
 *     dx = (double)x_i - (double)x_j;  dy likewise;
 *     neighbor  <=>  dx*dx + dy*dy < cutoff*cutoff     (cutoff as double)
 * so the pair set is a deterministic function of the FP32 input.
 *
 * Output is CSR: the list of circle i is col[row[i]] .. col[row[i+1]-1],
 * ascending.  row has total_n + 1 entries (int32), row[0] = 0.  format:
 *   PECC_LIST_HALF     int32 global circle indices, only j > i (each pair
 *                      once);
 *   PECC_LIST_FULL     int32 global circle indices, both orientations;
 *   PECC_LIST_LOCAL16  uint16 instance-local indices (j - offset[b]), both
 *                      orientations: 2 bytes per entry, so the list costs
 *                      as many bytes as the half list in int32 (col must
 *                      be 2-byte aligned).
 * (The values 0 and 1 are the former full = 0 / full = 1.)
 * *num_pairs (device, one int64) receives the number of entries required.
 * If it exceeds capacity, row is still complete, nothing is written at or
 * beyond col[capacity], rows ending within the capacity are complete and
 * the row crossing it holds only part of its entries: re-run with a larger
 * col.
 * cell_size <= 0 selects cutoff; otherwise it must be >= cutoff.
 * Errors: PECC_ERR_INVALID for an unknown format or a misaligned col.
 * Workspace: pecc_build_neighbors_workspace_size().
 * ------------------------------------------------------------------------ */
#define PECC_LIST_HALF    0
#define PECC_LIST_FULL    1
#define PECC_LIST_LOCAL16 2
int pecc_build_neighbors_workspace_size(const pecc_instances *inst, size_t *bytes /*host*/);
int pecc_build_neighbors(const pecc_instances *inst, const float *xy,
                         double cutoff, float cell_size, int32_t format,
                         int32_t *row, void *col, int64_t capacity,
                         int64_t *num_pairs, void *workspace, size_t workspace_bytes,
                         hipStream_t stream);

/* ------------------------------------------------------------------------
 * Energy and gradient (Def. 3.1, Def. 3.2; E = sum_{i<j} d_ij^2 +
 * sum_i d_i0^2) in FP32 over a neighbor list from pecc_build_neighbors in
 * the given format (PECC_LIST_*).  Pairs outside the list contribute
 * nothing, so the list must contain every overlapping pair (any list built
 * with cutoff >= 2*rad at positions each circle has since moved less than
 * (cutoff - 2*rad)/2 from qualifies).  Entries j <= i of a PECC_LIST_HALF
 * row are skipped, so a list with both orientations passed as HALF holds
 * the same pairs.  Each circle's gradient is accumulated by one thread in
 * ascending order of the other circle (no atomics), so the result is
 * bitwise reproducible; the two forms with both orientations give the same
 * bits, the half form the same values to FP32 rounding.
 *   PECC_LIST_LOCAL16  the compact form (2 bytes per entry, 4 bytes per
 *                      pair): the sweep of choice;
 *   PECC_LIST_FULL     the same sweep over int32 global indices;
 *   PECC_LIST_HALF     each pair's term formed once and the partners below
 *                      a circle gathered on chip (a counting sort of the
 *                      list by the higher circle).
 * rad is the circle radius used by the energy (1 for unit circles).
 * col_len is the number of entries col holds: list entries at or beyond it
 * are never read.  An instance whose row range leaves [0, col_len) gets
 * energy NaN, and so does, with PECC_LIST_HALF, one whose row offsets
 * decrease (its gradient is then not written).
 * energy: device [B]; grad: device [2*total_n] or NULL.
 * Errors: PECC_ERR_INVALID for an unknown format or a misaligned col.
 * ------------------------------------------------------------------------ */
int pecc_energy_grad(const pecc_instances *inst, const float *xy,
                     const int32_t *row, const void *col, int64_t col_len, int32_t format,
                     float rad, float *energy, float *grad, hipStream_t stream);

/* ------------------------------------------------------------------------
 * L-BFGS descent of E at fixed R (Alg. 1 with the limited-memory reading of
 * Eq. 8-11 and a backtracking line search in place of the exact one of
 * Eq. 9), run for every instance of the batch in ONE persistent launch.
 * Each workgroup takes instances from a queue (largest n first), keeps the
 * instance's positions, neighbor list and curvature history on chip and
 * iterates until a stop test holds.  xy is updated in place.  The FP32
 * arithmetic uses R; the FP64 decisions (FEASIBLE, the near-zero
 * sufficient-decrease test) use R64 when it is given, like pecc_verify.
 * ------------------------------------------------------------------------ */
typedef struct pecc_descent_params {
    int32_t m;              /* L-BFGS memory, 1..PECC_MAX_M (10)               */
    int32_t max_iter;       /* iteration budget (paper: MaxIter = 5000)        */
    int32_t max_halvings;   /* step halvings per line search (40)              */
    int32_t ftol_window;    /* iterations spanned by the decrease test (20)    */
    float   c1;             /* sufficient-decrease constant (1e-4)             */
    float   eps_curv;       /* keep (s,y) only if s'y > eps_curv * y'y (1e-8)  */
    float   cutoff;         /* neighbor-list cutoff (2.3)                      */
    float   skin_half;      /* rebuild when a circle moved more than this (0.15) */
    float   cell_size;      /* cell side, >= cutoff; <= 0 selects cutoff       */
    float   g_tol;          /* stop when ||g||_2 <= g_tol (FP32)               */
    float   ftol;           /* stop when E fell by <= ftol*E over the window; 0 = off */
    float   contact_margin; /* mu >= 0: the descent works on circles of radius 1+mu */
    double  e_feasible;     /* FEASIBLE when FP64 E of unit circles < this (1e-20) */
    double  tau64;          /* FP64 regime once min(E32, FP32 E of unit circles)
                               < tau64 (3e-6): from then on every evaluation also
                               forms the FP64 energies, the sufficient-decrease
                               test uses them and FEASIBLE can be decided;
                               0 = never                                        */
} pecc_descent_params;

typedef struct pecc_descent_result {
    int32_t status;         /* PECC_STATUS_*                                   */
    int32_t iters;          /* accepted iterations                             */
    int32_t evals;          /* energy/gradient evaluations                     */
    int32_t rebuilds;       /* neighbor-list rebuilds (the first one included) */
    int64_t pair_evals;     /* sum over evaluations of listed pairs (i<j)      */
    float   E32;            /* final FP32 energy of the descent's objective    */
    float   gnorm;          /* final ||g||_2 (FP32)                             */
    double  E64;            /* final FP64 energy of unit circles, or -1 if the
                               descent never entered the FP64 regime           */
    int32_t cell_evals;     /* evaluations swept over the cell grid instead of
                               the neighbor lists: a list overflowed, or (the
                               geometric batch descent) a trial moved a circle
                               of its batch beyond the skin                    */
    int32_t reserved;       /* 0                                               */
} pecc_descent_result;

/* Fill *p with the defaults listed above. (host) */
void pecc_descent_params_default(pecc_descent_params *p);

int pecc_lbfgs_descend_workspace_size(const pecc_instances *inst, size_t *bytes /*host*/);
int pecc_lbfgs_descend(const pecc_instances *inst, float *xy,
                       const pecc_descent_params *params /*host*/,
                       pecc_descent_result *out /*device [B]*/,
                       void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * pecc_lbfgs_descend without a workspace, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  The descent's scratch memory (its work queue,
 * num_instances + 1 int32) is a fixed array inside the library, one per
 * device, held until the process ends: PECC_NOALLOC_MAX_INSTANCES + 1 words
 * (256 KiB).  The call allocates nothing; the caller still owns xy and out.
 * Same arguments, results and errors as pecc_lbfgs_descend, bit for bit,
 * plus PECC_ERR_INVALID when num_instances exceeds
 * PECC_NOALLOC_MAX_INSTANCES.  Every call on a device shares that device's
 * array: calls that overlap on one device (other streams, other host
 * threads) race and must be serialised by the caller; consecutive calls on
 * one stream are fine (the queue is re-initialised by a kernel each call).
 * ------------------------------------------------------------------------ */
#define PECC_NOALLOC_MAX_INSTANCES 65536
int pecc_lbfgs_descend_noalloc(const pecc_instances *inst, float *xy,
                               const pecc_descent_params *params /*host*/,
                               pecc_descent_result *out /*device [B]*/, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Geometric batch descent (Alg. 1 with the batch energy of Eq. 7 and the
 * limited-memory reading of Eq. 8-11) for every instance of the batch, one
 * persistent launch.  The circles are partitioned once, from the input
 * positions, into the blocks of a blocks x blocks grid over [-R, R]^2
 * (block side 2R / blocks, computed in FP64); block (bx, by) has colour
 * (bx mod 2) + 2 (by mod 2).  An outer iteration visits the colours in
 * turn; every batch of the colour takes one quasi-Newton step on its batch
 * energy with the other circles at their positions from the start of the
 * colour.  Each batch keeps its own (s, y) history (memory params->m).
 * A trial step that would move a circle more than skin_half from the
 * positions of the last neighbor-list rebuild is halved.
 * params->max_iter counts outer iterations; result.iters as well,
 * result.gnorm is the sum over batches of ||g(x_p)||_2 of the last outer
 * iteration (the stop quantity of Alg. 1), result.E64 the FP64 energy of
 * unit circles.  Stop tests (FP32 except E64): E64 < e_feasible, that sum
 * <= g_tol, relative decrease of E over ftol_window outer iterations <=
 * ftol, max_iter.  tau64 is not used.
 * sweep_fp64 = 1 evaluates the pair terms and batch energies in FP64 (the
 * line search then tests FP64 energies; directions stay FP32).
 * Limits: 1 <= blocks <= 8 and at most 128 circles per block (a larger
 * block makes that instance report PECC_STATUS_BAD_INSTANCE).
 * ------------------------------------------------------------------------ */
int pecc_gbo_descend_workspace_size(const pecc_instances *inst, int32_t blocks,
                                    size_t *bytes /*host*/);
int pecc_gbo_descend(const pecc_instances *inst, float *xy,
                     const pecc_descent_params *params /*host*/, int32_t blocks,
                     int32_t sweep_fp64, pecc_descent_result *out /*device [B]*/,
                     void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * k-batch partitions (Sec. 4.1).  The circles of every instance are ordered
 * by a key and cut into k consecutive runs: batch p holds floor(n/k) +
 * [p < n mod k] circles (every size floor(n/k) or ceil(n/k), the larger
 * ones first).  Equal keys order by circle index.  Keys:
 *   PECC_PARTITION_SECTOR   polar angle atan2(y, x) in (-pi, pi] (the full
 *                           angle: arctan(y/x) would merge opposite
 *                           quadrants), compared exactly from the FP32
 *                           positions without evaluating an angle;
 *   PECC_PARTITION_ANNULUS  x^2 + y^2 (FP64);
 *   PECC_PARTITION_FENCE    x;
 *   PECC_PARTITION_RANDOM   word 0 of Philox4x64-10 at counter (i, b, 0,
 *                           2^62) with key (seed, 0), i the circle's index
 *                           in instance b: a uniformly random partition.
 * xy: device [2*total_n]; batch_of: device int32 [total_n] (caller-owned),
 * batch of every circle.  seed is used by the random kind only.
 * Errors: PECC_ERR_INVALID for an unknown kind, k outside [1, PECC_MAX_N]
 * or null pointers.  Instances with invalid offsets are skipped.
 * ------------------------------------------------------------------------ */
#define PECC_PARTITION_SECTOR  0
#define PECC_PARTITION_ANNULUS 1
#define PECC_PARTITION_FENCE   2
#define PECC_PARTITION_RANDOM  3
int pecc_partition(const pecc_instances *inst, const float *xy, int32_t kind, int32_t k,
                   uint64_t seed, int32_t *batch_of, hipStream_t stream);

/* ------------------------------------------------------------------------
 * k-batch descent: Alg. 1 over a given partition, the batches visited one
 * after another (Gauss-Seidel), each visit one L-BFGS iteration (the
 * limited-memory reading of Eq. 8-11, memory params->m per batch) on the
 * batch energy of Eq. 7 with the other circles where the earlier visits
 * left them.  Every outer iteration starts with the whole instance's
 * energy and the stop tests: FP64 energy of unit circles < e_feasible
 * (FEASIBLE), the sum over batches of ||g(x_p)||_2 of the previous outer
 * iteration <= g_tol (STATIONARY, the stop rule of Alg. 1), relative
 * decrease of E over ftol_window outer iterations <= ftol (CONVERGED), every
 * visit of the previous outer iteration failed its line search (STALLED),
 * max_iter outer iterations (MAX_ITER).  The line searches test FP64 batch
 * energies once E32 < tau64 at the top of an outer iteration.
 * anm = 0: neighbor lists with cutoff params->cutoff, rebuilt when a circle
 * moved more than skin_half (every pair within the cutoff is seen).
 * anm = 1: ANM (Sec. 4.3, Alg. 3) with l_cut = params->cutoff (the paper:
 * 4): after every outer iteration a counter grows, and once it reaches the
 * deferring length the lists of the current positions are compared with
 * the stored ones -- different: they replace them and the length is reset
 * to 1; equal: the length doubles.  Energies are then over the stored lists
 * only (a pair that came closer than 2 without being listed is not seen;
 * a circle with more than 32 neighbors within l_cut makes the sweep use the
 * cell grid of the last rebuild, a superset).
 * batch_of: device int32 [total_n], batch of every circle in [0, k) (e.g.
 * from pecc_partition); an id outside makes that instance report
 * PECC_STATUS_BAD_INSTANCE.  With one non-empty batch the descent is the
 * whole-instance L-BFGS descent (ANM after every iteration).
 * Results: iters = outer iterations, gnorm = the sum of batch gradient
 * norms of the last outer iteration, E32 = whole-instance FP32 energy,
 * E64 = FP64 energy of unit circles (over the lists).  rebuilds counts list
 * builds.  Workspace: pecc_gbo_kbatch_descend_workspace_size bytes.
 * Errors: PECC_ERR_INVALID for k outside [1, PECC_MAX_BATCHES], anm not 0
 * or 1, or the descent parameters pecc_lbfgs_descend rejects.
 * ------------------------------------------------------------------------ */
#define PECC_MAX_BATCHES 16
int pecc_gbo_kbatch_descend_workspace_size(const pecc_instances *inst, size_t *bytes /*host*/);
int pecc_gbo_kbatch_descend(const pecc_instances *inst, float *xy, const int32_t *batch_of,
                            int32_t k, int32_t anm, const pecc_descent_params *params /*host*/,
                            pecc_descent_result *out /*device [B]*/, void *workspace,
                            size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * The same k-batch descent with the paper's dense inverse-Hessian
 * approximation of every batch (Eq. 8-11) instead of the limited-memory
 * history: H_p = I at the start; a visit moves along p = -H_p g(x_p) with
 * the backtracking line search (alpha0 = 1 once H_p has been updated,
 * 1/max(1, ||g||) before) and, when s'y > eps_curv y'y, applies Eq. 11
 *     H_p <- (I - s y'/beta) H_p (I - y s'/beta) + s s'/beta,  beta = y's,
 * as H_p - (w s' + s w')/beta + (y'w/beta^2 + 1/beta) s s' with w = H_p y.
 * A direction with g'p >= 0 resets H_p to I.  FP32 matrices of 2|B_p|
 * rows of 2|B_p| floats, each row padded to a multiple of 4 floats (64
 * above 1024 floats), and four vectors of 2|B_p| floats per batch live in
 * the workspace (per instance 4 * max_batch * max_n + 12 * max_n floats,
 * + 132 * max_n when 2 * max_batch > 1024, rounded up to a multiple of 64;
 * max_batch >= every batch's size; an instance whose batches need more
 * reports PECC_STATUS_BAD_INSTANCE).  The stored matrix runs one
 * update behind (the newest update is carried as vectors and applied by
 * the next visit's pass), so a visit reads H_p once and writes it once: the
 * memory traffic per outer iteration falls as 1/k, which is where the
 * paper's batching gains.  One batch (k = 1) is dense BFGS on the whole
 * instance.  Other arguments, stop tests and results as
 * pecc_gbo_kbatch_descend (params->m only caps the update count that
 * selects alpha0).  The workspace must be 256-byte aligned.
 * ------------------------------------------------------------------------ */
int pecc_gbo_kbatch_bfgs_workspace_size(const pecc_instances *inst, int32_t max_batch,
                                        size_t *bytes /*host*/);
int pecc_gbo_kbatch_bfgs_descend(const pecc_instances *inst, float *xy, const int32_t *batch_of,
                                 int32_t k, int32_t anm, int32_t max_batch,
                                 const pecc_descent_params *params /*host*/,
                                 pecc_descent_result *out /*device [B]*/, void *workspace,
                                 size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * FP64 feasibility check of Eq. 1-2 through the energy of Def. 3.2 with
 * unit circles: every pair i<j of each instance is enumerated (no list),
 * in FP64 on the FP32 positions.  Per instance: energy64 = E,
 * max_pair_overlap = max_{i<j} d_ij, max_cont_overlap = max_i d_i0 (both
 * >= 0), feasible = (E < tol).  Any output pointer except energy64 may be
 * NULL.  Radii come from R64 when given, else from R.
 * ------------------------------------------------------------------------ */
int pecc_verify(const pecc_instances *inst, const float *xy, double tol,
                double *energy64, double *max_pair_overlap, double *max_cont_overlap,
                int32_t *feasible, hipStream_t stream);

/* ------------------------------------------------------------------------
 * The smallest FP32 container radius of each layout (the radius that the
 * framework of Alg. 4 records), from the same FP64 enumeration as
 * pecc_verify.  rho_max = max_i fl(|c_i| + 1) in FP64; at any radius
 * R >= rho_max every containment term of Eq. 2 vanishes, so the unit
 * circles fit exactly when their pair energy is below tol.  Per instance:
 * R_out[b] = rho_max rounded up to an FP32 value when the pair energy is
 * below tol and that value is below the instance's radius (R64 when given,
 * else R), otherwise R[b]; feasible[b] = 1 when the layout is feasible
 * (E < tol) at radius R_out[b].  An instance with no circles keeps R[b];
 * one with a non-finite coordinate keeps R[b] with feasible 0.
 * R_out: device float [B]; feasible: device int32 [B]; both required.
 * Errors: PECC_ERR_INVALID for a NULL output, or xy NULL with circles.
 * ------------------------------------------------------------------------ */
int pecc_verify_tighten(const pecc_instances *inst, const float *xy, double tol, float *R_out,
                        int32_t *feasible, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Container adjustment (Sec. 4.2, Eq. 12, Alg. 2): the radius becomes a
 * variable and U(z, lambda) = E + lambda R^2 is minimised over z = (x, R),
 * `rounds` times (35 in the paper) with lambda halved after each round from
 * lambda0 (1e-4), every round a fresh L-BFGS descent with the stop rules of
 * p (g_tol / ftol / max_iter per round; no FEASIBLE stop since U > 0 and no
 * FP64 regime: tau64 and e_feasible are not used).  The radius component of
 * the gradient is dU/dR = -2 sum_i d_i0 + 2 lambda R.
 * inst->R holds the starting radii; R_out (device float [B]) receives the
 * final ones and xy the final layouts.  out[b].iters counts iterations over
 * all rounds, out[b].status is the last round's, out[b].E32 the energy E
 * (circles of radius 1 + contact_margin) at the final layout and radius.
 * FP32 positions bound the radius to about the FP32 spacing of the
 * coordinates times a few; check feasibility of unit circles with
 * pecc_verify at the returned radii (a contact margin leaves slack for it).
 * Errors: as pecc_lbfgs_descend, plus lambda0 < 0 or not finite, rounds
 * outside [0, 64], R_out NULL.
 * ------------------------------------------------------------------------ */
int pecc_adjust_container_workspace_size(const pecc_instances *inst, size_t *bytes);
int pecc_adjust_container(const pecc_instances *inst, float *xy, const pecc_descent_params *p,
                          float lambda0, int32_t rounds, float *R_out, pecc_descent_result *out,
                          void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ========================================================================
 * SED, the solution-space exploring and descent heuristic (Sec. 5, Alg. 5),
 * batched over B independent chains (a chain = an instance of `chains`, all
 * at a fixed radius).  One SED iteration of every chain:
 *   pecc_sed_plan      m_b = max(1, J(E_cur[b])) candidates, J = ceil(-log10 E)
 *                      capped at M (E <= 0 counts as the cap), and m_b = 0 once
 *                      E_best[b] <= e_stop (1e-25); lays the candidates out as
 *                      one packed batch of B*M instances (slot b*M + j holds n_b
 *                      circles when j < m_b, none otherwise): cand_offset
 *                      [B*M + 1], cand_R / cand_R64 [B*M] (the chain's radius);
 *   pecc_sed_perturb   candidate j of chain b = xy_b + r, every coordinate k
 *                      shifted by r = u * 1.6 - 0.8 (FP32, two roundings),
 *                      u = (w >> 40) 2^-24 with w word k mod 4 of the
 *                      Philox4x64-10 block at counter (k / 4, j, iter, b) and
 *                      key (seed, 0) (Salmon et al., SC 2011);
 *   (pecc_lbfgs_descend and pecc_verify on the candidate batch; cand_E [B*M]
 *    = its energy64)
 *   pecc_sed_select    Eq. 18: the lowest-energy candidate if it is below
 *                      E_cur[b] (lowest j among equal energies), else candidate
 *                      k with probability exp(J_k) / sum exp(J), drawn with
 *                      u = (w >> 11) 2^-53, w word 0 of the Philox block at
 *                      counter (2^63, 0, iter, b); xy_cur/E_cur take it, and
 *                      xy_best/E_best when it is below E_best.  chosen [B]
 *                      (nullable) gets k, -1 for an inactive chain.
 * M in [1, PECC_SED_MAX_CAND], B * M <= 2^24.  All arrays are device memory.
 * ======================================================================== */
#define PECC_SED_MAX_CAND 64

int pecc_sed_plan(const pecc_instances *chains, const double *E_cur, const double *E_best,
                  int32_t M, double e_stop, int32_t *m, int32_t *cand_offset, float *cand_R,
                  double *cand_R64, hipStream_t stream);
int pecc_sed_perturb(const pecc_instances *chains, const float *xy, int32_t M, const int32_t *m,
                     const int32_t *cand_offset, uint64_t seed, int32_t iter, float *cand_xy,
                     hipStream_t stream);
int pecc_sed_select(const pecc_instances *chains, int32_t M, const int32_t *m,
                    const int32_t *cand_offset, const float *cand_xy, const double *cand_E,
                    uint64_t seed, int32_t iter, float *xy_cur, double *E_cur, float *xy_best,
                    double *E_best, int32_t *chosen, hipStream_t stream);

/* ========================================================================
 * Learned proposal for the perturbation step of SED (Sec. 5, Alg. 5).
 *
 * SED perturbs the current layout and descends again.  Here the
 * perturbation relocates k distinct circles; a candidate is a pair
 * (circle i, destination q), q drawn by the caller uniformly in the disk of
 * radius R - 1.  A small network scores candidates from local features and
 * the k best-scored distinct circles move to their candidates' points.  The
 * network is the project's addition (the paper perturbs every circle by a
 * random shift); uniform random choice is the fallback, and the descent's
 * final FP64 energy decides what is kept (pecc_accept).
 * ======================================================================== */
#define PECC_FEATURES     8     /* features per candidate                       */
#define PECC_MLP_PARAMS   4801  /* network parameters (layout below)            */

/* Features of candidates: for instance b, candidate c (0 <= c < C) names the
 * local circle cand_circle[b*C + c] (0-based within the instance) and the
 * point cand_dest[2*(b*C + c) + {0,1}].  Output features[8*(b*C + c) + f]:
 *   f = 0..3 around the circle's own centre, 4..7 around the destination,
 *   each time over the other circles j != i (i lifted out):
 *   0/4  overlap energy e of a unit circle there (sum over j of
 *        max(0, 2 - l)^2 plus max(0, rho + 1 - R)^2), as log10(e + 1e-20)/20 + 1
 *   1/5  number of j with l < 2.3
 *   2/6  boundary gap (R - 1 - rho) / R
 *   3/7  number of j with l < 4, divided by 16 pi
 * Distances are FP64 on the FP32 coordinates (counts are exact); results
 * are rounded to FP32.  A candidate whose circle index is outside
 * [0, n_b) gets NaN features.  Errors: PECC_ERR_INVALID for null pointers,
 * C < 0 or B*C >= 2^31. */
int pecc_features(const pecc_instances *inst, const float *xy, int32_t cands_per_inst,
                  const int32_t *cand_circle, const float *cand_dest, float *features,
                  hipStream_t stream);

/* Network 8 -> 64 -> 64 -> 1 with GELU(t) = t Phi(t) (erf form) after both
 * hidden layers.  params: FP32 master values, device [PECC_MLP_PARAMS]:
 *   W1 [64][8] at 0, b1 [64] at 512, W2 [64][64] at 576, b2 [64] at 4672,
 *   W3 [64] at 4736, b3 at 4800  (W[out][in], row-major).
 * The weight matrices are used as their BF16 roundings (nearest even);
 * biases stay FP32.  Products run on BF16 matrix cores with FP32
 * accumulation, hidden activations enter them as BF16.
 * features: device [rows][8] FP32; logits: device [rows] FP32 (the score).
 * Errors: PECC_ERR_INVALID for rows < 0 or null pointers (rows > 0). */
int pecc_mlp_forward(const float *params, const float *features, int64_t rows, float *logits,
                     hipStream_t stream);

/* Workspace of pecc_mlp_grad / pecc_mlp_train_step for a given row count. */
int pecc_mlp_grad_workspace_size(int64_t rows, size_t *bytes);

/* Mean binary cross-entropy of sigmoid(logit) against labels (device
 * [rows], values 0 or 1) and its gradient with respect to the parameters as
 * used (the BF16 weights; apply it to the FP32 masters).  loss: device [1]
 * (nullable); grad: device [PECC_MLP_PARAMS].  Per-workgroup partial sums
 * are added in a fixed order: the result does not depend on timing.
 * rows = 0 gives loss 0 and a zero gradient.  Errors: PECC_ERR_INVALID,
 * PECC_ERR_WORKSPACE. */
int pecc_mlp_grad(const float *params, const float *features, const float *labels, int64_t rows,
                  float *loss, float *grad, void *ws, size_t ws_bytes, hipStream_t stream);

typedef struct pecc_adam_params {
    float lr;       /* step size (1e-3)                                           */
    float beta1;    /* first-moment decay (0.9)                                   */
    float beta2;    /* second-moment decay (0.999)                                */
    float eps;      /* denominator guard (1e-8)                                   */
} pecc_adam_params;

/* One Adam step (Kingma & Ba, bias-corrected) on FP32 params, moments m and
 * v (device [PECC_MLP_PARAMS] each, zero before the first step).  step:
 * device int32 [1], the number of steps taken so far; the call uses
 * t = *step + 1 and then stores t, so it can be replayed from a graph.
 * Errors: PECC_ERR_INVALID for null pointers, lr < 0, beta outside [0, 1),
 * eps <= 0. */
int pecc_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t *step,
                  const pecc_adam_params *hp, hipStream_t stream);

/* pecc_mlp_grad followed by pecc_mlp_adam on the same stream; grad is the
 * caller's buffer for the gradient in between. */
int pecc_mlp_train_step(float *params, float *m, float *v, int32_t *step,
                        const pecc_adam_params *hp, const float *features, const float *labels,
                        int64_t rows, float *loss, float *grad, void *ws, size_t ws_bytes,
                        hipStream_t stream);

/* Proposal.  Per instance: every circle named by a candidate is represented
 * by its best candidate (highest score, the lower candidate index among
 * equal scores); circles are ranked by that score, equal scores by the lower
 * candidate index, and the first k (or as many distinct circles as there
 * are) are chosen.  scores: device [B*C] or NULL; NULL, or a NaN among an
 * instance's scores, makes all of that instance's scores equal: the choice is
 * then the first k distinct circles in candidate order, a uniform random
 * subset for uniformly drawn candidates.  Candidates naming a circle outside
 * [0, n_b) are ignored.
 * xy_out (device, layout of xy; may equal xy) receives xy with each chosen
 * circle moved to its candidate's destination.  selected (device [B*k],
 * nullable) receives the chosen candidate indices in rank order, -1 past
 * the last.  Errors: PECC_ERR_INVALID for null pointers, C < 0, k < 0. */
int pecc_propose(const pecc_instances *inst, const float *xy, int32_t cands_per_inst,
                 const int32_t *cand_circle, const float *cand_dest, const float *scores,
                 int32_t k, int32_t *selected, float *xy_out, hipStream_t stream);

/* Acceptance (SED keeps a candidate layout that lowers the energy): for each
 * instance with e_new[b] < e_cur[b] (FP64, e.g. pecc_verify's energy64),
 * copy its circles from xy_new into xy_cur and set e_cur[b] = e_new[b].
 * accepted: device [B] (nullable), 1 where taken.  A NaN e_new is never
 * taken. */
int pecc_accept(const pecc_instances *inst, float *xy_cur, double *e_cur, const float *xy_new,
                const double *e_new, int32_t *accepted, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* PECC_H */
