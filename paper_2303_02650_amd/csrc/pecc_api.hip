// C ABI of libpecc: argument validation, workspace sizing, launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "pecc.h"
#include "pecc_launch.hpp"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return PECC_OK;
    return fail(PECC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int check_inst(const pecc_instances *in, const char *fn)
{
    if (!in) return fail(PECC_ERR_INVALID, "%s: instances is NULL", fn);
    if (in->num_instances < 1) return fail(PECC_ERR_INVALID, "%s: num_instances must be >= 1", fn);
    if (!in->offset || !in->R) return fail(PECC_ERR_INVALID, "%s: offset and R must be set", fn);
    if (in->max_n < 0 || in->max_n > PECC_MAX_N)
        return fail(PECC_ERR_INVALID, "%s: max_n = %d outside [0, %d]", fn, in->max_n, PECC_MAX_N);
    if (in->total_n < 0 || in->total_n > 0x7ffffffeLL)
        return fail(PECC_ERR_INVALID, "%s: total_n = %lld outside [0, 2^31-2]", fn,
                    (long long)in->total_n);
    return PECC_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

const char *pecc_last_error(void) { return g_err; }

const char *pecc_version(void) { return "pecc-mi355x 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
int pecc_build_neighbors_workspace_size(const pecc_instances *inst, size_t *bytes)
{
    int rc = check_inst(inst, "pecc_build_neighbors_workspace_size");
    if (rc) return rc;
    if (!bytes) return fail(PECC_ERR_INVALID, "pecc_build_neighbors_workspace_size: bytes is NULL");
    *bytes = align256(sizeof(int64_t) * (size_t)inst->num_instances);
    return PECC_OK;
}

int pecc_build_neighbors(const pecc_instances *inst, const float *xy, double cutoff,
                         float cell_size, int32_t format, int32_t *row, void *col,
                         int64_t capacity, int64_t *num_pairs, void *workspace,
                         size_t workspace_bytes, hipStream_t stream)
{
    const char *fn = "pecc_build_neighbors";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (format != PECC_LIST_HALF && format != PECC_LIST_FULL && format != PECC_LIST_LOCAL16)
        return fail(PECC_ERR_INVALID, "%s: unknown list format %d", fn, format);
    if (format == PECC_LIST_LOCAL16 && (reinterpret_cast<uintptr_t>(col) & 1))
        return fail(PECC_ERR_INVALID, "%s: a 16-bit list must be 2-byte aligned", fn);
    if (!(cutoff > 0.0) || !isfinite(cutoff)) return fail(PECC_ERR_INVALID, "%s: cutoff must be > 0", fn);
    if (cell_size > 0.f && (double)cell_size < cutoff)
        return fail(PECC_ERR_INVALID, "%s: cell_size %g < cutoff %g", fn, cell_size, cutoff);
    if (!row || !num_pairs) return fail(PECC_ERR_INVALID, "%s: row and num_pairs must be set", fn);
    if (inst->total_n > 0 && !xy) return fail(PECC_ERR_INVALID, "%s: xy is NULL", fn);
    if (capacity < 0 || capacity > 0x7fffffffLL)
        return fail(PECC_ERR_INVALID, "%s: capacity outside [0, 2^31-1]", fn);
    if (capacity > 0 && !col) return fail(PECC_ERR_INVALID, "%s: col is NULL", fn);
    size_t need = 0;
    pecc_build_neighbors_workspace_size(inst, &need);
    if (!workspace || workspace_bytes < need)
        return fail(PECC_ERR_WORKSPACE, "%s: workspace needs %zu bytes", fn, need);
    const float h = (float)((cell_size > 0.f ? (double)cell_size : cutoff) * (1.0 + 1e-4));
    return check_hip(pecc::launch_build(inst->offset, inst->R, xy, inst->num_instances,
                                        inst->total_n, cutoff, h, format, row, col,
                                        capacity, num_pairs, (int64_t *)workspace, stream),
                     fn);
}

// ---------------------------------------------------------------------------
int pecc_energy_grad(const pecc_instances *inst, const float *xy, const int32_t *row,
                     const void *col, int64_t col_len, int32_t format, float rad,
                     float *energy, float *grad, hipStream_t stream)
{
    const char *fn = "pecc_energy_grad";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (format != PECC_LIST_HALF && format != PECC_LIST_FULL && format != PECC_LIST_LOCAL16)
        return fail(PECC_ERR_INVALID, "%s: unknown list format %d", fn, format);
    if (format == PECC_LIST_LOCAL16 && (reinterpret_cast<uintptr_t>(col) & 1))
        return fail(PECC_ERR_INVALID, "%s: a 16-bit list must be 2-byte aligned", fn);
    if (!energy) return fail(PECC_ERR_INVALID, "%s: energy is NULL", fn);
    if (!row) return fail(PECC_ERR_INVALID, "%s: row is NULL", fn);
    if (inst->total_n > 0 && !xy) return fail(PECC_ERR_INVALID, "%s: xy is NULL", fn);
    if (!(rad > 0.f) || !isfinite(rad)) return fail(PECC_ERR_INVALID, "%s: rad must be > 0", fn);
    if (col_len < 0) return fail(PECC_ERR_INVALID, "%s: col_len < 0", fn);
    if (col_len > 0 && !col) return fail(PECC_ERR_INVALID, "%s: col is NULL", fn);
    return check_hip(pecc::launch_energy_grad(inst->offset, inst->R, xy, inst->num_instances,
                                              inst->total_n, row, col, col_len, format, rad,
                                              energy, grad, stream),
                     fn);
}

// ---------------------------------------------------------------------------
void pecc_descent_params_default(pecc_descent_params *p)
{
    if (!p) return;
    p->m = 10;
    p->max_iter = 5000;
    p->max_halvings = 40;
    p->ftol_window = 20;
    p->c1 = 1e-4f;
    p->eps_curv = 1e-8f;
    p->cutoff = 2.3f;
    p->skin_half = 0.15f;
    p->cell_size = 0.f;
    p->g_tol = 1e-6f;
    p->ftol = 1e-7f;
    p->contact_margin = 0.f;
    p->e_feasible = 1e-20;
    p->tau64 = 3e-6;
}

int pecc_lbfgs_descend_workspace_size(const pecc_instances *inst, size_t *bytes)
{
    int rc = check_inst(inst, "pecc_lbfgs_descend_workspace_size");
    if (rc) return rc;
    if (!bytes) return fail(PECC_ERR_INVALID, "pecc_lbfgs_descend_workspace_size: bytes is NULL");
    *bytes = align256(sizeof(int32_t) * ((size_t)inst->num_instances + 1));
    return PECC_OK;
}

namespace {

// Largest float x >= 0 with sqrtf(x) <= t.  Both host and device square
// roots are correctly rounded, hence monotonic, so sqrtf(x) <= t exactly
// when x <= sqrt_threshold(t).
float sqrt_threshold(float t)
{
    if (!(t >= 0.f)) return -1.f;
    if (isinf(t)) return INFINITY;
    float x = t * t;
    if (isinf(x)) x = 3.40282347e38f;
    while (x > 0.f && sqrtf(x) > t) x = nextafterf(x, 0.f);
    for (;;) {
        const float up = nextafterf(x, INFINITY);
        if (isinf(up) || sqrtf(up) > t) break;
        x = up;
    }
    return x;
}

// Validates the descent constants and derives the kernels' form of them.
int descent_args(const pecc_descent_params *p, const char *fn, pecc::DescentArgs *a)
{
    if (p->m < 1 || p->m > PECC_MAX_M) return fail(PECC_ERR_INVALID, "%s: m = %d outside [1, %d]", fn, p->m, PECC_MAX_M);
    if (p->max_iter < 0) return fail(PECC_ERR_INVALID, "%s: max_iter < 0", fn);
    if (p->max_halvings < 0 || p->max_halvings > 200) return fail(PECC_ERR_INVALID, "%s: max_halvings outside [0, 200]", fn);
    if (p->ftol_window < 1 || p->ftol_window > 63) return fail(PECC_ERR_INVALID, "%s: ftol_window outside [1, 63]", fn);
    if (!(p->c1 > 0.f && p->c1 < 1.f)) return fail(PECC_ERR_INVALID, "%s: c1 outside (0, 1)", fn);
    if (!(p->eps_curv >= 0.f)) return fail(PECC_ERR_INVALID, "%s: eps_curv < 0", fn);
    if (!(p->contact_margin >= 0.f && p->contact_margin < 0.5f)) return fail(PECC_ERR_INVALID, "%s: contact_margin outside [0, 0.5)", fn);
    if (!(p->skin_half > 0.f)) return fail(PECC_ERR_INVALID, "%s: skin_half must be > 0", fn);
    if (!(p->g_tol >= 0.f) || !(p->ftol >= 0.f)) return fail(PECC_ERR_INVALID, "%s: g_tol and ftol must be >= 0", fn);
    const double rad = 1.0 + (double)p->contact_margin;
    // a pair can only be missed if both circles moved by more than half of
    // the margin between the list cutoff and the overlap distance 2*rad
    const double room = ((double)p->cutoff - 2.0 * rad) / 2.0;
    if (!(room > 0.0))
        return fail(PECC_ERR_INVALID, "%s: cutoff %g must exceed 2*(1+contact_margin)", fn, p->cutoff);
    if (p->cell_size > 0.f && p->cell_size < p->cutoff)
        return fail(PECC_ERR_INVALID, "%s: cell_size %g < cutoff %g", fn, p->cell_size, p->cutoff);
    a->m = p->m;
    a->max_iter = p->max_iter;
    a->max_halvings = p->max_halvings;
    a->ftol_window = p->ftol_window;
    a->c1 = p->c1;
    a->eps_curv = p->eps_curv;
    a->h_req = (float)((p->cell_size > 0.f ? p->cell_size : p->cutoff) * (1.0 + 1e-4));
    a->g_tol = p->g_tol;
    a->g_tol_sq = sqrt_threshold(p->g_tol);
    a->ftol = p->ftol;
    a->rad = (float)rad;
    a->c2 = (double)p->cutoff * (double)p->cutoff;
    const double skin = (double)p->skin_half < room ? (double)p->skin_half : room;
    a->skin2 = skin * skin;
    a->e_feasible = p->e_feasible;
    a->tau64 = p->tau64;
    a->lambda0 = 0.f;
    a->rounds = 0;
    a->nbat = 1;
    a->anm = 0;
    a->hstride = 0;
    return PECC_OK;
}

}  // namespace

int pecc_lbfgs_descend(const pecc_instances *inst, float *xy, const pecc_descent_params *p,
                       pecc_descent_result *out, void *workspace, size_t workspace_bytes,
                       hipStream_t stream)
{
    const char *fn = "pecc_lbfgs_descend";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (!p || !out) return fail(PECC_ERR_INVALID, "%s: params and out must be set", fn);
    if (inst->total_n > 0 && !xy) return fail(PECC_ERR_INVALID, "%s: xy is NULL", fn);
    pecc::DescentArgs a;
    rc = descent_args(p, fn, &a);
    if (rc) return rc;
    size_t need = 0;
    pecc_lbfgs_descend_workspace_size(inst, &need);
    if (!workspace || workspace_bytes < need)
        return fail(PECC_ERR_WORKSPACE, "%s: workspace needs %zu bytes", fn, need);
    const int grid = pecc::descend_grid(inst->num_instances);
    return check_hip(pecc::launch_descend(inst->offset, inst->R, inst->R64, xy, inst->num_instances,
                                          inst->total_n, a, out, (int32_t *)workspace, grid,
                                          stream),
                     fn);
}

int pecc_lbfgs_descend_noalloc(const pecc_instances *inst, float *xy,
                               const pecc_descent_params *p, pecc_descent_result *out,
                               hipStream_t stream)
{
    const char *fn = "pecc_lbfgs_descend_noalloc";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (inst->num_instances > PECC_NOALLOC_MAX_INSTANCES)
        return fail(PECC_ERR_INVALID, "%s: %d instances exceed the limit of %d", fn,
                    inst->num_instances, PECC_NOALLOC_MAX_INSTANCES);
    if (!p || !out) return fail(PECC_ERR_INVALID, "%s: params and out must be set", fn);
    if (inst->total_n > 0 && !xy) return fail(PECC_ERR_INVALID, "%s: xy is NULL", fn);
    pecc::DescentArgs a;
    rc = descent_args(p, fn, &a);
    if (rc) return rc;
    const int grid = pecc::descend_grid(inst->num_instances);
    return check_hip(pecc::launch_descend_noalloc(inst->offset, inst->R, inst->R64, xy,
                                                  inst->num_instances, inst->total_n, a, out,
                                                  grid, stream),
                     fn);
}

int pecc_adjust_container_workspace_size(const pecc_instances *inst, size_t *bytes)
{
    return pecc_lbfgs_descend_workspace_size(inst, bytes);
}

int pecc_adjust_container(const pecc_instances *inst, float *xy, const pecc_descent_params *p,
                          float lambda0, int32_t rounds, float *R_out, pecc_descent_result *out,
                          void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    const char *fn = "pecc_adjust_container";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (!p || !out || !R_out) return fail(PECC_ERR_INVALID, "%s: params, out and R_out must be set", fn);
    if (inst->total_n > 0 && !xy) return fail(PECC_ERR_INVALID, "%s: xy is NULL", fn);
    if (!(lambda0 >= 0.f && lambda0 < 1e30f))
        return fail(PECC_ERR_INVALID, "%s: lambda0 must be finite and >= 0", fn);
    if (rounds < 0 || rounds > 64) return fail(PECC_ERR_INVALID, "%s: rounds outside [0, 64]", fn);
    pecc::DescentArgs a;
    rc = descent_args(p, fn, &a);
    if (rc) return rc;
    a.lambda0 = lambda0;
    a.rounds = rounds;
    size_t need = 0;
    pecc_lbfgs_descend_workspace_size(inst, &need);
    if (!workspace || workspace_bytes < need)
        return fail(PECC_ERR_WORKSPACE, "%s: workspace needs %zu bytes", fn, need);
    const int grid = pecc::descend_grid(inst->num_instances);
    return check_hip(pecc::launch_adjust(inst->offset, inst->R, xy, inst->num_instances,
                                         inst->total_n, a, R_out, out, (int32_t *)workspace, grid,
                                         stream),
                     fn);
}

int pecc_partition(const pecc_instances *inst, const float *xy, int32_t kind, int32_t k,
                   uint64_t seed, int32_t *batch_of, hipStream_t stream)
{
    const char *fn = "pecc_partition";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (kind < PECC_PARTITION_SECTOR || kind > PECC_PARTITION_RANDOM)
        return fail(PECC_ERR_INVALID, "%s: unknown kind %d", fn, kind);
    if (k < 1 || k > PECC_MAX_N) return fail(PECC_ERR_INVALID, "%s: k = %d outside [1, %d]", fn, k, PECC_MAX_N);
    if (inst->total_n > 0 && (!xy || !batch_of))
        return fail(PECC_ERR_INVALID, "%s: xy and batch_of must be set", fn);
    return check_hip(pecc::launch_partition(inst->offset, xy, inst->num_instances, inst->total_n,
                                            kind, k, seed, batch_of, stream),
                     fn);
}

int pecc_gbo_kbatch_descend_workspace_size(const pecc_instances *inst, size_t *bytes)
{
    return pecc_lbfgs_descend_workspace_size(inst, bytes);
}

int pecc_gbo_kbatch_descend(const pecc_instances *inst, float *xy, const int32_t *batch_of,
                            int32_t k, int32_t anm, const pecc_descent_params *p,
                            pecc_descent_result *out, void *workspace, size_t workspace_bytes,
                            hipStream_t stream)
{
    const char *fn = "pecc_gbo_kbatch_descend";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (!p || !out) return fail(PECC_ERR_INVALID, "%s: params and out must be set", fn);
    if (inst->total_n > 0 && (!xy || !batch_of))
        return fail(PECC_ERR_INVALID, "%s: xy and batch_of must be set", fn);
    if (k < 1 || k > PECC_MAX_BATCHES)
        return fail(PECC_ERR_INVALID, "%s: k = %d outside [1, %d]", fn, k, PECC_MAX_BATCHES);
    if (anm != 0 && anm != 1) return fail(PECC_ERR_INVALID, "%s: anm must be 0 or 1", fn);
    pecc::DescentArgs a;
    rc = descent_args(p, fn, &a);
    if (rc) return rc;
    a.nbat = k;
    a.anm = anm;
    size_t need = 0;
    pecc_lbfgs_descend_workspace_size(inst, &need);
    if (!workspace || workspace_bytes < need)
        return fail(PECC_ERR_WORKSPACE, "%s: workspace needs %zu bytes", fn, need);
    const int grid = pecc::descend_grid(inst->num_instances);
    return check_hip(pecc::launch_seq(inst->offset, inst->R, inst->R64, xy, inst->num_instances,
                                      inst->total_n, a, batch_of, out, (int32_t *)workspace, grid,
                                      stream),
                     fn);
}

namespace {
// floats of storage per instance for batches of at most max_batch circles:
// the matrices, d_p = 2|B_p| rows of d_p floats rounded up to a multiple of
// 4 (d_p <= 1024) or 64 (above), so sum_p d_p (d_p + pad) <= (2 max_batch
// + pad) sum_p d_p <= 4 max_batch max_n + 2 pad max_n with pad = 2 or 62,
// and four vectors of d_p floats per batch (8 max_n); rounded up to a
// multiple of 64 floats, so every instance's region starts on a 256-byte
// boundary like the workspace
int64_t dense_stride(const pecc_instances *inst, int32_t max_batch)
{
    const int64_t n = inst->max_n > 0 ? inst->max_n : 1;
    const int64_t pad = 2 * (int64_t)max_batch <= 1024 ? 2 : 62;
    return (4 * (int64_t)max_batch * n + (2 * pad + 8) * n + 63) & ~(int64_t)63;
}
}  // namespace

int pecc_gbo_kbatch_bfgs_workspace_size(const pecc_instances *inst, int32_t max_batch,
                                        size_t *bytes)
{
    const char *fn = "pecc_gbo_kbatch_bfgs_workspace_size";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (!bytes) return fail(PECC_ERR_INVALID, "%s: bytes is NULL", fn);
    if (max_batch < 1 || max_batch > PECC_MAX_N)
        return fail(PECC_ERR_INVALID, "%s: max_batch = %d outside [1, %d]", fn, max_batch, PECC_MAX_N);
    size_t q = 0;
    pecc_lbfgs_descend_workspace_size(inst, &q);
    *bytes = q + align256(sizeof(float) * (size_t)dense_stride(inst, max_batch) *
                          (size_t)inst->num_instances);
    return PECC_OK;
}

int pecc_gbo_kbatch_bfgs_descend(const pecc_instances *inst, float *xy, const int32_t *batch_of,
                                 int32_t k, int32_t anm, int32_t max_batch,
                                 const pecc_descent_params *p, pecc_descent_result *out,
                                 void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    const char *fn = "pecc_gbo_kbatch_bfgs_descend";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (!p || !out) return fail(PECC_ERR_INVALID, "%s: params and out must be set", fn);
    if (inst->total_n > 0 && (!xy || !batch_of))
        return fail(PECC_ERR_INVALID, "%s: xy and batch_of must be set", fn);
    if (k < 1 || k > PECC_MAX_BATCHES)
        return fail(PECC_ERR_INVALID, "%s: k = %d outside [1, %d]", fn, k, PECC_MAX_BATCHES);
    if (anm != 0 && anm != 1) return fail(PECC_ERR_INVALID, "%s: anm must be 0 or 1", fn);
    size_t need = 0;
    rc = pecc_gbo_kbatch_bfgs_workspace_size(inst, max_batch, &need);
    if (rc) return rc;
    if (!workspace || workspace_bytes < need)
        return fail(PECC_ERR_WORKSPACE, "%s: workspace needs %zu bytes", fn, need);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(PECC_ERR_WORKSPACE, "%s: workspace must be 256-byte aligned", fn);
    pecc::DescentArgs a;
    rc = descent_args(p, fn, &a);
    if (rc) return rc;
    a.nbat = k;
    a.anm = anm;
    a.hstride = dense_stride(inst, max_batch);
    size_t q = 0;
    pecc_lbfgs_descend_workspace_size(inst, &q);
    float *H = reinterpret_cast<float *>(static_cast<char *>(workspace) + q);
    const int grid = pecc::descend_grid(inst->num_instances);
    return check_hip(pecc::launch_dense(inst->offset, inst->R, inst->R64, xy, inst->num_instances,
                                        inst->total_n, a, batch_of, H, out, (int32_t *)workspace,
                                        grid, stream),
                     fn);
}

int pecc_gbo_descend_workspace_size(const pecc_instances *inst, int32_t blocks, size_t *bytes)
{
    const char *fn = "pecc_gbo_descend_workspace_size";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (!bytes) return fail(PECC_ERR_INVALID, "%s: bytes is NULL", fn);
    if (blocks < 1 || blocks > 8) return fail(PECC_ERR_INVALID, "%s: blocks = %d outside [1, 8]", fn, blocks);
    *bytes = align256(pecc::gbo_workspace_bytes(inst->num_instances, blocks) + 256);
    return PECC_OK;
}

int pecc_gbo_descend(const pecc_instances *inst, float *xy, const pecc_descent_params *p,
                     int32_t blocks, int32_t sweep_fp64, pecc_descent_result *out,
                     void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    const char *fn = "pecc_gbo_descend";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (!p || !out) return fail(PECC_ERR_INVALID, "%s: params and out must be set", fn);
    if (inst->total_n > 0 && !xy) return fail(PECC_ERR_INVALID, "%s: xy is NULL", fn);
    if (blocks < 1 || blocks > 8) return fail(PECC_ERR_INVALID, "%s: blocks = %d outside [1, 8]", fn, blocks);
    pecc::DescentArgs a;
    rc = descent_args(p, fn, &a);
    if (rc) return rc;
    size_t need = 0;
    pecc_gbo_descend_workspace_size(inst, blocks, &need);
    if (!workspace || workspace_bytes < need)
        return fail(PECC_ERR_WORKSPACE, "%s: workspace needs %zu bytes", fn, need);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(PECC_ERR_WORKSPACE, "%s: workspace must be 256-byte aligned", fn);
    return check_hip(pecc::launch_gbo(inst->offset, inst->R, inst->R64, xy, inst->num_instances,
                                      inst->total_n, a, blocks, sweep_fp64 ? 1 : 0, out, workspace,
                                      stream),
                     fn);
}

// ---------------------------------------------------------------------------
int pecc_verify(const pecc_instances *inst, const float *xy, double tol, double *energy64,
                double *max_pair_overlap, double *max_cont_overlap, int32_t *feasible,
                hipStream_t stream)
{
    const char *fn = "pecc_verify";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (!energy64) return fail(PECC_ERR_INVALID, "%s: energy64 is NULL", fn);
    if (inst->total_n > 0 && !xy) return fail(PECC_ERR_INVALID, "%s: xy is NULL", fn);
    return check_hip(pecc::launch_verify(inst->offset, inst->R, inst->R64, xy,
                                         inst->num_instances, inst->total_n, tol, energy64,
                                         max_pair_overlap, max_cont_overlap, feasible, stream),
                     fn);
}

int pecc_verify_tighten(const pecc_instances *inst, const float *xy, double tol, float *R_out,
                        int32_t *feasible, hipStream_t stream)
{
    const char *fn = "pecc_verify_tighten";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (!R_out || !feasible) return fail(PECC_ERR_INVALID, "%s: R_out and feasible must be set", fn);
    if (inst->total_n > 0 && !xy) return fail(PECC_ERR_INVALID, "%s: xy is NULL", fn);
    return check_hip(pecc::launch_verify_tighten(inst->offset, inst->R, inst->R64, xy,
                                                 inst->num_instances, inst->total_n, tol, R_out,
                                                 feasible, stream),
                     fn);
}

// ---------------------------------------------------------------------------
// Learned proposal
// ---------------------------------------------------------------------------
int pecc_features(const pecc_instances *inst, const float *xy, int32_t cands_per_inst,
                  const int32_t *cand_circle, const float *cand_dest, float *features,
                  hipStream_t stream)
{
    const char *fn = "pecc_features";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (cands_per_inst < 0) return fail(PECC_ERR_INVALID, "%s: cands_per_inst < 0", fn);
    if (cands_per_inst == 0) return PECC_OK;
    if ((int64_t)cands_per_inst * inst->num_instances > 0x7fffffffLL)
        return fail(PECC_ERR_INVALID, "%s: more than 2^31-1 candidates", fn);
    if (!xy || !cand_circle || !cand_dest || !features)
        return fail(PECC_ERR_INVALID, "%s: xy, cand_circle, cand_dest and features must be set",
                    fn);
    return check_hip(pecc::launch_features(inst->offset, inst->R, inst->R64, xy,
                                           inst->num_instances, cands_per_inst, cand_circle,
                                           cand_dest, features, stream),
                     fn);
}

int pecc_mlp_forward(const float *params, const float *features, int64_t rows, float *logits,
                     hipStream_t stream)
{
    const char *fn = "pecc_mlp_forward";
    if (rows < 0) return fail(PECC_ERR_INVALID, "%s: rows < 0", fn);
    if (rows == 0) return PECC_OK;
    if (!params || !features || !logits)
        return fail(PECC_ERR_INVALID, "%s: params, features and logits must be set", fn);
    return check_hip(pecc::launch_mlp_forward(params, features, rows, logits, stream), fn);
}

int pecc_mlp_grad_workspace_size(int64_t rows, size_t *bytes)
{
    if (rows < 0 || !bytes) return fail(PECC_ERR_INVALID, "pecc_mlp_grad_workspace_size: bad arguments");
    *bytes = align256(pecc::mlp_grad_workspace_bytes(rows));
    return PECC_OK;
}

static int mlp_grad_checks(const char *fn, const float *params, const float *features,
                           const float *labels, int64_t rows, const float *grad, const void *ws,
                           size_t ws_bytes)
{
    if (rows < 0) return fail(PECC_ERR_INVALID, "%s: rows < 0", fn);
    if (!params || !grad) return fail(PECC_ERR_INVALID, "%s: params and grad must be set", fn);
    if (rows > 0 && (!features || !labels))
        return fail(PECC_ERR_INVALID, "%s: features and labels must be set", fn);
    const size_t need = align256(pecc::mlp_grad_workspace_bytes(rows));
    if (!ws || ws_bytes < need)
        return fail(PECC_ERR_WORKSPACE, "%s: workspace needs %zu bytes", fn, need);
    return PECC_OK;
}

int pecc_mlp_grad(const float *params, const float *features, const float *labels, int64_t rows,
                  float *loss, float *grad, void *ws, size_t ws_bytes, hipStream_t stream)
{
    const char *fn = "pecc_mlp_grad";
    int rc = mlp_grad_checks(fn, params, features, labels, rows, grad, ws, ws_bytes);
    if (rc) return rc;
    return check_hip(pecc::launch_mlp_grad(params, features, labels, rows, loss, grad, ws, stream),
                     fn);
}

static int adam_checks(const char *fn, const float *params, const float *m, const float *v,
                       const float *grad, const int32_t *step, const pecc_adam_params *hp,
                       pecc::AdamArgs *a)
{
    if (!params || !m || !v || !grad || !step || !hp)
        return fail(PECC_ERR_INVALID, "%s: params, m, v, grad, step and hp must be set", fn);
    if (!(hp->lr >= 0.0f) || !(hp->beta1 >= 0.0f && hp->beta1 < 1.0f) ||
        !(hp->beta2 >= 0.0f && hp->beta2 < 1.0f) || !(hp->eps > 0.0f))
        return fail(PECC_ERR_INVALID, "%s: need lr >= 0, 0 <= beta < 1, eps > 0", fn);
    *a = pecc::AdamArgs{hp->lr, hp->beta1, hp->beta2, hp->eps};
    return PECC_OK;
}

int pecc_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t *step,
                  const pecc_adam_params *hp, hipStream_t stream)
{
    const char *fn = "pecc_mlp_adam";
    pecc::AdamArgs a;
    int rc = adam_checks(fn, params, m, v, grad, step, hp, &a);
    if (rc) return rc;
    return check_hip(pecc::launch_adam(params, m, v, grad, step, a, stream), fn);
}

int pecc_mlp_train_step(float *params, float *m, float *v, int32_t *step,
                        const pecc_adam_params *hp, const float *features, const float *labels,
                        int64_t rows, float *loss, float *grad, void *ws, size_t ws_bytes,
                        hipStream_t stream)
{
    const char *fn = "pecc_mlp_train_step";
    int rc = mlp_grad_checks(fn, params, features, labels, rows, grad, ws, ws_bytes);
    if (rc) return rc;
    pecc::AdamArgs a;
    rc = adam_checks(fn, params, m, v, grad, step, hp, &a);
    if (rc) return rc;
    rc = check_hip(pecc::launch_mlp_grad(params, features, labels, rows, loss, grad, ws, stream),
                   fn);
    if (rc) return rc;
    return check_hip(pecc::launch_adam(params, m, v, grad, step, a, stream), fn);
}

int pecc_propose(const pecc_instances *inst, const float *xy, int32_t cands_per_inst,
                 const int32_t *cand_circle, const float *cand_dest, const float *scores,
                 int32_t k, int32_t *selected, float *xy_out, hipStream_t stream)
{
    const char *fn = "pecc_propose";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (cands_per_inst < 0 || k < 0)
        return fail(PECC_ERR_INVALID, "%s: cands_per_inst and k must be >= 0", fn);
    if ((int64_t)cands_per_inst * inst->num_instances > 0x7fffffffLL)
        return fail(PECC_ERR_INVALID, "%s: more than 2^31-1 candidates", fn);
    if (inst->total_n > 0 && (!xy || !xy_out))
        return fail(PECC_ERR_INVALID, "%s: xy and xy_out must be set", fn);
    if (cands_per_inst > 0 && (!cand_circle || !cand_dest))
        return fail(PECC_ERR_INVALID, "%s: cand_circle and cand_dest must be set", fn);
    return check_hip(pecc::launch_propose(inst->offset, xy, inst->num_instances, cands_per_inst,
                                          cand_circle, cand_dest, scores, k, selected, xy_out,
                                          stream),
                     fn);
}

int pecc_accept(const pecc_instances *inst, float *xy_cur, double *e_cur, const float *xy_new,
                const double *e_new, int32_t *accepted, hipStream_t stream)
{
    const char *fn = "pecc_accept";
    int rc = check_inst(inst, fn);
    if (rc) return rc;
    if (!e_cur || !e_new) return fail(PECC_ERR_INVALID, "%s: e_cur and e_new must be set", fn);
    if (inst->total_n > 0 && (!xy_cur || !xy_new))
        return fail(PECC_ERR_INVALID, "%s: xy_cur and xy_new must be set", fn);
    return check_hip(pecc::launch_accept(inst->offset, xy_cur, e_cur, xy_new, e_new,
                                         inst->num_instances, accepted, stream),
                     fn);
}

// ---------------------------------------------------------------------------
// SED (Alg. 5)
// ---------------------------------------------------------------------------
static int sed_checks(const char *fn, const pecc_instances *chains, int32_t M)
{
    int rc = check_inst(chains, fn);
    if (rc) return rc;
    if (M < 1 || M > PECC_SED_MAX_CAND)
        return fail(PECC_ERR_INVALID, "%s: M = %d outside [1, %d]", fn, M, PECC_SED_MAX_CAND);
    if ((int64_t)chains->num_instances * M > (1 << 24))
        return fail(PECC_ERR_INVALID, "%s: chains x M above 2^24", fn);
    return PECC_OK;
}

int pecc_sed_plan(const pecc_instances *chains, const double *E_cur, const double *E_best,
                  int32_t M, double e_stop, int32_t *m, int32_t *cand_offset, float *cand_R,
                  double *cand_R64, hipStream_t stream)
{
    const char *fn = "pecc_sed_plan";
    int rc = sed_checks(fn, chains, M);
    if (rc) return rc;
    if (!E_cur || !E_best || !m || !cand_offset || !cand_R || !cand_R64)
        return fail(PECC_ERR_INVALID, "%s: every array must be set", fn);
    return check_hip(pecc::launch_sed_plan(chains->offset, chains->R, chains->R64,
                                           chains->num_instances, M, E_cur, E_best, e_stop, m,
                                           cand_offset, cand_R, cand_R64, stream),
                     fn);
}

int pecc_sed_perturb(const pecc_instances *chains, const float *xy, int32_t M, const int32_t *m,
                     const int32_t *cand_offset, uint64_t seed, int32_t iter, float *cand_xy,
                     hipStream_t stream)
{
    const char *fn = "pecc_sed_perturb";
    int rc = sed_checks(fn, chains, M);
    if (rc) return rc;
    if (iter < 0) return fail(PECC_ERR_INVALID, "%s: iter < 0", fn);
    if (!m || !cand_offset || !cand_xy || (chains->total_n > 0 && !xy))
        return fail(PECC_ERR_INVALID, "%s: every array must be set", fn);
    return check_hip(pecc::launch_sed_perturb(chains->offset, xy, chains->num_instances, M, m,
                                              cand_offset, seed, iter, cand_xy, stream),
                     fn);
}

int pecc_sed_select(const pecc_instances *chains, int32_t M, const int32_t *m,
                    const int32_t *cand_offset, const float *cand_xy, const double *cand_E,
                    uint64_t seed, int32_t iter, float *xy_cur, double *E_cur, float *xy_best,
                    double *E_best, int32_t *chosen, hipStream_t stream)
{
    const char *fn = "pecc_sed_select";
    int rc = sed_checks(fn, chains, M);
    if (rc) return rc;
    if (iter < 0) return fail(PECC_ERR_INVALID, "%s: iter < 0", fn);
    if (!m || !cand_offset || !cand_E || !E_cur || !E_best ||
        (chains->total_n > 0 && (!cand_xy || !xy_cur || !xy_best)))
        return fail(PECC_ERR_INVALID, "%s: every array must be set", fn);
    return check_hip(pecc::launch_sed_select(chains->offset, chains->num_instances, M, m,
                                             cand_offset, cand_xy, cand_E, seed, iter, xy_cur,
                                             E_cur, xy_best, E_best, chosen, stream),
                     fn);
}

}  // extern "C"

static_assert(sizeof(pecc_descent_result) == 48, "result layout");
static_assert(sizeof(pecc_descent_params) == 64, "params layout");
static_assert(PECC_MAX_BATCHES == pecc::kMaxSeqBatches, "batch limit");
static_assert(PECC_NOALLOC_MAX_INSTANCES == pecc::kNoAllocMaxInstances, "no-alloc limit");
static_assert(PECC_LIST_HALF == pecc::kListHalf && PECC_LIST_FULL == pecc::kListFull &&
              PECC_LIST_LOCAL16 == pecc::kListLocal16, "list forms");
static_assert(sizeof(pecc_adam_params) == 16, "adam params layout");
