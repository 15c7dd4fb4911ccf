// Host-side launchers of the library's kernels (called by the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pecc {

// Neighbor-list forms (the values of PECC_LIST_*): int32 global indices
// with each pair once or in both orientations, uint16 instance-local
// indices in both orientations.
constexpr int kListHalf = 0, kListFull = 1, kListLocal16 = 2;

hipError_t launch_build(const int32_t *offset, const float *R, const float *xy, int B,
                        int64_t total_n, double cutoff, float h_req, int format,
                        int32_t *row, void *col, int64_t capacity, int64_t *num_pairs,
                        int64_t *inst_total, hipStream_t s);

hipError_t launch_energy_grad(const int32_t *offset, const float *R, const float *xy, int B,
                              int64_t total_n, const int32_t *row, const void *col,
                              int64_t col_len, int format, float rad, float *energy, float *grad,
                              hipStream_t s);

hipError_t launch_verify(const int32_t *offset, const float *R, const double *R64,
                         const float *xy, int B, int64_t total_n, double tol, double *e64,
                         double *mp, double *mc, int32_t *feas, hipStream_t s);
hipError_t launch_verify_tighten(const int32_t *offset, const float *R, const double *R64,
                                 const float *xy, int B, int64_t total_n, double tol,
                                 float *R_out, int32_t *feas, hipStream_t s);

// Descent constants as the kernels use them (derived from the public params).
struct DescentArgs {
    int m, max_iter, max_halvings, ftol_window;
    float c1, eps_curv, h_req, g_tol, ftol, rad;
    float g_tol_sq;   // largest x with sqrtf(x) <= g_tol: the gradient test without a square root
    double c2, skin2, e_feasible, tau64;
    float lambda0;    // container adjustment: first penalty coefficient
    int rounds;       // container adjustment: minimisations, lambda halved after each
    int nbat;         // batch descent: batches of the partition (1..kMaxSeqBatches)
    int anm;          // batch descent: 1 = adaptive neighbor maintenance (Alg. 3)
    int64_t hstride;  // dense batch descent: floats of matrix storage per instance
};

constexpr int kMaxSeqBatches = 16;   // batches of the batch descent at most

struct DescentResultDev;  // layout-identical to pecc_descent_result

hipError_t launch_descend(const int32_t *offset, const float *R, const double *R64, float *xy,
                          int B, int64_t total_n, const DescentArgs &a, void *out,
                          int32_t *queue, int grid, hipStream_t s);

int descend_grid(int B);   // persistent workgroups to launch for B instances

// The same descent with its work queue in a library-held array (no
// allocation anywhere): at most kNoAllocMaxInstances instances.
constexpr int kNoAllocMaxInstances = 65536;
hipError_t launch_descend_noalloc(const int32_t *offset, const float *R, const double *R64,
                                  float *xy, int B, int64_t total_n, const DescentArgs &a,
                                  void *out, int grid, hipStream_t s);

// Container adjustment: the descent with the radius as a variable (Rout[B]
// receives the final radii; the initial ones come from R).
hipError_t launch_adjust(const int32_t *offset, const float *R, float *xy, int B,
                         int64_t total_n, const DescentArgs &a, float *Rout, void *out,
                         int32_t *queue, int grid, hipStream_t s);

// Batch descent of Alg. 1 over a given partition (batch_of: global circle
// index -> batch in [0, a.nbat)), batches visited in order.
hipError_t launch_seq(const int32_t *offset, const float *R, const double *R64, float *xy, int B,
                      int64_t total_n, const DescentArgs &a, const int32_t *batch_of, void *out,
                      int32_t *queue, int grid, hipStream_t s);

// Dense batch descent (the paper's per-batch inverse-Hessian matrices,
// Eq. 8-11): H holds a.hstride floats per instance.
hipError_t launch_dense(const int32_t *offset, const float *R, const double *R64, float *xy,
                        int B, int64_t total_n, const DescentArgs &a, const int32_t *batch_of,
                        float *H, void *out, int32_t *queue, int grid, hipStream_t s);

// k-batch partitions of Sec. 4.1 (kind: 0 sector, 1 annulus, 2 fence, 3 random).
hipError_t launch_partition(const int32_t *offset, const float *xy, int B, int64_t total_n,
                            int kind, int k, uint64_t seed, int32_t *batch_of, hipStream_t s);

// Geometric batch descent: workspace bytes and launch.
size_t gbo_workspace_bytes(int B, int blocks);
hipError_t launch_gbo(const int32_t *offset, const float *R, const double *R64, float *xy, int B,
                      int64_t total_n, const DescentArgs &a, int blocks, int sweep_fp64, void *out,
                      void *ws, hipStream_t s);

// Learned proposal: features, network forward / gradient, Adam, proposal, acceptance.
hipError_t launch_features(const int32_t *offset, const float *R, const double *R64,
                           const float *xy, int B, int C, const int32_t *cand_circle,
                           const float *cand_dest, float *feat, hipStream_t s);
hipError_t launch_mlp_forward(const float *params, const float *X, int64_t rows, float *Z,
                              hipStream_t s);
size_t mlp_grad_workspace_bytes(int64_t rows);
hipError_t launch_mlp_grad(const float *params, const float *X, const float *Y, int64_t rows,
                           float *loss, float *grad, void *ws, hipStream_t s);
struct AdamArgs {
    float lr, b1, b2, eps;
};
hipError_t launch_adam(float *params, float *m, float *v, const float *grad, int32_t *step,
                       const AdamArgs &a, hipStream_t s);
hipError_t launch_propose(const int32_t *offset, const float *xy, int B, int C,
                          const int32_t *cand_circle, const float *cand_dest, const float *scores,
                          int k, int32_t *selected, float *xy_out, hipStream_t s);
hipError_t launch_accept(const int32_t *offset, float *xy_cur, double *e_cur, const float *xy_new,
                         const double *e_new, int B, int32_t *accepted, hipStream_t s);

// SED (Alg. 5) over chains: plan, perturbation, selection.
hipError_t launch_sed_plan(const int32_t *offset, const float *R, const double *R64, int B, int M,
                           const double *E_cur, const double *E_best, double e_stop,
                           int32_t *m_out, int32_t *cand_offset, float *cand_R, double *cand_R64,
                           hipStream_t s);
hipError_t launch_sed_perturb(const int32_t *offset, const float *xy, int B, int M,
                              const int32_t *m, const int32_t *cand_offset, uint64_t seed,
                              int iter, float *cand_xy, hipStream_t s);
hipError_t launch_sed_select(const int32_t *offset, int B, int M, const int32_t *m,
                             const int32_t *cand_offset, const float *cand_xy,
                             const double *cand_E, uint64_t seed, int iter, float *xy_cur,
                             double *E_cur, float *xy_best, double *E_best, int32_t *chosen,
                             hipStream_t s);

}  // namespace pecc
