// Persistent L-BFGS descent of the elastic energy at fixed container radius.
//
// Mapping (one workgroup of 512 threads per instance, n <= 1024):
//   * thread t owns circles t and t + 512: their positions, gradients, search
//     directions and their coordinates of every stored curvature pair
//     (s_j, y_j) live in registers, so the L-BFGS history never leaves the
//     chip (two circles per thread leave a 256-register budget, enough for
//     the 80 history registers without spilling);
//   * positions of the instance sit in LDS (the pair sweep reads them), next
//     to the cell grid and a CSR neighbor list of 16-bit local indices;
//   * the inverse-Hessian product is formed without per-vector dot products
//     (vector-free two-loop): every wave keeps the Gram matrix B of the basis
//     {s_0..s_{m-1}, y_0..y_{m-1}, g} (double-buffered in LDS), runs the
//     two-loop recursion on B's entries with lanes as columns and obtains the
//     direction as a combination of the basis.  All new entries of B come
//     from ONE fused reduction per line-search trial (63 dot products plus
//     the energy), so a trial costs two workgroup barriers.
// Workgroups take instances from a queue, largest n first, until the queue
// is empty (the launch is sized to the resident capacity of the device).
#include "pecc_device.hpp"
#include "pecc_launch.hpp"

namespace pecc {

constexpr int kDB = 512;                  // threads per workgroup
constexpr int kDW = kDB / kWave;          // waves per workgroup
constexpr int kCPT = kMaxN / kDB;         // circles per thread
constexpr int kMM = 10;                   // history slots (max m)
constexpr int kNB = 2 * kMM + 1;          // basis size: s_0..s_9, y_0..y_9, g
constexpr int kEll = 24;                  // neighbor slots per circle (ELL list)
constexpr int kG = 2 * kMM;               // basis index of g

// Slots of the fused reduction.  gt: trial gradient, sc = xt - x, yc = gt - g.
constexpr int sGS(int j) { return j; }                      // gt . s_j
constexpr int sGY(int j) { return kMM + j; }                // gt . y_j
constexpr int sSS(int j) { return 2 * kMM + j - 1; }        // sc . s_j   (j >= 1)
constexpr int sSY(int j) { return 3 * kMM - 1 + j - 1; }    // sc . y_j   (j >= 1)
constexpr int sYS(int j) { return 4 * kMM - 2 + j - 1; }    // yc . s_j   (j >= 1)
constexpr int sYY(int j) { return 5 * kMM - 3 + j - 1; }    // yc . y_j   (j >= 1)
constexpr int sGG = 6 * kMM - 4;                            // gt . gt
constexpr int sScSc = sGG + 1;                              // sc . sc
constexpr int sScYc = sGG + 2;                              // sc . yc
constexpr int sYcYc = sGG + 3;                              // yc . yc
constexpr int sScG = sGG + 4;                               // sc . gt
constexpr int sYcG = sGG + 5;                               // yc . gt
constexpr int sE = sGG + 6;                                 // trial energy (radius rad)
constexpr int sE1 = sGG + 7;                                // trial energy of unit circles
static_assert(sE1 < kWave, "fused reduction must fit one slot per lane");

struct DescentShared {
    float2 pos[kMaxN];
    int cell_start[kMaxCells + 1];
    uint16_t cell_circ[kMaxN];
    uint16_t slot_tmp[kMaxN];
    uint16_t list[kEll][kMaxN];    // slot-major: lanes read consecutive entries
    uint8_t  list_n[kMaxN];
    float red[2][kDW][kWave];
    double red64[2][kDW][2];
    float Bm[2][kNB * kNB];
    float tot_s[2][kWave];
    uint16_t bsrc[2][kNB * kNB];   // Gram update sources, see gram_source
    int scan_tmp[kDW + 1];
    int flag[2];
    int over;                      // a circle had more than kEll neighbors
    int work;
};

// Layout-identical mirror of pecc_descent_result.
struct DescentResultDev {
    int32_t status, iters, evals, rebuilds;
    int64_t pair_evals;
    float E32, gnorm;
    double E64;
};

__device__ __forceinline__ float dot2(float2 a, float2 b) { return a.x * b.x + a.y * b.y; }

// Value of reduction slot v summed over this thread's circles (v is a
// constant after unrolling, so the branches fold away).
__device__ __forceinline__ float slot_value(int v, const float2 (&gt)[kCPT], const float2 (&sc)[kCPT],
                                            const float2 (&yc)[kCPT],
                                            const float2 (&S)[kMM][kCPT],
                                            const float2 (&Y)[kMM][kCPT], float e, float e1)
{
    if (v == sE) return e;
    if (v == sE1) return e1;
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < kCPT; ++c) {
        float t;
        if (v < kMM) t = dot2(gt[c], S[v][c]);
        else if (v < 2 * kMM) t = dot2(gt[c], Y[v - kMM][c]);
        else if (v < 3 * kMM - 1) t = dot2(sc[c], S[v - 2 * kMM + 1][c]);
        else if (v < 4 * kMM - 2) t = dot2(sc[c], Y[v - (3 * kMM - 1) + 1][c]);
        else if (v < 5 * kMM - 3) t = dot2(yc[c], S[v - (4 * kMM - 2) + 1][c]);
        else if (v < 6 * kMM - 4) t = dot2(yc[c], Y[v - (5 * kMM - 3) + 1][c]);
        else if (v == sGG) t = dot2(gt[c], gt[c]);
        else if (v == sScSc) t = dot2(sc[c], sc[c]);
        else if (v == sScYc) t = dot2(sc[c], yc[c]);
        else if (v == sYcYc) t = dot2(yc[c], yc[c]);
        else if (v == sScG) t = dot2(sc[c], gt[c]);
        else t = dot2(yc[c], gt[c]);   // sYcG
        acc += t;
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Cross-lane moves.  DPP (data-parallel primitives) patterns run at VALU
// rate; quad_perm and the row mirrors stay inside 16-lane rows, row_bcast
// crosses rows.  Lane builtins work on 32-bit integers, so floats travel as
// bit patterns.
// ---------------------------------------------------------------------------
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppRowMirror = 0x140;  // lane i <- 15-i inside a row
constexpr int kDppHalfMirror = 0x141; // lane i <- 7-i inside half a row
constexpr int kDppBcast15 = 0x142;    // lane 15 of row r -> row r+1
constexpr int kDppBcast31 = 0x143;    // lane 31 -> rows 2 and 3

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 CTRL, ROW_MASK, 0xf, false));
}

__device__ __forceinline__ float uniform_first(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float lane_value(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Sum over the 64 lanes, returned wave-uniform.  Every wave adds in the same
// order, so every wave gets the same bits.
__device__ __forceinline__ float wave_sum_dpp(float v)
{
    v += dpp<kDppXor1>(v);
    v += dpp<kDppXor2>(v);
    v += dpp<kDppHalfMirror>(v);
    v += dpp<kDppRowMirror>(v);          // every lane of a row holds the row sum
    v += dpp<kDppBcast15, 0xa>(v);       // rows 1, 3 add rows 0, 2
    v += dpp<kDppBcast31, 0xc>(v);       // rows 2, 3 add lane 31 (rows 0 + 1)
    return lane_value(v, 63);
}

// Slot held by lane L after wave_reduce_scatter (stages decided by lane bits
// 3, 2, 1, 0, 4, 5 in this order).
__device__ __forceinline__ int lane_slot(int L)
{
    return 32 * ((L >> 3) & 1) + 16 * ((L >> 2) & 1) + 8 * ((L >> 1) & 1) + 4 * (L & 1) +
           2 * ((L >> 4) & 1) + ((L >> 5) & 1);
}

// Reduce-scatter of the 64 slot values over the wave: afterwards lane L
// holds the wave sum of slot lane_slot(L).  Each stage pairs a lane with a
// partner holding the same slot subset; the lane whose deciding bit is set
// keeps the upper half.  Partners: stage 1 row mirror (bit 3), stage 2 half
// mirror (bit 2), stage 3 xor 2, stage 4 xor 1 (all DPP), stage 5 xor 16,
// stage 6 xor 32 (shuffles).  Slots are produced in the order the first three
// stages consume them (u, u+8, ..., u+56) so only 8 values are live at once.
__device__ __forceinline__ float wave_reduce_scatter(const float2 (&gt)[kCPT],
                                                     const float2 (&sc)[kCPT],
                                                     const float2 (&yc)[kCPT],
                                                     const float2 (&S)[kMM][kCPT],
                                                     const float2 (&Y)[kMM][kCPT], float e,
                                                     float e1)
{
    const int lane = threadIdx.x & (kWave - 1);
    const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0, b1 = (lane & 2) != 0;
    const bool b0 = (lane & 1) != 0, b4 = (lane & 16) != 0, b5 = (lane & 32) != 0;
    float h[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        float t1[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float lo = slot_value(u + 8 * k, gt, sc, yc, S, Y, e, e1);
            const float hi = slot_value(u + 8 * k + 32, gt, sc, yc, S, Y, e, e1);
            t1[k] = (b3 ? hi : lo) + dpp<kDppRowMirror>(b3 ? lo : hi);
        }
        float t2[2];
#pragma unroll
        for (int k = 0; k < 2; ++k)
            t2[k] = (b2 ? t1[k + 2] : t1[k]) + dpp<kDppHalfMirror>(b2 ? t1[k] : t1[k + 2]);
        h[u] = (b1 ? t2[1] : t2[0]) + dpp<kDppXor2>(b1 ? t2[0] : t2[1]);
        // keep the streaming order: the next group is not hoisted above here
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) h[v] = (b0 ? h[v + 4] : h[v]) + dpp<kDppXor1>(b0 ? h[v] : h[v + 4]);
#pragma unroll
    for (int v = 0; v < 2; ++v) h[v] = (b4 ? h[v + 2] : h[v]) + __shfl_xor(b4 ? h[v] : h[v + 2], 16, kWave);
    return (b5 ? h[1] : h[0]) + __shfl_xor(b5 ? h[0] : h[1], 32, kWave);
}

// Which vector basis index a of the updated basis is: 0 = an old basis
// vector (index in *old), 1 = sc, 2 = yc, 3 = gt.
__device__ __forceinline__ int new_basis_kind(int a, bool push, int *old)
{
    if (a == kG) return 3;
    if (push) {
        if (a < kMM) {
            if (a == kMM - 1) return 1;
            *old = a + 1;
            return 0;
        }
        if (a == 2 * kMM - 1) return 2;
        *old = a + 1;
        return 0;
    }
    *old = a;
    return 0;
}

// Slot holding <kind-vector, old basis vector o>, kind in {1,2,3}.
__device__ __forceinline__ int slot_new_old(int kind, int o)
{
    const bool is_s = o < kMM;
    const int j = is_s ? o : o - kMM;
    if (kind == 3) return is_s ? sGS(j) : sGY(j);
    if (kind == 1) return is_s ? sSS(j) : sSY(j);
    return is_s ? sYS(j) : sYY(j);
}

__device__ __forceinline__ int slot_new_new(int ka, int kb)
{
    if (ka > kb) { const int t = ka; ka = kb; kb = t; }
    if (ka == 1 && kb == 1) return sScSc;
    if (ka == 1 && kb == 2) return sScYc;
    if (ka == 2 && kb == 2) return sYcYc;
    if (ka == 1 && kb == 3) return sScG;
    if (ka == 2 && kb == 3) return sYcG;
    return sGG;
}

// Where entry ent = a * kNB + l of the updated Gram matrix comes from:
// an old entry (index < 0x8000) or a reduction slot (0x8000 + slot).
__device__ __forceinline__ uint16_t gram_source(int ent, bool push)
{
    const int a = ent / kNB, l = ent - a * kNB;
    int oa = 0, ol = 0;
    const int ka = new_basis_kind(a, push, &oa);
    const int kl = new_basis_kind(l, push, &ol);
    if (ka == 0 && kl == 0) return (uint16_t)(oa * kNB + ol);
    int sl;
    if (ka == 0) sl = slot_new_old(kl, oa);
    else if (kl == 0) sl = slot_new_old(ka, ol);
    else sl = slot_new_new(ka, kl);
    return (uint16_t)(0x8000 + sl);
}

// FP64 neighbor predicate with an FP32 pre-test.  FP32 evaluation of
// dx*dx + dy*dy carries a relative error below 3e-7, so outside a band of
// +-1e-5 around c2 its answer is the FP64 one; inside the band the FP64
// predicate itself decides.  Same pair set as near64, fewer FP64 ops.
__device__ __forceinline__ bool near_cut(float2 a, float2 b, float c2lo, float c2hi, double c2)
{
    const float dx = a.x - b.x, dy = a.y - b.y;
    const float l2 = dx * dx + dy * dy;
    if (l2 < c2lo) return true;
    if (l2 > c2hi) return false;
    return near64(a, b, c2);
}

// FP32 pair term of circle i (at q) with circle j (at pj): energy on the
// i < j side only, gradient of circle i always.  Branch-free (selects only):
// non-overlapping pairs give d = 0, coincident centres d = 2 rad with no
// gradient.  (With branches the compiler merges the accumulations into one
// store through a selected address and moves the accumulators to memory.)
__device__ __forceinline__ void pair_term32(float2 q, float2 pj, bool count_e, float two_r,
                                            float four_r2, float &e, float &e1, float &gx,
                                            float &gy)
{
    const float dx = q.x - pj.x, dy = q.y - pj.y;
    const float l2 = dx * dx + dy * dy;
    const bool ov = l2 < four_r2;
    const float il = (ov && l2 > 0.f) ? __builtin_amdgcn_rsqf(l2) : 0.f;
    const float d = ov ? two_r - l2 * il : 0.f;
    // the same pair for unit circles (rad <= the descent's radius): overlap
    // 2 - l, which is d - (two_r - 2) whenever it is positive
    const float d1 = fmaxf(d - (two_r - 2.f), 0.f);
    e += count_e ? d * d : 0.f;
    e1 += count_e ? d1 * d1 : 0.f;
    const float kf = -2.f * d * il;
    gx += kf * dx;
    gy += kf * dy;
}

// FP64 pair energies (descent objective, unit circles) of a pair i < j.
__device__ __forceinline__ void pair_term64(float2 q, float2 pj, double two_r64, double four_r2_64,
                                            double &eo, double &et)
{
    const double ex = (double)q.x - (double)pj.x, ey = (double)q.y - (double)pj.y;
    const double m2 = ex * ex + ey * ey;
    if (m2 < four_r2_64) {
        const double l = sqrt(m2);
        const double d = two_r64 - l;
        const double dt = m2 < 4.0 ? 2.0 - l : 0.0;
        eo += d * d;
        et += dt * dt;
    }
}

// Evaluation requests of the descent's state machine.
enum : int { kReqInit = 0, kReqFp64 = 1, kReqTrial = 2 };

__global__ __launch_bounds__(kDB) void lbfgs_descend_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ Rv,
    const double *__restrict__ Rv64, float *__restrict__ xy,
    int B, int64_t total_n, DescentArgs A, DescentResultDev *__restrict__ out,
    int32_t *__restrict__ queue)
{
    __shared__ DescentShared sh;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    for (int q = tid; q < 2 * kNB * kNB; q += kDB)
        sh.bsrc[q / (kNB * kNB)][q % (kNB * kNB)] = gram_source(q % (kNB * kNB), q >= kNB * kNB);
    const float c2lo = (float)(A.c2 * (1.0 - 1e-5)), c2hi = (float)(A.c2 * (1.0 + 1e-5));

    for (;;) {
        // ---- next instance from the queue ------------------------------------
        __syncthreads();
        if (tid == 0) sh.work = atomicAdd(&queue[0], 1);
        __syncthreads();
        const int slot = sh.work;
        if (slot >= B) break;
        const int b = queue[1 + slot];
        const int off = offset[b], n = offset[b + 1] - off;
        if (!(off >= 0 && n >= 0 && n <= kMaxN && (int64_t)off + n <= total_n)) {
            if (tid == 0) {
                DescentResultDev r = {};
                r.status = 7;  // BAD_INSTANCE
                r.E32 = __builtin_nanf("");
                r.gnorm = __builtin_nanf("");
                r.E64 = -1.0;
                out[b] = r;
            }
            continue;
        }
        const float R = Rv[b];
        const float rad = A.rad, two_r = 2.0f * rad, four_r2 = two_r * two_r;
        const float four_r2_band = four_r2 * (1.0f + 1e-5f);
        const double rad64 = (double)rad, two_r64 = 2.0 * rad64, four_r2_64 = two_r64 * two_r64;
        // FP64 decisions (feasibility, the near-zero line search) use the
        // caller's FP64 radius when there is one, as pecc_verify does
        const double R64 = Rv64 ? Rv64[b] : (double)R;
        const Grid grid = make_grid(R, A.h_req);

        // ---- per-thread state (circle c of this thread is tid + c*kDB) ----
        bool act[kCPT];
        float2 x[kCPT], g[kCPT], xr[kCPT], p[kCPT];
        float2 S[kMM][kCPT], Y[kMM][kCPT];      // curvature pairs, newest at kMM-1
#pragma unroll
        for (int c = 0; c < kCPT; ++c) {
            const int i = tid + c * kDB;
            act[c] = i < n;
            x[c] = act[c] ? reinterpret_cast<const float2 *>(xy)[off + i] : make_float2(0.f, 0.f);
            g[c] = make_float2(0.f, 0.f);
            xr[c] = x[c];
            p[c] = make_float2(0.f, 0.f);
#pragma unroll
            for (int j = 0; j < kMM; ++j) { S[j][c] = make_float2(0.f, 0.f); Y[j][c] = make_float2(0.f, 0.f); }
        }
        // ---- uniform state ---------------------------------------------------
        int k = 0;                     // valid pairs, slots kMM-k .. kMM-1
        int cur = 0;                   // Bm buffer in use
        int tcount = 0;                // evaluations so far (flag parity)
        bool overflow = false;         // list did not fit: sweep the cell grid
        int half_mine[kCPT] = {};      // listed pairs i<j of this thread's circles
        int64_t pair_mine = 0;         // summed over evaluations
        int rebuilds = 0, evals = 0;
        bool fp64 = false;
        double E64o = 0.0, E64t = -1.0;   // FP64 energies (objective / unit circles)
        float E = 0.0f, gp = 0.f, alpha = 0.f;
        double ehist = 0.0;               // lane w: energy of iteration w mod (W+1)
        int status = 0, it = 0, h = 0;
        int req = kReqInit;
        const int W = A.ftol_window;

        for (int q = tid; q < kNB * kNB; q += kDB) { sh.Bm[0][q] = 0.f; sh.Bm[1][q] = 0.f; }
        if (tid == 0) { sh.flag[0] = 1; sh.flag[1] = 0; }

        for (;;) {
            // ================= one evaluation ==================================
            float2 xt[kCPT], sc[kCPT];
            const int par = tcount & 1;
#pragma unroll
            for (int c = 0; c < kCPT; ++c) {
                xt[c] = req == kReqTrial ? make_float2(fmaf(alpha, p[c].x, x[c].x), fmaf(alpha, p[c].y, x[c].y))
                                         : x[c];
                sc[c] = make_float2(xt[c].x - x[c].x, xt[c].y - x[c].y);
                if (act[c]) {
                    sh.pos[tid + c * kDB] = xt[c];
                    const double dx = (double)xt[c].x - (double)xr[c].x;
                    const double dy = (double)xt[c].y - (double)xr[c].y;
                    if (dx * dx + dy * dy > A.skin2) sh.flag[par] = 1;
                }
            }
            __syncthreads();                                            // B1
            if (tid == 0) sh.flag[par ^ 1] = 0;
            if (sh.flag[par]) {
                // ---- neighbor list rebuild at the positions in sh.pos -------
                if (tid == 0) sh.over = 0;    // set again below only after bin_circles' barriers
                bin_circles<kDB>(sh.pos, n, grid, sh.cell_start, sh.cell_circ, sh.slot_tmp,
                                 sh.scan_tmp);
                // ascending circle index inside every cell: lists (cells in
                // row order, then index) are then a function of the
                // positions alone, and so is every sum over them
                for (int cc = tid; cc < grid.nc * grid.nc; cc += kDB) {
                    const int a = sh.cell_start[cc], z = sh.cell_start[cc + 1];
                    for (int q = a + 1; q < z; ++q) {
                        const uint16_t key = sh.cell_circ[q];
                        int t = q - 1;
                        while (t >= a && sh.cell_circ[t] > key) { sh.cell_circ[t + 1] = sh.cell_circ[t]; --t; }
                        sh.cell_circ[t + 1] = key;
                    }
                }
                __syncthreads();
                // one pass: every circle writes its neighbors into its own
                // kEll slots; more than kEll switches this list epoch to
                // sweeping the cell grid instead
#pragma unroll
                for (int c = 0; c < kCPT; ++c) {
                    const int i = tid + c * kDB;
                    if (act[c]) {
                        int m = 0, up = 0;
                        const int cx = cell_coord(xt[c].x, grid), cy = cell_coord(xt[c].y, grid);
                        const int y0 = cy > 0 ? cy - 1 : 0, y1 = cy < grid.nc - 1 ? cy + 1 : grid.nc - 1;
                        const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < grid.nc - 1 ? cx + 1 : grid.nc - 1;
                        for (int yy = y0; yy <= y1; ++yy) {
                            const int a = sh.cell_start[yy * grid.nc + x0];
                            const int z = sh.cell_start[yy * grid.nc + x1 + 1];
                            for (int t = a; t < z; ++t) {
                                const int j = sh.cell_circ[t];
                                if (j != i && near_cut(xt[c], sh.pos[j], c2lo, c2hi, A.c2)) {
                                    if (m < kEll) sh.list[m][i] = (uint16_t)j;
                                    ++m;
                                    up += j > i;
                                }
                            }
                        }
                        if (m > kEll) sh.over = 1;
                        sh.list_n[i] = (uint8_t)(m < kEll ? m : kEll);
                        half_mine[c] = up;
                        xr[c] = xt[c];
                    }
                }
                ++rebuilds;
                __syncthreads();
                overflow = sh.over != 0;
            }
            ++tcount;
            ++evals;
#pragma unroll
            for (int c = 0; c < kCPT; ++c) pair_mine += half_mine[c];
            // ---- pair sweep: energy and gradient of this thread's circles ----
            float e = 0.f, e1 = 0.f;
            double eo = 0.0, et = 0.0;
            float2 gt[kCPT], yc[kCPT];
#pragma unroll
            for (int c = 0; c < kCPT; ++c) {
                const int i = tid + c * kDB;
                const float2 q = xt[c];
                float gx = 0.f, gy = 0.f;
                if (act[c]) {
                    float ec = 0.f, e1c = 0.f;
                    double eoc = 0.0, etc = 0.0;
                    if (!overflow) {
                        const int mcount = sh.list_n[i];
                        for (int t = 0; t < mcount; ++t) {
                            const int j = sh.list[t][i];
                            const float2 pj = sh.pos[j];
                            pair_term32(q, pj, j > i, two_r, four_r2, ec, e1c, gx, gy);
                            // FP64 energies only where FP32 sees (nearly) an overlap:
                            // outside a 1e-5 band the FP64 terms are zero
                            if (fp64 && j > i) {
                                const float dx = q.x - pj.x, dy = q.y - pj.y;
                                if (dx * dx + dy * dy < four_r2_band)
                                    pair_term64(q, pj, two_r64, four_r2_64, eoc, etc);
                            }
                        }
                    } else {
                        // list overflow: every circle of the 3 x 3 cells
                        const int cx = cell_coord(q.x, grid), cy = cell_coord(q.y, grid);
                        const int y0 = cy > 0 ? cy - 1 : 0, y1 = cy < grid.nc - 1 ? cy + 1 : grid.nc - 1;
                        const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < grid.nc - 1 ? cx + 1 : grid.nc - 1;
                        for (int yy = y0; yy <= y1; ++yy) {
                            const int a = sh.cell_start[yy * grid.nc + x0];
                            const int z = sh.cell_start[yy * grid.nc + x1 + 1];
                            for (int t = a; t < z; ++t) {
                                const int j = sh.cell_circ[t];
                                if (j == i) continue;
                                const float2 pj = sh.pos[j];
                                pair_term32(q, pj, j > i, two_r, four_r2, ec, e1c, gx, gy);
                                if (fp64 && j > i) {
                                    const float dx = q.x - pj.x, dy = q.y - pj.y;
                                    if (dx * dx + dy * dy < four_r2_band)
                                        pair_term64(q, pj, two_r64, four_r2_64, eoc, etc);
                                }
                            }
                        }
                    }
                    e += ec;
                    e1 += e1c;
                    eo += eoc;
                    et += etc;
                    // containment (branch-free, as the pair term)
                    const float r2 = q.x * q.x + q.y * q.y;
                    const float ir = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
                    const float d0 = fmaxf(r2 * ir + rad - R, 0.f);
                    e += d0 * d0;
                    const float d01 = fmaxf(d0 - (rad - 1.f), 0.f);
                    e1 += d01 * d01;
                    const float kc = 2.f * d0 * ir;
                    gx += kc * q.x;
                    gy += kc * q.y;
                    if (fp64) {
                        const double r64 = sqrt((double)q.x * q.x + (double)q.y * q.y);
                        const double c0 = r64 + rad64 - R64;
                        if (c0 > 0.0) eo += c0 * c0;
                        const double ct = r64 + 1.0 - R64;
                        if (ct > 0.0) et += ct * ct;
                    }
                    // E sums over every circle: a non-finite position makes it NaN
                    if (!(isfinite(q.x) && isfinite(q.y))) {
                        e = e1 = __builtin_nanf("");
                        eo = et = __builtin_nan("");
                    }
                }
                gt[c] = make_float2(gx, gy);
                yc[c] = make_float2(gx - g[c].x, gy - g[c].y);
            }
            // ---- fused reduction: 63 dot products and E in one pass ----------
            const float wsum = wave_reduce_scatter(gt, sc, yc, S, Y, e, e1);
            sh.red[par][wv][lane_slot(lane)] = wsum;
            if (fp64) {
                const double wo = wave_sum(eo), wt = wave_sum(et);
                if (lane == 0) { sh.red64[par][wv][0] = wo; sh.red64[par][wv][1] = wt; }
            }
            __syncthreads();                                            // B2
            float tot = 0.f;
#pragma unroll
            for (int w = 0; w < kDW; ++w) tot += sh.red[par][w][lane];
            double so = 0.0, st = 0.0;
            if (fp64) {
#pragma unroll
                for (int w = 0; w < kDW; ++w) { so += sh.red64[par][w][0]; st += sh.red64[par][w][1]; }
            }
            const float Et = lane_value(tot, sE);
            const float E1t = lane_value(tot, sE1);

            // ================= what the evaluation was for =====================
            bool accept = false, push = false;
            if (req == kReqTrial) {
                const bool ok = fp64 ? so <= E64o + (double)A.c1 * (double)alpha * (double)gp
                                     : Et <= E + A.c1 * alpha * gp;
                if (ok) {
                    accept = true;
                    const float sy = lane_value(tot, sScYc), yy = lane_value(tot, sYcYc);
                    push = sy > A.eps_curv * yy;
                } else {
                    alpha *= 0.5f;
                    if (++h > A.max_halvings) { status = 4; break; }   // STALLED
                    continue;
                }
            } else if (req == kReqInit) {
                accept = true;   // g and the g row of B from this evaluation
            } else {             // kReqFp64: FP64 energies of the current point
                E64o = so;
                E64t = st;
            }
            if (accept) {
                // ---- Gram matrix of the updated basis (every wave) -----------
                // slot totals to LDS (every wave writes the same bits), then
                // each lane fills 7 of the 21 x 21 entries
                const int nxt = cur ^ 1;
                sh.tot_s[par][lane] = tot;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                for (int r = 0; r < (kNB * kNB + kWave - 1) / kWave; ++r) {
                    const int ent = lane + kWave * r;
                    if (ent < kNB * kNB) {
                        const int src = sh.bsrc[push ? 1 : 0][ent];
                        sh.Bm[nxt][ent] = (src & 0x8000) ? sh.tot_s[par][src & 0x7fff] : sh.Bm[cur][src];
                    }
                }
                cur = nxt;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                for (int c = 0; c < kCPT; ++c) {
                    if (push) {
#pragma unroll
                        for (int j = 0; j < kMM - 1; ++j) { S[j][c] = S[j + 1][c]; Y[j][c] = Y[j + 1][c]; }
                        S[kMM - 1][c] = sc[c];
                        Y[kMM - 1][c] = yc[c];
                    }
                    x[c] = xt[c];
                    g[c] = gt[c];
                }
                if (push) k = k + 1 > A.m ? A.m : k + 1;
                if (req == kReqTrial) ++it;
                E = Et;
                if (fp64) { E64o = so; E64t = st; }
                // FP64 regime once either FP32 energy is small: with a contact
                // margin the unit circles can be overlap-free while E (radius
                // rad) still sums (2 mu)^2 over every contact
                if (!fp64 && A.tau64 > 0.0 && (double)fminf(E, E1t) < A.tau64) {
                    fp64 = true;
                    req = kReqFp64;          // FP64 energies of x before going on
                    continue;
                }
            }

            // ================= top of an iteration: stop tests =================
            const float gg = sh.Bm[cur][kG * kNB + kG];
            const float gn = sqrtf(fmaxf(gg, 0.f));
            const double Eacc = fp64 ? E64o : (double)E;
            if (!isfinite(E) || !isfinite(gn)) { status = 6; break; }
            if (fp64 && E64t < A.e_feasible) { status = 1; break; }
            if (gn <= A.g_tol) { status = 2; break; }
            if (A.ftol > 0.f && it >= W) {
                const int src = (it - W) % (W + 1);
                const long long bits = __builtin_bit_cast(long long, ehist);
                const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), src);
                const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
                const double eold = __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
                if (eold - Eacc <= (double)A.ftol * eold) { status = 3; break; }
            }
            if (lane == it % (W + 1)) ehist = Eacc;
            if (it >= A.max_iter) { status = 5; break; }

            // ================= direction: two-loop recursion on B ===============
            // lane l plays basis vector l (column l of B in registers); dl is
            // its coefficient in H g.
            float Bc[kNB];
#pragma unroll
            for (int a2 = 0; a2 < kNB; ++a2) Bc[a2] = lane < kNB ? sh.Bm[cur][a2 * kNB + lane] : 0.f;
            float dl = lane == kG ? 1.f : 0.f;
            float alph[kMM], rhoj[kMM];
#pragma unroll
            for (int j = kMM - 1; j >= 0; --j) {
                alph[j] = 0.f;
                rhoj[j] = 0.f;
                if (j >= kMM - k) {
                    rhoj[j] = 1.f / lane_value(Bc[j], kMM + j);          // 1 / s_j'y_j
                    const float a = rhoj[j] * wave_sum_dpp(dl * Bc[j]);
                    alph[j] = a;
                    if (lane == kMM + j) dl -= a;
                }
            }
            if (k > 0) {
                const float sy = lane_value(Bc[kMM - 1], 2 * kMM - 1);
                const float yy = lane_value(Bc[2 * kMM - 1], 2 * kMM - 1);
                dl *= sy / yy;
            }
#pragma unroll
            for (int j = 0; j < kMM; ++j) {
                if (j >= kMM - k) {
                    const float bb = rhoj[j] * wave_sum_dpp(dl * Bc[kMM + j]);
                    if (lane == j) dl += alph[j] - bb;
                }
            }
            {
                gp = -wave_sum_dpp(dl * Bc[kG]);
                const float cg = lane_value(dl, kG);
                float cs[kMM], cy[kMM];
#pragma unroll
                for (int j = 0; j < kMM; ++j) {
                    cs[j] = lane_value(dl, j);
                    cy[j] = lane_value(dl, kMM + j);
                }
#pragma unroll
                for (int c = 0; c < kCPT; ++c) {
                    float px = -cg * g[c].x, py = -cg * g[c].y;
#pragma unroll
                    for (int j = 0; j < kMM; ++j) {
                        px -= cs[j] * S[j][c].x + cy[j] * Y[j][c].x;
                        py -= cs[j] * S[j][c].y + cy[j] * Y[j][c].y;
                    }
                    p[c] = make_float2(px, py);
                }
            }
            if (k > 0 && !(gp < 0.f)) {
                k = 0;
#pragma unroll
                for (int c = 0; c < kCPT; ++c) p[c] = make_float2(-g[c].x, -g[c].y);
                gp = -gg;
            }
            alpha = k > 0 ? 1.f : 1.f / fmaxf(1.f, gn);
            h = 0;
            req = kReqTrial;
        }

        // ---- write back ------------------------------------------------------
        {
            // listed pairs i<j summed over evaluations (each pair once: by the
            // thread of its lower index)
            unsigned long long pm = (unsigned long long)pair_mine;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) pm += __shfl_xor(pm, o, kWave);
            __syncthreads();
            if (lane == 0) sh.red64[0][wv][0] = __builtin_bit_cast(double, pm);
            __syncthreads();
            pm = 0;
            for (int w = 0; w < kDW; ++w) pm += __builtin_bit_cast(unsigned long long, sh.red64[0][w][0]);
            pair_mine = (int64_t)pm;
        }
#pragma unroll
        for (int c = 0; c < kCPT; ++c)
            if (act[c]) reinterpret_cast<float2 *>(xy)[off + tid + c * kDB] = x[c];
        if (tid == 0) {
            DescentResultDev r;
            r.status = status;
            r.iters = it;
            r.evals = evals;
            r.rebuilds = rebuilds;
            r.pair_evals = pair_mine;
            r.E32 = E;
            r.gnorm = sqrtf(fmaxf(sh.Bm[cur][kG * kNB + kG], 0.f));
            r.E64 = fp64 ? E64t : -1.0;
            out[b] = r;
        }
    }
}

// Queue set-up: counter = 0 and instance order by n descending, one
// workgroup, counting sort over n in [0, kMaxN]; invalid sizes go last.
constexpr int kQB = 1024;
__global__ __launch_bounds__(kQB) void queue_init_kernel(const int32_t *__restrict__ offset,
                                                         int B, int32_t *__restrict__ queue)
{
    __shared__ int hist[kMaxN + 2];
    __shared__ int scan_tmp[kQB / kWave + 1];
    for (int i = threadIdx.x; i < kMaxN + 2; i += kQB) hist[i] = 0;
    __syncthreads();
    auto key = [&](int b) {
        const int n = offset[b + 1] - offset[b];
        return (n >= 0 && n <= kMaxN) ? kMaxN - n : kMaxN + 1;   // descending n
    };
    for (int b = threadIdx.x; b < B; b += kQB) atomicAdd(&hist[key(b)], 1);
    __syncthreads();
    // exclusive scan of the histogram (kMaxN + 2 bins, 2 per thread at most)
    const int c0 = threadIdx.x * 2;
    const int v0 = c0 < kMaxN + 2 ? hist[c0] : 0;
    const int v1 = c0 + 1 < kMaxN + 2 ? hist[c0 + 1] : 0;
    int total;
    const int ex = block_exclusive_scan<kQB>(v0 + v1, scan_tmp, &total);
    if (c0 < kMaxN + 2) hist[c0] = ex;
    if (c0 + 1 < kMaxN + 2) hist[c0 + 1] = ex + v0;
    __syncthreads();
    // scatter; the order among instances of equal n does not affect any result
    for (int b = threadIdx.x; b < B; b += kQB) queue[1 + atomicAdd(&hist[key(b)], 1)] = b;
    if (threadIdx.x == 0) queue[0] = 0;
}

int descend_grid(int B)
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    static int per_cu = 0;
    if (per_cu == 0) {
        int occ = 0;
        per_cu = (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, lbfgs_descend_kernel, kDB, 0) ==
                      hipSuccess && occ > 0) ? occ : 1;
    }
    const int cap = cus * per_cu;
    return B < cap ? B : cap;
}

hipError_t launch_descend(const int32_t *offset, const float *R, const double *R64, float *xy,
                          int B, int64_t total_n, const DescentArgs &a, void *out,
                          int32_t *queue, int grid, hipStream_t s)
{
    queue_init_kernel<<<1, kQB, 0, s>>>(offset, B, queue);
    if (grid < 1) grid = 1;
    lbfgs_descend_kernel<<<grid, kDB, 0, s>>>(offset, R, R64, xy, B, total_n, a,
                                              reinterpret_cast<DescentResultDev *>(out), queue);
    return hipGetLastError();
}

}  // namespace pecc
