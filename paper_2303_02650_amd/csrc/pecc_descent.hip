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
//
// Three instantiations share this code: the whole-instance descent, the
// container adjustment (the radius as a variable) and the batch descent of
// Alg. 1 over a given k-batch partition, visited one batch after another
// (see the kernel's comment).
#include "pecc_device.hpp"
#include "pecc_host.hpp"
#include "pecc_launch.hpp"
#include "pecc_lbfgs.hpp"

#include <type_traits>

namespace pecc {

constexpr int kDB = 512;                  // threads per workgroup
constexpr int kDW = kDB / kWave;          // waves per workgroup
constexpr int kCPT = kMaxN / kDB;         // circles per thread
constexpr int kEll = 24;                  // neighbor slots per circle (ELL list)
constexpr int kEllSeq = 32;               // ... in the batch descent (l_cut up to 4)

enum : int { kModeWhole = 0, kModeAdj = 1, kModeSeq = 2, kModeDense = 3 };

// Byte offset (into the position array) of the far point that pads every
// neighbor list up to the longest list of its wave: a pair with it has no
// overlap, so its terms add exact zeros and the list loop needs no test.
constexpr int kFarOff = kMaxN * (int)sizeof(float2);
constexpr float kFarCoord = 3.0e18f;      // (3e18)^2 * 2 is finite in FP32

// Whole-instance descent: row length of the Gram ring in LDS.  Row r (the
// basis vector in storage slot r: s 0..9, y 10..19, g 20) holds the s
// storage slots twice (0..9, 10..19), the y slots twice (20..29, 30..39)
// and g (40), so that the row of any basis vector read in pair order (pair
// j at storage (hd + j) mod 10) is contiguous from offset hd.
constexpr int kRS = 4 * kMM + 1;

template <int ELL>
struct DescentShared {
    float2 pos[kMaxN + 1];         // pos[kMaxN]: the far point
    int cell_start[kMaxCells + 1];
    uint16_t cell_circ[kMaxN];
    uint16_t slot_tmp[kMaxN];
    uint16_t list[ELL][kMaxN];     // slot-major: lanes read consecutive entries; byte offsets into pos
    uint8_t  list_n[kMaxN];
    float red[2][kDW][kWave];
    double red64[2][kDW][2];
    float Bm[2][kNB * kNB];
    float Bring[kNB * kRS];        // whole-instance descent: Gram ring, rows as above
    uint32_t bperm[kWave];         // source slots of the Gram update per lane (byte addresses)
    float tot_s[2][kWave];
    float rho[2][kMM];             // 1 / s_j'y_j of the Gram buffer of the same index
    uint16_t bsrc[2][kNB * kNB];   // Gram update sources, see gram_source
    int scan_tmp[kDW + 1];
    int flag[2];
    int over;                      // a circle had more than ELL neighbors
    int work;
    int cell_evals;                // evaluations over the cell grid (instance)
    int npair[kMaxSeqBatches + 1]; // listed pairs i<j of the current lists: per batch, and in all
    // whole-instance descent: what the deciding wave leaves for the others
    int dec_flags;                 // kDec* bits
    int dec_cb;                    // batch descent: the batch of the next evaluation
    int dec_req;                   // what the next evaluation is for
    int dec_fp64;                  // FP64 regime from the next evaluation on
    float dec_alpha;               // step length of the next trial
    float dec_gam;                 // gamma of the direction
    float coef[2][kMM];            // coefficients of s_j and y_j in the direction
    // the constants of the decisions, read where used (kept in registers
    // they would crowd out the loop's scalar state)
    struct {
        double tau64, e_feasible;
        float c1, eps_curv, ftol, g_tol_sq, g_tol;
        int m, max_halvings, max_iter, nbat, anm;
    } dk;
    float dec_Rz, dec_pR;          // container adjustment: radius and its search component
};

// Batch descent only: the saved Gram matrix of every batch, batch ids and
// batch sizes.
struct SeqShared {
    float BmP[kMaxSeqBatches][kNB * kNB];
    uint8_t bat[kMaxN];
    int cnt[kMaxSeqBatches];
};
// Dense batch descent: batch ids and sizes, every circle's index inside its
// batch, each batch's matrix and vector offsets in the workspace, four
// vectors of a batch's coordinates staged for a matrix pass, per-wave
// partial sums, and the pass's per-item partial sums (two products).
struct DenseShared {
    uint8_t bat[kMaxN];
    int cnt[kMaxSeqBatches];
    uint16_t memb[kMaxN];
    int hoff[kMaxSeqBatches + 1];
    int voff[kMaxSeqBatches + 1];
    float4 vr[2 * kMaxN];       // (g, y_Q, s_K, w_K) by row of the batch matrix
    float wpart[4][kDB / kWave];
    float4 part[2 * kDB];
};

// Per-batch state of the dense descent (bits of a lane-indexed word): the
// stored matrix S still stands for I (never written), a known pending
// update K, a newest curvature pair Q, which of the two s slots holds K's s.
enum : int { kDnIdent = 1, kDnK = 2, kDnQ = 4, kDnSlot = 8 };

// Work split of a pass over a symmetric d x d matrix (d even, d <= 2048)
// stored row-major with rows of sym_ld(d) floats (the padding columns from
// d on belong to no entry; the quads cover d rounded up to 4 columns): an
// item is a column quad (four consecutive columns, one 16-byte load per
// row, consecutive across a wave) and a slice of the rows; there are at
// most BLOCK items, one per thread.
struct QuadSplit {
    int cq, nq, items;
    __device__ QuadSplit(int ld, int nthreads)
    {
        cq = ld / 4;
        nq = cq > 0 ? nthreads / cq : 1;
        nq = nq < 1 ? 1 : (nq > 16 ? 16 : nq);
        items = cq * nq;
    }
};

// Row length of a dense batch matrix of order d (the largest order the
// workspace bound allows for rows of d + 2 floats is 1024).  Up to 1024 a
// multiple of 4 floats; above, a multiple of 64, so that rows start on
// 256-byte boundaries (a wave's 1 KB of a row then spans 8 cache lines,
// not 9: 6 % more matrix bandwidth at d = 2000 with every CU busy).
// Smaller matrices are not padded further: a batch of them largely stays in
// the last-level cache, where padding only adds footprint (measured slower
// at d = 1000, 400 and 336).
__device__ __forceinline__ int sym_ld(int d) { return d <= 1024 ? (d + 3) & ~3 : (d + 63) & ~63; }

// One row of a thread's column quad: h holds S's four entries of the row
// (I's when nothing is read), vq = (g, y, s, w) at the row, cs and cw s
// and w at the four columns.  acc[0..3] gather (S g) and acc[4..7] (S y) of
// the four columns; with STORE h becomes S + U for the symmetric rank-2
// update U = -(w s' + s w') ib + a2 s s'.
template <bool STORE>
__device__ __forceinline__ void quad_elem(float4 &h, float4 vq, float4 cs, float4 cw, float ib,
                                          float a2, float (&acc)[8])
{
    acc[0] += h.x * vq.x;
    acc[1] += h.y * vq.x;
    acc[2] += h.z * vq.x;
    acc[3] += h.w * vq.x;
    acc[4] += h.x * vq.y;
    acc[5] += h.y * vq.y;
    acc[6] += h.z * vq.y;
    acc[7] += h.w * vq.y;
    if constexpr (STORE) {
        h.x = h.x - (vq.w * cs.x + vq.z * cw.x) * ib + a2 * vq.z * cs.x;
        h.y = h.y - (vq.w * cs.y + vq.z * cw.y) * ib + a2 * vq.z * cs.y;
        h.z = h.z - (vq.w * cs.z + vq.z * cw.z) * ib + a2 * vq.z * cs.z;
        h.w = h.w - (vq.w * cs.w + vq.z * cw.w) * ib + a2 * vq.z * cs.w;
    }
}

template <bool LOAD>
__device__ __forceinline__ float4 quad_load(const float4 *col, int64_t st, int rr, int r, int c0)
{
    if constexpr (LOAD) return col[(int64_t)rr * st];
    else
        return make_float4(r == c0 ? 1.f : 0.f, r == c0 + 1 ? 1.f : 0.f, r == c0 + 2 ? 1.f : 0.f,
                           r == c0 + 3 ? 1.f : 0.f);
}

// One pass over a symmetric d x d matrix S (rows of sym_ld(d) floats,
// 16-byte aligned at least): S g and S y as column sums (y_c = sum_r S[r][c] v[r] in
// ascending r per row slice, slices added in order: deterministic) into
// part[k] = ((S g)_{2k}, (S g)_{2k+1}, (S y)_{2k}, (S y)_{2k+1}) for k <
// d / 2, and with STORE S + U written back (U as in quad_elem, with ib and
// a2).  vr[r] = (g, y, s, w) at row r.  LOAD = false takes S = I without
// reading it.  The row loop keeps U loads of 16 bytes in flight per thread
// before it waits.  part holds 2 BLOCK entries; every thread of the block
// calls it; ends with a barrier.
template <int BLOCK, bool LOAD, bool STORE>
__device__ void sym_pass(float *__restrict__ H, int d, const float4 *__restrict__ vr, float ib,
                         float a2, float4 *part)
{
    constexpr int U = 8;
    const int t = (int)threadIdx.x;
    const int ld = sym_ld(d), dq = (d + 3) & ~3;
    const QuadSplit sp(dq, BLOCK);
    const bool on = t < sp.items;
    const int qd = on ? t % sp.cq : 0, sl = on ? t / sp.cq : 0;
    const int q0 = on ? (int)((int64_t)d * sl / sp.nq) : 0;
    const int q1 = on ? (int)((int64_t)d * (sl + 1) / sp.nq) : 0;
    const int c0 = 4 * qd;
    const int64_t st = ld / 4;
    float4 *col = reinterpret_cast<float4 *>(H) + (int64_t)q0 * st + qd;
    // s and w at the quad's columns (zero at padding columns)
    float4 cs = make_float4(0.f, 0.f, 0.f, 0.f), cw = cs;
    if (on) {
        const float4 v0 = vr[c0], v1 = vr[c0 + 1];
        cs.x = v0.z;
        cw.x = v0.w;
        cs.y = v1.z;
        cw.y = v1.w;
        if (c0 + 2 < d) {
            const float4 v2 = vr[c0 + 2], v3 = vr[c0 + 3];
            cs.z = v2.z;
            cw.z = v2.w;
            cs.w = v3.z;
            cw.w = v3.w;
        }
    }
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int L = q1 - q0;
    int r = 0;
    for (; r + U <= L; r += U) {
        float4 h[U];
#pragma unroll
        for (int u = 0; u < U; ++u) h[u] = quad_load<LOAD>(col, st, r + u, q0 + r + u, c0);
#pragma unroll
        for (int u = 0; u < U; ++u) quad_elem<STORE>(h[u], vr[q0 + r + u], cs, cw, ib, a2, acc);
        if constexpr (STORE) {
#pragma unroll
            for (int u = 0; u < U; ++u) col[(int64_t)(r + u) * st] = h[u];
        }
    }
    for (; r < L; ++r) {
        float4 h = quad_load<LOAD>(col, st, r, q0 + r, c0);
        quad_elem<STORE>(h, vr[q0 + r], cs, cw, ib, a2, acc);
        if constexpr (STORE) col[(int64_t)r * st] = h;
    }
    const int cpl = dq / 2;
    if (on) {
        part[sl * cpl + 2 * qd] = make_float4(acc[0], acc[1], acc[4], acc[5]);
        part[sl * cpl + 2 * qd + 1] = make_float4(acc[2], acc[3], acc[6], acc[7]);
    }
    __syncthreads();
    // slice sums in place: entry k < d / 2 is read and written by one thread only
    for (int k = t; k < d / 2; k += BLOCK) {
        float4 a = part[k];
        for (int j = 1; j < sp.nq; ++j) {
            const float4 o = part[j * cpl + k];
            a.x += o.x;
            a.y += o.y;
            a.z += o.z;
            a.w += o.w;
        }
        part[k] = a;
    }
    __syncthreads();
}
struct NoShared {
    int unused;
};

// Evaluation requests of the descent's state machine.
enum : int { kReqInit = 0, kReqFp64 = 1, kReqTrial = 2, kReqTotal = 3 };
// outcome of an evaluation in the whole-instance descent
enum : int { kDecAccept = 1, kDecPush = 2, kDecStop = 4, kDecNext = 8, kDecSteepest = 16, kDecAnm = 32 };

// ADJ: container adjustment (Sec. 4.2, Eq. 12, Alg. 2).  The radius joins
// the variables, the objective is U = E + lambda R^2 and A.rounds
// minimisations run with lambda halved after each (a fresh history every
// round).  The deciding wave additionally holds in lane l the radius
// component of basis vector l (hR_v), so after the fused reduction every
// Gram entry gets its R x R product added, and the unit-circle energy slot
// carries sum_i d_i0 instead, from which dU/dR = -2 sum_i d_i0 + 2 lambda R;
// the radius and its search component reach the other waves with the
// decision.  FP32 throughout (no FP64 regime, no FEASIBLE stop: U > 0);
// Rout[b] receives the final radius.
//
// SEQ: batch descent of Alg. 1 over the partition part[] into A.nbat
// batches.  An outer iteration visits the non-empty batches in index order;
// a visit is one L-BFGS iteration on the batch energy of Eq. 7 with the
// other circles where the earlier visits left them: an evaluation at the
// current positions (the batch's gradient and its Gram row), the two-loop
// over the batch's own history (each circle's history registers belong to
// its batch; the batch's Gram matrix is saved in LDS between visits), and
// the backtracking line search, whose accepted trial gives the curvature
// pair.  Only the batch's circles are swept and move; a pair counts in the
// batch energy when its other circle is outside the batch or has the
// higher index (each pair once).  A visit whose line search fails leaves
// the batch where it was.  Every outer iteration starts with an evaluation
// of the whole instance (E, and the FP64 energies for the FEASIBLE test)
// and the stop tests on it; the sum of the visits' gradient norms stands
// for ||g||.  A.anm = 1 replaces the displacement trigger of the neighbor
// lists by ANM (Alg. 3): after every outer iteration cnt += 1, and once cnt
// >= len the lists of the current positions are compared with the stored
// ones -- different: rebuild, len = 1; equal: len doubles.  With one
// non-empty batch the descent is the whole-instance one (ANM after every
// iteration, the point re-evaluated when the lists change).
template <int MODE>
__global__ __launch_bounds__(kDB) void lbfgs_descend_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ Rv,
    const double *__restrict__ Rv64, float *__restrict__ xy,
    int B, int64_t total_n, DescentArgs A, DescentResultDev *__restrict__ out,
    int32_t *__restrict__ queue, float *__restrict__ Rout, const int32_t *__restrict__ part,
    float *__restrict__ Hws)
{
    constexpr bool ADJ = MODE == kModeAdj;
    constexpr bool DENSE = MODE == kModeDense;
    constexpr bool SEQ = MODE == kModeSeq || DENSE;
    // whole instance: one wave takes the uniform decisions of an evaluation
    constexpr bool SOLO = MODE == kModeWhole || MODE == kModeSeq || MODE == kModeAdj;
    // every wave decides only in the dense mode
    static_assert(SOLO || DENSE, "the limited-memory modes decide on one wave");
    constexpr int ELL = SEQ ? kEllSeq : kEll;
    __shared__ DescentShared<ELL> sh;
    __shared__ std::conditional_t<DENSE, DenseShared, std::conditional_t<SEQ, SeqShared, NoShared>> sq;
    const int tid = threadIdx.x;
    // (lane ids are recomputed per evaluation from an opaque copy of tid)
    // wave index, wave-uniform to the compiler (branches on it stay scalar)
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    for (int q = tid; q < 2 * kNB * kNB; q += kDB)
        sh.bsrc[q / (kNB * kNB)][q % (kNB * kNB)] = gram_source(q % (kNB * kNB), q >= kNB * kNB);
    if constexpr (SOLO)
        if (tid < kWave) sh.bperm[tid] = gram_perm_bytes(tid);
    const float c2lo = (float)(A.c2 * (1.0 - 1e-5)), c2hi = (float)(A.c2 * (1.0 + 1e-5));

    for (;;) {
        // ---- next instance from the queue ------------------------------------
        __syncthreads();
        if (tid == 0) sh.work = atomicAdd(&queue[0], 1);
        __syncthreads();
        const int slot = sh.work;
        if (slot >= B) break;
        // an opaque copy of the thread id for this instance: set-up addresses
        // are recomputed per instance instead of staying live across them
        int tid_i = (int)threadIdx.x;
        asm volatile("" : "+v"(tid_i));
        const int tid = tid_i;
        const int b = queue[1 + slot];
        const int off = offset[b], n = offset[b + 1] - off;
        if (!(off >= 0 && n >= 0 && n <= kMaxN && (int64_t)off + n <= total_n)) {
            if (tid == 0) {
                store_bad_instance(out, b);   // BAD_INSTANCE
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

        // ---- batch descent: batch of every circle, batch sizes --------------
        // batch of circle tid + c * kDB (read from LDS where needed, so no
        // registers stay live for it; stale for circles beyond n, which no
        // use reads without act[c])
        auto batc_of = [&](int c) -> int {
            if constexpr (SEQ) return sq.bat[(int)threadIdx.x + c * kDB];
            else return 0;
        };
        bool visits = false;            // more than one non-empty batch
        int first_b = 0;                // first non-empty batch
        if constexpr (SEQ) {
            for (int q = tid; q < kMaxSeqBatches; q += kDB) sq.cnt[q] = 0;
            if constexpr (!DENSE)
                for (int q = tid; q < kMaxSeqBatches * kNB * kNB; q += kDB)
                    sq.BmP[q / (kNB * kNB)][q % (kNB * kNB)] = 0.f;
            __syncthreads();
            int bad = 0;
#pragma unroll
            for (int c = 0; c < kCPT; ++c) {
                const int i = tid + c * kDB;
                if (i < n) {
                    const int v = part[off + i];
                    if (v < 0 || v >= A.nbat) {
                        bad = 1;
                    } else {
                        sq.bat[i] = (uint8_t)v;
                        atomicAdd(&sq.cnt[v], 1);
                    }
                }
            }
            if (__syncthreads_or(bad)) {
                if (tid == 0) {
                    store_bad_instance(out, b);   // BAD_INSTANCE: a batch id out of range
                }
                continue;
            }
            int ne = 0;
            first_b = -1;
            for (int q = 0; q < A.nbat; ++q)
                if (sq.cnt[q] > 0) { ++ne; if (first_b < 0) first_b = q; }
            if (first_b < 0) first_b = 0;
            visits = ne > 1;
        }
        // dense: every circle's index inside its batch (ascending circle
        // index); each batch's matrix and its four vectors (s slots 0 and 1,
        // y, w) in this instance's region.  The matrices are not written
        // here: a batch's S stands for I until its first update is applied.
        float *Hbase = nullptr;
        if constexpr (DENSE) {
            visits = true;                   // one batch too: the dense update
            Hbase = Hws + (int64_t)b * A.hstride;
#pragma unroll
            for (int c = 0; c < kCPT; ++c) {
                const int i = tid + c * kDB;
                if (i < n) {
                    int r = 0;
                    const int bi = sq.bat[i];
                    for (int j = 0; j < i; ++j) r += sq.bat[j] == bi ? 1 : 0;
                    sq.memb[i] = (uint16_t)r;
                }
            }
            if (tid == 0) {
                int o = 0;
                for (int q = 0; q < A.nbat; ++q) {
                    sq.hoff[q] = o;
                    const int d = 2 * sq.cnt[q];
                    o += d * sym_ld(d);
                }
                sq.hoff[A.nbat] = o;
                for (int q = 0; q < A.nbat; ++q) {
                    sq.voff[q] = o;
                    o += 4 * 2 * sq.cnt[q];
                }
                sq.voff[A.nbat] = o;
            }
            __syncthreads();
            if ((int64_t)sq.voff[A.nbat] > A.hstride) {
                if (tid == 0) {
                    store_bad_instance(out, b);   // BAD_INSTANCE: the matrices do not fit the workspace
                }
                continue;
            }
        }

        // ---- per-thread state (circle c of this thread is tid + c*kDB) ----
        bool act[kCPT];
        float2 x[kCPT], g[kCPT], xr[kCPT], p[kCPT];
        double S[kMM][kCPT], Y[kMM][kCPT];      // curvature pairs (float2 bits), newest at kMM-1
#pragma unroll
        for (int c = 0; c < kCPT; ++c) {
            const int i = tid + c * kDB;
            act[c] = i < n;
            x[c] = act[c] ? reinterpret_cast<const float2 *>(xy)[off + i] : make_float2(0.f, 0.f);
            g[c] = make_float2(0.f, 0.f);
            xr[c] = x[c];
            p[c] = make_float2(0.f, 0.f);
#pragma unroll
            for (int j = 0; j < kMM; ++j) { S[j][c] = 0.0; Y[j][c] = 0.0; }
        }
        // ---- uniform state ---------------------------------------------------
        int k = 0;                     // valid pairs, slots kMM-k .. kMM-1
        int cur = 0;                   // Bm buffer in use
        int tcount = 0;                // evaluations so far (flag parity)
        bool overflow = false;         // list did not fit: sweep the cell grid
        int64_t pair_mine = 0;         // listed pairs i<j swept, summed over evaluations (uniform)
        int rebuilds = 0, evals = 0;
        bool fp64 = false;
        double E64o = 0.0, E64t = -1.0;   // FP64 energies (objective / unit circles)
        float E = 0.0f, gp = 0.f, alpha = 0.f;
        double ehist = 0.0;               // lane w: energy of iteration w mod (W+1)
        int status = 0, it = 0, h = 0;
        int itw = 0;                      // it mod (W + 1), kept by the deciding wave
        int hd = 0;                       // storage pair of pair 0 (ring form of B)
        int req = (SEQ && visits) ? kReqTotal : kReqInit;
        const int W = A.ftol_window;
        // batch descent (uniform): current batch, history count of batch p
        // at lane p, gradient-norm sums, visits and stalled visits of the
        // outer iteration, ANM counter and deferring length
        int cb = first_b, kb_v = 0;
        float gsum = 0.f, gsum_prev = 0.f, E_tot = 0.f;
        int nvis = 0, nstall = 0;
        int anm_cnt = 0, anm_len = 1, anm_it = 0;
        // dense (lane p: batch p): kDn* flags, 1/beta and a2 of K, beta of Q
        int dst_v = kDnIdent;
        float ibK_v = 0.f, a2K_v = 0.f, bQ_v = 0.f;

        // relative decrease of the accepted energy over the last W iterations
        // (lane w of ehist holds iteration w mod (W + 1); src: lane of
        // iteration it - W) at most ftol
        auto decreased_too_little = [&](double Eacc, int src, float ftol) -> bool {
            const long long bits = __builtin_bit_cast(long long, ehist);
            const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), src);
            const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
            const double eold = __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
            return eold - Eacc <= (double)ftol * eold;
        };
        // batch descent: batch bb's saved Gram matrix into B (every wave
        // writes the same values and reads back its own)
        // ANM (Alg. 3), one call: cnt += 1; once cnt >= len the neighbor
        // lists of the current positions are compared with the stored ones
        // (same predicate; as sets).  Different (or the stored lists did not
        // fit): the next evaluation rebuilds them and len = 1; equal: len
        // doubles.  Returns whether the lists change.
        auto anm_tick = [&]() -> bool {
            if (++anm_cnt < anm_len) return false;
            anm_cnt = 0;
            return true;
        };
        auto anm_compare = [&]() -> bool {
            const int t0 = (int)threadIdx.x;
#pragma unroll
            for (int c = 0; c < kCPT; ++c)
                if (act[c]) sh.pos[t0 + c * kDB] = x[c];
            __syncthreads();
            bin_circles<kDB>(sh.pos, n, grid, sh.cell_start, sh.cell_circ, sh.slot_tmp,
                             sh.scan_tmp);
            int diff = overflow ? 1 : 0;
#pragma unroll
            for (int c = 0; c < kCPT; ++c) {
                const int i = t0 + c * kDB;
                if (act[c] && !diff) {
                    const int old = sh.list_n[i];
                    int m = 0;
                    for_each_candidate(i, x[c], grid, sh.cell_start, sh.cell_circ, [&](int j) {
                        if (near_cut(x[c], sh.pos[j], c2lo, c2hi, A.c2)) {
                            bool found = false;
                            for (int t = 0; t < old; ++t) found = found || sh.list[t][i] == j * (int)sizeof(float2);
                            if (!found) diff = 1;
                            ++m;
                        }
                    });
                    if (m != old) diff = 1;
                }
            }
            const bool changed = __syncthreads_or(diff) != 0;
            if (changed) {
                if (t0 == 0) sh.flag[tcount & 1] = 1;
                anm_len = 1;
            } else if (anm_len < (1 << 29)) {
                anm_len *= 2;
            }
            return changed;
        };
        auto anm_step = [&]() -> bool { return anm_tick() && anm_compare(); };
        // dense batch descent (Eq. 8-11).  Each batch's matrix is kept one
        // update behind: the stored S, a known pending update K = (s_K, w_K,
        // 1/beta_K, a2_K) and the newest curvature pair Q = (s_Q, y_Q, beta_Q)
        // whose w = H' y_Q is not formed yet, so that H_p = S + K + Q with
        // Eq. 11 written as the symmetric rank-2 update
        //   -(w s' + s w')/beta + (y'w/beta^2 + 1/beta) s s',  w = H' y.
        // A visit makes one pass over S: it reads S (unless S stands for I),
        // forms S g and S y_Q, and writes S + K back; (S + K) y_Q = w_Q and
        // H_p g = (S + K) g + Q g then follow from dot products, and Q
        // becomes the next K.  One read and one write of the matrix per
        // visit.  Sums over a batch's coordinates go lane 0 -> per-wave slot
        // -> every thread in wave order (deterministic).
        auto batch_sum4 = [&](float4 v) -> float4 {
            float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
            if constexpr (DENSE) {
                const int t0 = (int)threadIdx.x;
                const float s0 = wave_sum(v.x), s1 = wave_sum(v.y), s2 = wave_sum(v.z),
                            s3 = wave_sum(v.w);
                if ((t0 & (kWave - 1)) == 0) {
                    sq.wpart[0][t0 / kWave] = s0;
                    sq.wpart[1][t0 / kWave] = s1;
                    sq.wpart[2][t0 / kWave] = s2;
                    sq.wpart[3][t0 / kWave] = s3;
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < kDW; ++q) {
                    r.x += sq.wpart[0][q];
                    r.y += sq.wpart[1][q];
                    r.z += sq.wpart[2][q];
                    r.w += sq.wpart[3][q];
                }
                __syncthreads();
            }
            return r;
        };
        // p = -H_p g on the batch's circles (zero elsewhere); returns g'p
        auto dense_direction = [&]() -> float {
            float gpv = 0.f;
            if constexpr (DENSE) {
                const int t0 = (int)threadIdx.x, ln = t0 & (kWave - 1);
                const int d = 2 * sq.cnt[cb];
                float *H = Hbase + sq.hoff[cb];
                float *V = Hbase + sq.voff[cb];
                const int fl = __builtin_amdgcn_readlane(dst_v, cb);
                const bool ident = fl & kDnIdent, hasK = fl & kDnK, hasQ = fl & kDnQ;
                const int ks = (fl & kDnSlot) ? 1 : 0;
                const float ibK = lane_value(ibK_v, cb), a2K = lane_value(a2K_v, cb);
                const float2 *sK = reinterpret_cast<const float2 *>(V + ks * d);
                const float2 *sQ = reinterpret_cast<const float2 *>(V + (ks ^ 1) * d);
                const float2 *yQ = reinterpret_cast<const float2 *>(V + 2 * d);
                float2 *wK = reinterpret_cast<float2 *>(V + 3 * d);
                const float2 z2 = make_float2(0.f, 0.f);
                // stage g, y_Q, s_K, w_K (zeros where absent)
#pragma unroll
                for (int c = 0; c < kCPT; ++c) {
                    const int i = t0 + c * kDB;
                    if (act[c] && batc_of(c) == cb) {
                        const int m = sq.memb[i];
                        const float2 yv = hasQ ? yQ[m] : z2;
                        const float2 sv = hasK ? sK[m] : z2;
                        const float2 wvv = hasK ? wK[m] : z2;
                        sq.vr[2 * m] = make_float4(g[c].x, yv.x, sv.x, wvv.x);
                        sq.vr[2 * m + 1] = make_float4(g[c].y, yv.y, sv.y, wvv.y);
                    }
                }
                __syncthreads();
                const bool pass = !ident || hasK;
                if (ident && hasK) sym_pass<kDB, false, true>(H, d, sq.vr, ibK, a2K, sq.part);
                else if (hasK) sym_pass<kDB, true, true>(H, d, sq.vr, ibK, a2K, sq.part);
                else if (pass) sym_pass<kDB, true, false>(H, d, sq.vr, ibK, a2K, sq.part);
                // S g, S y_Q of this thread's circles; K's dot products
                float2 Hg[kCPT], wq[kCPT];
                float4 dk = make_float4(0.f, 0.f, 0.f, 0.f);   // s_K'g, w_K'g, s_K'y_Q, w_K'y_Q
#pragma unroll
                for (int c = 0; c < kCPT; ++c) {
                    Hg[c] = wq[c] = z2;
                    const int i = t0 + c * kDB;
                    if (act[c] && batc_of(c) == cb) {
                        const int m = sq.memb[i];
                        const float2 yv = make_float2(sq.vr[2 * m].y, sq.vr[2 * m + 1].y);
                        if (pass) {
                            const float4 pr = sq.part[m];
                            Hg[c] = make_float2(pr.x, pr.y);
                            wq[c] = make_float2(pr.z, pr.w);
                        } else {
                            Hg[c] = g[c];
                            wq[c] = yv;
                        }
                        const float2 sv = make_float2(sq.vr[2 * m].z, sq.vr[2 * m + 1].z);
                        const float2 wvv = make_float2(sq.vr[2 * m].w, sq.vr[2 * m + 1].w);
                        dk.x += sv.x * g[c].x + sv.y * g[c].y;
                        dk.y += wvv.x * g[c].x + wvv.y * g[c].y;
                        dk.z += sv.x * yv.x + sv.y * yv.y;
                        dk.w += wvv.x * yv.x + wvv.y * yv.y;
                    }
                }
                // (S + K) g and (S + K) y_Q
                if (hasK) {
                    dk = batch_sum4(dk);
#pragma unroll
                    for (int c = 0; c < kCPT; ++c) {
                        const int i = t0 + c * kDB;
                        if (act[c] && batc_of(c) == cb) {
                            const int m = sq.memb[i];
                            const float2 sv = make_float2(sq.vr[2 * m].z, sq.vr[2 * m + 1].z);
                            const float2 wvv = make_float2(sq.vr[2 * m].w, sq.vr[2 * m + 1].w);
                            Hg[c].x += -(wvv.x * dk.x + sv.x * dk.y) * ibK + a2K * sv.x * dk.x;
                            Hg[c].y += -(wvv.y * dk.x + sv.y * dk.y) * ibK + a2K * sv.y * dk.x;
                            wq[c].x += -(wvv.x * dk.z + sv.x * dk.w) * ibK + a2K * sv.x * dk.z;
                            wq[c].y += -(wvv.y * dk.z + sv.y * dk.w) * ibK + a2K * sv.y * dk.z;
                        }
                    }
                }
                int nf = fl & ~(kDnIdent | kDnK);
                if (!pass) nf |= kDnIdent;
                if (hasQ) {
                    // Q's update with w_Q = (S + K) y_Q; Q becomes K
                    float4 dq = make_float4(0.f, 0.f, 0.f, 0.f);  // y_Q'w_Q, s_Q'g, w_Q'g
                    float2 sqv[kCPT];
#pragma unroll
                    for (int c = 0; c < kCPT; ++c) {
                        sqv[c] = z2;
                        const int i = t0 + c * kDB;
                        if (act[c] && batc_of(c) == cb) {
                            const int m = sq.memb[i];
                            const float2 yv = make_float2(sq.vr[2 * m].y, sq.vr[2 * m + 1].y);
                            sqv[c] = sQ[m];
                            dq.x += yv.x * wq[c].x + yv.y * wq[c].y;
                            dq.y += sqv[c].x * g[c].x + sqv[c].y * g[c].y;
                            dq.z += wq[c].x * g[c].x + wq[c].y * g[c].y;
                        }
                    }
                    dq = batch_sum4(dq);
                    const float ibQ = 1.f / lane_value(bQ_v, cb);
                    const float a2Q = dq.x * ibQ * ibQ + ibQ;
#pragma unroll
                    for (int c = 0; c < kCPT; ++c) {
                        const int i = t0 + c * kDB;
                        if (act[c] && batc_of(c) == cb) {
                            const int m = sq.memb[i];
                            Hg[c].x += -(wq[c].x * dq.y + sqv[c].x * dq.z) * ibQ + a2Q * sqv[c].x * dq.y;
                            Hg[c].y += -(wq[c].y * dq.y + sqv[c].y * dq.z) * ibQ + a2Q * sqv[c].y * dq.y;
                            wK[m] = wq[c];
                        }
                    }
                    nf = (nf & ~(kDnQ | kDnSlot)) | kDnK | (ks ? 0 : kDnSlot);
                    ibK_v = ln == cb ? ibQ : ibK_v;
                    a2K_v = ln == cb ? a2Q : a2K_v;
                }
                dst_v = ln == cb ? nf : dst_v;
                float part = 0.f;
#pragma unroll
                for (int c = 0; c < kCPT; ++c) {
                    if (act[c] && batc_of(c) == cb) {
                        part += g[c].x * Hg[c].x + g[c].y * Hg[c].y;
                        p[c] = make_float2(-Hg[c].x, -Hg[c].y);
                    } else {
                        p[c] = z2;
                    }
                }
                gpv = -batch_sum4(make_float4(part, 0.f, 0.f, 0.f)).x;
            }
            return gpv;
        };
        // an accepted step with s'y > eps_curv y'y becomes the batch's Q
        auto dense_record = [&](float beta, const float2 (&s_)[kCPT], const float2 (&y_)[kCPT]) {
            if constexpr (DENSE) {
                const int t0 = (int)threadIdx.x, ln = t0 & (kWave - 1);
                const int d = 2 * sq.cnt[cb];
                float *V = Hbase + sq.voff[cb];
                const int fl = __builtin_amdgcn_readlane(dst_v, cb);
                float2 *sQ = reinterpret_cast<float2 *>(V + ((fl & kDnSlot) ? 0 : 1) * d);
                float2 *yQ = reinterpret_cast<float2 *>(V + 2 * d);
#pragma unroll
                for (int c = 0; c < kCPT; ++c) {
                    const int i = t0 + c * kDB;
                    if (act[c] && batc_of(c) == cb) {
                        const int m = sq.memb[i];
                        sQ[m] = s_[c];
                        yQ[m] = y_[c];
                    }
                }
                dst_v = ln == cb ? (fl | kDnQ) : dst_v;
                bQ_v = ln == cb ? beta : bQ_v;
            }
        };
        // H_p = I: nothing pending, S stands for I again
        auto dense_reset = [&]() {
            if constexpr (DENSE) {
                const int ln = (int)threadIdx.x & (kWave - 1);
                dst_v = ln == cb ? kDnIdent : dst_v;
            }
        };

        // Gram matrix of the updated basis: slot totals to LDS (every wave
        // that calls it writes the same bits), then each lane fills 7 of the
        // 21 x 21 entries of the other buffer, which becomes current
        auto gram_update = [&](float tot, int par, bool push, int lane) {
            const int nxt = cur ^ 1;
            sh.tot_s[par][lane] = tot;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // all reads before the writes, so that the LDS round trips of
            // the seven entries overlap (read-write pairs would serialise:
            // the two buffers of Bm are one array to the compiler)
            constexpr int kGR = (kNB * kNB + kWave - 1) / kWave;
            float gv[kGR];
#pragma unroll
            for (int r = 0; r < kGR; ++r) {
                const int ent = lane + kWave * r;
                const int src = sh.bsrc[push ? 1 : 0][ent < kNB * kNB ? ent : 0];
                const float *from = (src & 0x8000) ? &sh.tot_s[par][src & 0x7fff] : &sh.Bm[cur][src];
                gv[r] = *from;
            }
#pragma unroll
            for (int r = 0; r < kGR; ++r) {
                const int ent = lane + kWave * r;
                if (ent < kNB * kNB) sh.Bm[nxt][ent] = gv[r];
            }
            if constexpr (!SEQ) {
                // 1 / s_j'y_j follows the Gram entries (shifted on a push,
                // the newest from the new entry): the two-loop reads them
                // instead of dividing every iteration
                if (lane < kMM) {
                    const float keep = sh.rho[cur][lane < kMM - 1 ? lane + 1 : lane];
                    const float sy = lane_value(tot, sScYc);
                    sh.rho[nxt][lane] = !push ? sh.rho[cur][lane]
                                              : lane < kMM - 1 ? keep : 1.f / sy;
                }
            }
            cur = nxt;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        // Whole-instance descent: B is kept as a ring over the pair slots
        // (pair j of the basis at storage pair (hd + j) mod 10), so that an
        // update writes only the rows and columns of the vectors it changes
        // (g; on a push also the new s and y, stored over the evicted pair)
        // straight from the slot totals.  Storage index of basis vector a:
        auto ring_at = [&](int a) -> int {
            if (a == kG) return kG;
            const int base = a < kMM ? 0 : kMM;
            int q = a - base + hd;
            if (q >= kMM) q -= kMM;
            return base + q;
        };
        // the first of the two ring columns of storage slot c (g: its one column)
        auto ring_col = [](int c) -> int { return c < kMM ? c : c < kG ? c + kMM : 4 * kMM; };
        // batch descent, deciding wave: batch bb's saved Gram matrix (pair
        // order) into the ring, pair 0 at storage 0; and back.  ln: the lane
        // (from the loop's opaque thread id, so that no index stays live
        // across the loop)
        auto ring_load = [&](int bb, int ln) {
            if constexpr (SEQ && !DENSE) {
                hd = 0;
                constexpr int kQ = (kNB * kNB + kWave - 1) / kWave;
                float v[kQ];
#pragma unroll
                for (int q = 0; q < kQ; ++q) {
                    const int e = ln + kWave * q;
                    v[q] = e < kNB * kNB ? sq.BmP[bb][e] : 0.f;
                }
#pragma unroll
                for (int q = 0; q < kQ; ++q) {
                    const int e = ln + kWave * q;
                    if (e < kNB * kNB) {
                        const int r = e / kNB, c = e - r * kNB;       // storage = pair order
                        float *dst = &sh.Bring[r * kRS + ring_col(c)];
                        dst[0] = v[q];
                        if (c < kG) dst[kMM] = v[q];                   // the second copy
                    }
                }
            }
        };
        auto ring_save = [&](int bb, int ln) {
            if constexpr (SEQ && !DENSE) {
#pragma unroll
                for (int q = 0; q < (kNB * kNB + kWave - 1) / kWave; ++q) {
                    const int e = ln + kWave * q;
                    if (e < kNB * kNB) {
                        const int a = e / kNB, b2 = e - a * kNB;
                        sq.BmP[bb][e] = sh.Bring[ring_at(a) * kRS + ring_col(ring_at(b2))];
                    }
                }
            }
        };
        // Two-loop recursion on B. Lane l holds row l of B (the basis
        // s_0..s_9, y_0..y_9, g), so acc = (B c) for the current coefficient
        // vector c is one FMA per lane per step: q = g - sum_i a_i y_i gives
        // acc -= a_j B[l][y_j], r = gamma q + sum_j (a_j - b_j) s_j gives
        // acc += (a_j - b_j) B[l][s_j].  s_j'q and y_j'r are then single lanes
        // of acc (one readlane per step).  The per-pair scalars stay
        // lane-indexed in VGPRs (lane j: rho_j, a_j, the s_j coefficient; lane
        // 10 + j: rho_j and a_j again).  Returns g'p with p = -r; cs_v: the
        // coefficient of s_j at lane j; alph_v: a_j at lane j.
        auto two_loop_core = [&](int lane, const float (&Bc)[kNB], float rho_v, float &cs_out,
                                 float &alph_out, float &gam_out) -> float {
            const int jp = lane < kMM ? lane : lane - kMM;        // pair index of lanes 0..19
            float acc = Bc[kG];                                   // (B q)_l with q = g
            float alph_v = 0.f;                                   // a_j at lanes j and 10 + j
            // every pair slot in straight-line code: a slot without a pair
            // has rho = 0, so its a_j and coefficient are 0 and acc keeps its
            // bits (acc - 0 * B = acc for finite B)
#pragma unroll
            for (int j = kMM - 1; j >= 0; --j) {
                const float a = lane_value(rho_v * acc, j);         // rho_j s_j'q
                if (jp == j) alph_v = a;
                acc -= a * Bc[kMM + j];
            }
            float gam = 1.f;
            if (k > 0) {
                const float sy = lane_value(Bc[kMM - 1], 2 * kMM - 1);
                const float yy = lane_value(Bc[2 * kMM - 1], 2 * kMM - 1);
                gam = sy / yy;
            }
            acc *= gam;                                           // (B r)_l with r = gamma q
            float cs_v = 0.f;                                     // coefficient of s_j at lane j
#pragma unroll
            for (int j = 0; j < kMM; ++j) {
                const float c = lane_value(alph_v - rho_v * acc, kMM + j);   // a_j - rho_j y_j'r
                if (lane == j) cs_v = c;
                acc += c * Bc[j];
            }
            cs_out = cs_v;
            alph_out = alph_v;
            gam_out = gam;
            return -lane_value(acc, kG);                          // g'p = -g'r
        };
        // Loads this lane's row of B (pair order through the storage map at,
        // double-buffered form: hd = 0) and rho, then the recursion above.
        auto two_loop = [&](int lane, int hd, float &cs_out, float &alph_out, float &gam_out) -> float {
            // storage index of basis vector a
            auto at = [&](int a) -> int {
                if (a == kG) return kG;
                const int base = a < kMM ? 0 : kMM;
                int q = a - base + hd;
                if (q >= kMM) q -= kMM;
                return base + q;
            };
            // lanes past row 20 read row 20 again: their values are never read
            float Bc[kNB];
            const int lr = at(lane < kNB ? lane : kNB - 1);
#pragma unroll
            for (int a2 = 0; a2 < kNB; ++a2) Bc[a2] = sh.Bm[cur][at(a2) * kNB + lr];
            const int jp = lane < kMM ? lane : lane - kMM;        // pair index of lanes 0..19
            const bool live = lane < 2 * kMM && jp >= kMM - k;
            const int jq = lane < 2 * kMM ? jp : 0;               // in-range index on every lane
            float rho_v;
            if constexpr (SEQ) {
                rho_v = live ? 1.f / sh.Bm[cur][jq * kNB + kMM + jq] : 0.f;
            } else {
                rho_v = sh.rho[cur][at(jq)];
                rho_v = live ? rho_v : 0.f;
            }
            return two_loop_core(lane, Bc, rho_v, cs_out, alph_out, gam_out);
        };

        for (int q = tid; q < kNB * kNB; q += kDB) { sh.Bm[0][q] = 0.f; sh.Bm[1][q] = 0.f; }
        if constexpr (SOLO)
            for (int q = tid; q < kNB * kRS; q += kDB) sh.Bring[q] = 0.f;
        for (int q = tid; q < 2 * kMM; q += kDB) sh.rho[q / kMM][q % kMM] = 0.f;
        if (tid == 0) {
            sh.flag[0] = 1; sh.flag[1] = 0; sh.cell_evals = 0;
            sh.pos[kMaxN] = make_float2(kFarCoord, kFarCoord);
            sh.dk.tau64 = A.tau64; sh.dk.e_feasible = A.e_feasible;
            sh.dk.c1 = A.c1; sh.dk.eps_curv = A.eps_curv; sh.dk.ftol = A.ftol; sh.dk.g_tol_sq = A.g_tol_sq;
            sh.dk.m = A.m; sh.dk.max_halvings = A.max_halvings; sh.dk.max_iter = A.max_iter;
            sh.dk.g_tol = A.g_tol; sh.dk.nbat = A.nbat; sh.dk.anm = A.anm;
        }

        // container adjustment state (uniform): radius, its gradient and
        // search components, penalty coefficient; hR_v (deciding wave):
        // radius component of basis vector `lane`
        float Rz = R, gR = 0.f, pR = 0.f, lam = ADJ ? A.lambda0 : 0.f;
        float hR_v = 0.f;
        int iters_all = 0;
        for (int round = 0;; ++round) {
        if constexpr (ADJ) {
            if (round >= A.rounds) break;
            // fresh minimisation of U at this lambda; every wave has left
            // the previous round's reads of B before it is cleared
            __syncthreads();
            for (int q = tid; q < kNB * kNB; q += kDB) { sh.Bm[0][q] = 0.f; sh.Bm[1][q] = 0.f; }
            for (int q = tid; q < kNB * kRS; q += kDB) sh.Bring[q] = 0.f;
            for (int q = tid; q < 2 * kMM; q += kDB) sh.rho[q / kMM][q % kMM] = 0.f;
            k = 0; cur = 0; it = 0; itw = 0; hd = 0; h = 0; status = 0;
            req = kReqInit;
            hR_v = 0.f;
        }
        for (;;) {
            // Per-iteration opaque copies of the thread and lane ids: lane
            // predicates and LDS addresses are then recomputed inside the loop
            // (one VALU op each) instead of being hoisted and kept live as
            // dozens of SGPR masks and VGPR addresses, which spilled.
            int tid_l = (int)threadIdx.x;
            asm volatile("" : "+v"(tid_l));
            const int tid = tid_l, lane = tid_l & (kWave - 1);
            // ================= one evaluation ==================================
            float2 xt[kCPT], sc[kCPT];
            const int par = tcount & 1;
            // batch descent: only the current batch is swept (masked); the
            // evaluation at the top of an outer iteration covers every
            // circle and always takes the FP64 energies
            const bool masked = SEQ && visits && req != kReqTotal;
            const bool want64 = fp64 || (SEQ && req == kReqTotal);
            // the FP32 energy of unit circles decides the switch into the
            // FP64 regime and nothing else
            const bool want_e1 = !ADJ && !fp64;
            bool inb[kCPT];
#pragma unroll
            for (int c = 0; c < kCPT; ++c) inb[c] = !masked || batc_of(c) == cb;
            // container radius of this evaluation (a variable only when adjusting)
            const float Rt = ADJ ? (req == kReqTrial ? fmaf(alpha, pR, Rz) : Rz) : R;
#pragma unroll
            for (int c = 0; c < kCPT; ++c) {
                xt[c] = req == kReqTrial ? make_float2(fmaf(alpha, p[c].x, x[c].x), fmaf(alpha, p[c].y, x[c].y))
                                         : x[c];
                sc[c] = make_float2(xt[c].x - x[c].x, xt[c].y - x[c].y);
                if (act[c]) {
                    sh.pos[tid + c * kDB] = xt[c];
                    const double dx = (double)xt[c].x - (double)xr[c].x;
                    const double dy = (double)xt[c].y - (double)xr[c].y;
                    if (!(SEQ && A.anm) && dx * dx + dy * dy > A.skin2) sh.flag[par] = 1;
                }
            }
            __syncthreads();                                            // B1
            if (tid == 0) sh.flag[par ^ 1] = 0;
            if (sh.flag[par]) {
                // ---- neighbor list rebuild at the positions in sh.pos -------
                if (tid == 0) sh.over = 0;    // set again below only after bin_circles' barriers
                if (tid <= kMaxSeqBatches) sh.npair[tid] = 0;
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
                // ELL slots; more than ELL switches this list epoch to
                // sweeping the cell grid instead
                int up_c[kCPT] = {};
#pragma unroll
                for (int c = 0; c < kCPT; ++c) {
                    const int i = tid + c * kDB;
                    // the candidates are the circles of the 3 x 3 cells
                    // around the circle's own, in cell order: three cell rows
                    // (start, length), read together, indexed as one run
                    int ra[3], rl[3];
                    {
                        const int cx = cell_coord(xt[c].x, grid), cy = cell_coord(xt[c].y, grid);
                        const int y0 = cy > 0 ? cy - 1 : 0, y1 = cy < grid.nc - 1 ? cy + 1 : grid.nc - 1;
                        const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < grid.nc - 1 ? cx + 1 : grid.nc - 1;
#pragma unroll
                        for (int r = 0; r < 3; ++r) {
                            const bool row = act[c] && y0 + r <= y1;
                            const int yy = y0 + r <= y1 ? y0 + r : y0;
                            const int a = sh.cell_start[yy * grid.nc + x0];
                            const int z = sh.cell_start[yy * grid.nc + x1 + 1];
                            ra[r] = row ? a : 0;
                            rl[r] = row ? z - a : 0;
                        }
                    }
                    const int K = rl[0] + rl[1] + rl[2];
                    // the wave walks its longest run, four candidates per
                    // step with their index and position reads in flight
                    const int kmax = wave_max_dpp(K);
                    int m = 0, up = 0;
                    for (int k0 = 0; k0 < kmax; k0 += 4) {
                        int jv[4];
                        bool ok[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int k = k0 + u;
                            ok[u] = k < K;
                            const int t = k < rl[0]         ? ra[0] + k
                                        : k < rl[0] + rl[1] ? ra[1] + (k - rl[0])
                                                            : ra[2] + (k - rl[0] - rl[1]);
                            const int jj = sh.cell_circ[ok[u] ? t : 0];
                            jv[u] = ok[u] ? jj : i;
                        }
                        float2 pv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) pv[u] = sh.pos[jv[u]];
                        // the FP32 test decides outside a band of +-1e-5
                        // around the cutoff, the FP64 one inside it (the
                        // near_cut predicate; the band is rare, so one uniform
                        // branch covers the wave's four candidates)
                        bool nb[4], band[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const float dx = xt[c].x - pv[u].x, dy = xt[c].y - pv[u].y;
                            const float l2 = dx * dx + dy * dy;
                            const bool cand = ok[u] && jv[u] != i;
                            nb[u] = cand && l2 < c2lo;
                            band[u] = cand && l2 >= c2lo && l2 <= c2hi;
                        }
                        if (__builtin_amdgcn_ballot_w64(band[0] || band[1] || band[2] || band[3])) {
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                if (band[u]) nb[u] = near64(xt[c], pv[u], A.c2);
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (nb[u] && m < ELL) sh.list[m][i] = (uint16_t)(jv[u] * (int)sizeof(float2));
                            m += nb[u] ? 1 : 0;
                            up += (nb[u] && jv[u] > i) ? 1 : 0;
                        }
                    }
                    if (act[c]) {
                        if (m > ELL) sh.over = 1;
                        sh.list_n[i] = (uint8_t)(m < ELL ? m : ELL);
                        up_c[c] = up;
                        xr[c] = xt[c];
                    }
                }
                // listed pairs from their lower index, per wave, then one
                // integer add per wave (the same totals in any order): in all,
                // and per batch for the batch descent
                {
                    const int wsum = wave_sum_int(up_c[0] + up_c[1]);
                    if (lane == 0) atomicAdd(&sh.npair[kMaxSeqBatches], wsum);
                    if constexpr (SEQ) {
                        for (int q = 0; q < A.nbat; ++q) {
                            int v = 0;
#pragma unroll
                            for (int c = 0; c < kCPT; ++c) v += (act[c] && batc_of(c) == q) ? up_c[c] : 0;
                            v = wave_sum_int(v);
                            if (lane == 0 && v != 0) atomicAdd(&sh.npair[q], v);
                        }
                    }
                }
                // pad every list with the far point up to the longest list
                // of the wave (the sweep's trip count; circles past n count
                // as empty lists)
                {
                    int mlen[kCPT], mw = 0;
#pragma unroll
                    for (int c = 0; c < kCPT; ++c) {
                        mlen[c] = act[c] ? (int)sh.list_n[tid + c * kDB] : 0;
                        mw = mlen[c] > mw ? mlen[c] : mw;
                    }
                    mw = wave_max_dpp(mw);
#pragma unroll
                    for (int c = 0; c < kCPT; ++c)
                        for (int t = mlen[c]; t < mw; ++t) sh.list[t][tid + c * kDB] = (uint16_t)kFarOff;
                }
                ++rebuilds;
                __syncthreads();
                overflow = sh.over != 0;
            }
            ++tcount;
            ++evals;
            // evaluations over the cell grid, counted in LDS (no register
            // stays live for a number read once at the end)
            if (overflow && tid == 0) ++sh.cell_evals;
            pair_mine += __builtin_amdgcn_readfirstlane(sh.npair[masked ? cb : kMaxSeqBatches]);
            // ---- pair sweep: energy and gradient of this thread's circles ----
            // Both circles of the thread walk their lists in one loop, so their
            // list and position reads overlap; each circle still adds its
            // terms in list order.
            float e = 0.f, e1 = 0.f;
            double eo = 0.0, et = 0.0;
            float2 gt[kCPT], yc[kCPT];
            float ecA[kCPT], e1cA[kCPT], gxA[kCPT], gyA[kCPT];
            double eocA[kCPT], etcA[kCPT];
#pragma unroll
            for (int c = 0; c < kCPT; ++c) {
                ecA[c] = e1cA[c] = gxA[c] = gyA[c] = 0.f;
                eocA[c] = etcA[c] = 0.0;
            }
            if (!overflow) {
                // trip count: the longest swept list of the wave (uniform);
                // shorter lists are padded with the far point
                bool use[kCPT];
                int mm = 0;
#pragma unroll
                for (int c = 0; c < kCPT; ++c) {
                    use[c] = act[c] && inb[c];
                    const int mcc = use[c] ? (int)sh.list_n[tid + c * kDB] : 0;
                    mm = mcc > mm ? mcc : mm;
                }
                mm = wave_max_dpp(mm);
                // one copy of the loop per (unit-circle energy, FP64 terms)
                // regime, so neither costs instructions where it is off.  The
                // list entries of slot t + 1 are read while slot t is summed,
                // so a slot waits for one LDS read (its partners) instead of
                // two in a chain.
                auto sweep = [&](auto e1_tag, auto w64_tag) {
                    constexpr bool kE1 = decltype(e1_tag)::value, kW64 = decltype(w64_tag)::value;
                    int jn[kCPT];                      // byte offsets into pos, next slot
#pragma unroll
                    for (int c = 0; c < kCPT; ++c) jn[c] = sh.list[0][tid + c * kDB];
                    for (int t = 0; t < mm; ++t) {
                        int jv[kCPT];
                        float2 pj[kCPT];
                        const int tn = t + 1 < ELL ? t + 1 : ELL - 1;
#pragma unroll
                        for (int c = 0; c < kCPT; ++c) {
                            if constexpr (SEQ) {
                                // batch visit: circles outside the batch take the far point
                                jv[c] = sh.list[t][tid + c * kDB];
                                if (masked) jv[c] = use[c] ? jv[c] : kFarOff;
                            } else {
                                jv[c] = jn[c];
                                jn[c] = sh.list[tn][tid + c * kDB];
                            }
                        }
#pragma unroll
                        for (int c = 0; c < kCPT; ++c)
                            pj[c] = *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(sh.pos) + jv[c]);
#pragma unroll
                        for (int c = 0; c < kCPT; ++c) {
                            const int i = tid + c * kDB;
                            const int jb = jv[c];
                            const float2 q = xt[c];
                            // each pair once: from its lower index, or (batch
                            // energy, Eq. 7) from the batch's end
                            bool hf = jb > i * (int)sizeof(float2);
                            if constexpr (SEQ) {
                                const int jj = jb / (int)sizeof(float2);
                                if (masked) hf = hf || sq.bat[jj < kMaxN ? jj : kMaxN - 1] != cb;
                            }
                            float l2;
                            const float il = pair_term32s(q, pj[c], hf, two_r, four_r2, four_r2_band,
                                                          ecA[c], e1cA[c], gxA[c], gyA[c], l2, kE1);
                            // FP64 energies only where FP32 sees (nearly) an overlap:
                            // outside a 1e-5 band the FP64 terms are zero
                            if (kW64 && hf && l2 < four_r2_band)
                                pair_term64s(q, pj[c], l2 * il, il, two_r64, four_r2_64, eocA[c], etcA[c]);
                        }
                    }
                };
                using T_ = std::true_type;
                using F_ = std::false_type;
                if (want64) {
                    if (want_e1) sweep(T_{}, T_{}); else sweep(F_{}, T_{});
                } else {
                    if (want_e1) sweep(T_{}, F_{}); else sweep(F_{}, F_{});
                }
            }
#pragma unroll
            for (int c = 0; c < kCPT; ++c) {
                const int i = tid + c * kDB;
                const float2 q = xt[c];
                // the list sweep's sums carry the pair terms divided by -2
                float gx = -2.f * gxA[c], gy = -2.f * gyA[c];
                if (act[c] && inb[c]) {
                    float ec = ecA[c], e1c = e1cA[c];
                    double eoc = eocA[c], etc = etcA[c];
                    if (overflow) {
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
                                bool hf = j > i;
                                if constexpr (SEQ) if (masked) hf = hf || sq.bat[j] != cb;
                                pair_term32(q, pj, hf, two_r, four_r2, ec, e1c, gx, gy);
                                if (want64 && hf) {
                                    const float dx = q.x - pj.x, dy = q.y - pj.y;
                                    if (dx * dx + dy * dy < four_r2_band)
                                        pair_term64(q, pj, two_r64, four_r2_64, eoc, etc);
                                }
                            }
                        }
                    }
                    e += ec;
                    if constexpr (!ADJ) e1 += e1c;
                    eo += eoc;
                    et += etc;
                    // containment (branch-free, as the pair term)
                    const float r2 = q.x * q.x + q.y * q.y;
                    const float ir = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
                    const float d0 = fmaxf(r2 * ir + rad - Rt, 0.f);
                    e += d0 * d0;
                    if constexpr (ADJ) {
                        e1 += d0;                     // sum of d_i0: dU/dR
                    } else {
                        const float d01 = fmaxf(d0 - (rad - 1.f), 0.f);
                        e1 += d01 * d01;
                    }
                    const float kc = 2.f * d0 * ir;
                    gx += kc * q.x;
                    gy += kc * q.y;
                    if (want64) {
                        const double r64 =
                            sqrt64_from32((double)q.x * q.x + (double)q.y * q.y, r2 * ir, ir);
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
                yc[c] = inb[c] ? make_float2(gx - g[c].x, gy - g[c].y) : make_float2(0.f, 0.f);
            }
            // ---- fused reduction: 63 dot products and E in one pass ----------
            const float wsum = wave_reduce_scatter(gt, sc, yc, S, Y, e, e1);
            sh.red[par][wv][lane_slot(lane)] = wsum;
            if (want64) {
                const double wo = wave_sum_dpp(eo), wt = wave_sum_dpp(et);
                if (lane == 0) { sh.red64[par][wv][0] = wo; sh.red64[par][wv][1] = wt; }
            }
            __syncthreads();                                            // B2
            if constexpr (SOLO) {
                // ---- one wave decides ----------------------------------------
                // The uniform chain (slot totals, line search, Gram matrix,
                // stop tests, two-loop) runs on wave 0 alone: on every wave it
                // would share each SIMD with a copy of itself.  The outcome
                // reaches the other waves through LDS behind one barrier.
                if (wv == 0) {
                    auto ufl = [](float v) { return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v))); };
                    auto udb = [](double v) {
                        const long long b = __builtin_bit_cast(long long, v);
                        const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
                        const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
                        return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
                    };
                    const float c1 = ufl(sh.dk.c1), eps_curv = ufl(sh.dk.eps_curv), ftol = ufl(sh.dk.ftol);
                    const float g_tol_sq = ufl(sh.dk.g_tol_sq);
                    const double tau64 = udb(sh.dk.tau64), e_feasible = udb(sh.dk.e_feasible);
                    const int mm = __builtin_amdgcn_readfirstlane(sh.dk.m);
                    const int max_halvings = __builtin_amdgcn_readfirstlane(sh.dk.max_halvings);
                    const int max_iter = __builtin_amdgcn_readfirstlane(sh.dk.max_iter);
                    // source slots of this lane's Gram update (read early)
                    const uint32_t pa = sh.bperm[lane];
                    float tot = 0.f;
#pragma unroll
                    for (int w = 0; w < kDW; ++w) tot += sh.red[par][w][lane];
                    double so = 0.0, st = 0.0;
                    if (want64) {
                        // lane w of every group of eight holds wave w's FP64
                        // sums; a fixed tree over the eight (pairs, quads,
                        // halves), read from lane 0
                        const int wl = lane & (kDW - 1);
                        double vo = sh.red64[par][wl][0], vt = sh.red64[par][wl][1];
                        vo += dpp64<kDppXor1>(vo);
                        vt += dpp64<kDppXor1>(vt);
                        vo += dpp64<kDppXor2>(vo);
                        vt += dpp64<kDppXor2>(vt);
                        vo += dpp64<kDppHalfMirror>(vo);
                        vt += dpp64<kDppHalfMirror>(vt);
                        so = lane_value64(vo, 0);
                        st = lane_value64(vt, 0);
                    }
                    // container adjustment: the radius components of the reduced
                    // dot products (lane L holds slot L, whose operands are
                    // (trial gradient | step | change of gradient) and (a basis
                    // vector | one of those three)); hR_v: the radius component
                    // of basis vector `lane`, kept by this wave
                    float gRt = 0.f, scR = 0.f, ycR = 0.f;
                    if constexpr (ADJ) {
                        gRt = -2.f * lane_value(tot, sE1) + 2.f * lam * Rt;   // dU/dR at the trial
                        scR = Rt - Rz;
                        ycR = gRt - gR;
                        const int L = lane;
                        int bsel = 0;
                        float uR = 0.f;
                        if (L < 2 * kMM) { bsel = L; uR = gRt; }                                   // gt . s_j, gt . y_j
                        else if (L < 3 * kMM - 1) { bsel = L - 2 * kMM + 1; uR = scR; }            // sc . s_j
                        else if (L < 4 * kMM - 2) { bsel = kMM + L - (3 * kMM - 1) + 1; uR = scR; } // sc . y_j
                        else if (L < 5 * kMM - 3) { bsel = L - (4 * kMM - 2) + 1; uR = ycR; }      // yc . s_j
                        else if (L < 6 * kMM - 4) { bsel = kMM + L - (5 * kMM - 3) + 1; uR = ycR; } // yc . y_j
                        const float vR = __builtin_bit_cast(
                            float, __builtin_amdgcn_ds_bpermute(4 * bsel, __builtin_bit_cast(int, hR_v)));
                        float corr = uR * vR;
                        if (L == sGG) corr = gRt * gRt;
                        else if (L == sScSc) corr = scR * scR;
                        else if (L == sScYc) corr = scR * ycR;
                        else if (L == sYcYc) corr = ycR * ycR;
                        else if (L == sScG) corr = scR * gRt;
                        else if (L == sYcG) corr = ycR * gRt;
                        else if (L == sE) corr = lam * Rt * Rt;               // U = E + lambda R^2
                        else if (L == sE1) corr = 0.f;
                        tot += corr;
                    }
                    const float Et = lane_value(tot, sE);
                    const float E1t = lane_value(tot, sE1);
                    // batch descent: more than one batch, visited in turn
                    const bool vis = SEQ && visits;
                    int fl = 0;
                    bool accept = false, push = false;
                    bool vend = false;         // batch descent: the visit ends with this evaluation
                    if (vis && req == kReqTotal) {
                        // ---- top of an outer iteration: stop tests on the
                        // whole instance (FP64 energies of every circle), then
                        // the first batch's visit
                        E_tot = Et;
                        E64o = so;
                        E64t = st;
                        const double Eacc = fp64 ? E64o : (double)E_tot;
                        const bool dtl = ftol > 0.f && it >= W && decreased_too_little(Eacc, (it - W) % (W + 1), ftol);
                        status = !isfinite(E_tot)                          ? 6
                               : E64t < e_feasible                         ? 1
                               : (it > 0 && gsum_prev <= ufl(sh.dk.g_tol))  ? 2
                               : dtl                                        ? 3
                               : (it > 0 && nvis > 0 && nstall == nvis)     ? 4
                               : it >= max_iter                             ? 5 : 0;
                        if (lane == it % (W + 1)) ehist = Eacc;
                        if (status != 0) {
                            fl = kDecStop;
                        } else {
                            if (!fp64 && tau64 > 0.0 && (double)fminf(E_tot, E1t) < tau64) fp64 = true;
                            gsum = 0.f;
                            nvis = 0;
                            nstall = 0;
                            cb = first_b;
                            ring_load(cb, lane);
                            k = __builtin_amdgcn_readlane(kb_v, cb);
                            req = kReqInit;
                            fl = kDecNext;
                        }
                    } else {
                        if (req == kReqTrial) {
                            const bool ok = fp64 ? so <= E64o + (double)c1 * (double)alpha * (double)gp
                                                 : Et <= E + c1 * alpha * gp;
                            if (ok) {
                                accept = true;
                                const float sy = lane_value(tot, sScYc), yy = lane_value(tot, sYcYc);
                                push = sy > eps_curv * yy;
                                vend = vis;
                            } else {
                                alpha *= 0.5f;
                                if (++h > max_halvings) {
                                    if (!vis) { status = 4; fl = kDecStop; }   // STALLED
                                    else { vend = true; ++nstall; }           // the batch stays
                                } else {
                                    fl = kDecNext;
                                }
                            }
                        } else if (req == kReqInit) {
                            accept = true;   // g and the g row of B from this evaluation
                        } else {             // kReqFp64: FP64 energies of the current point
                            E64o = so;
                            E64t = st;
                        }
                        if (accept) {
                            fl = kDecAccept | (push ? kDecPush : 0);
                            // ---- Gram update, written into the ring before its
                            // rows are read below (LDS keeps a wave's order).
                            // Lane l (pair order of the updated basis) takes its
                            // entries <g, b_l> and, on a push, <s, b_l> and
                            // <y, b_l> of the new pair from the slot totals.
                            const int hd_old = hd;
                            if (push) {
                                hd = hd == kMM - 1 ? 0 : hd + 1;
                                k = k + 1 > mm ? mm : k + 1;
                            }
                            const int ti = __builtin_bit_cast(int, tot);
                            const float vg = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(
                                                 (int)__builtin_amdgcn_ubfe(pa, push ? 8u : 0u, 8u), ti));
                            const int sto = ring_at(lane < kNB ? lane : kG);      // storage slot of b_l
                            const int c0 = ring_col(sto);
                            const int c1c = sto < kG ? c0 + kMM : c0;             // its two columns
                            float *rowl = &sh.Bring[sto * kRS];
                            if (lane < kNB) {
                                sh.Bring[kG * kRS + c0] = vg;
                                sh.Bring[kG * kRS + c1c] = vg;
                                rowl[4 * kMM] = vg;
                            }
                            if (push) {
                                const float vs = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(
                                                     (int)__builtin_amdgcn_ubfe(pa, 16u, 8u), ti));
                                const float vy = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(
                                                     (int)__builtin_amdgcn_ubfe(pa, 24u, 8u), ti));
                                if (lane < kNB) {
                                    sh.Bring[hd_old * kRS + c0] = vs;
                                    sh.Bring[hd_old * kRS + c1c] = vs;
                                    sh.Bring[(kMM + hd_old) * kRS + c0] = vy;
                                    sh.Bring[(kMM + hd_old) * kRS + c1c] = vy;
                                    rowl[hd_old] = vs;
                                    rowl[kMM + hd_old] = vs;
                                    rowl[2 * kMM + hd_old] = vy;
                                    rowl[3 * kMM + hd_old] = vy;
                                }
                                if (!SEQ && lane == 0) sh.rho[0][hd_old] = 1.f / lane_value(tot, sScYc);
                            }
                            if constexpr (ADJ) {
                                if (push) {             // shift the radius components like S and Y
                                    const int L = lane;
                                    const int src = (L < kMM - 1 || (L >= kMM && L < 2 * kMM - 1)) ? L + 1 : L;
                                    float v = __builtin_bit_cast(
                                        float, __builtin_amdgcn_ds_bpermute(4 * src, __builtin_bit_cast(int, hR_v)));
                                    if (L == kMM - 1) v = scR;
                                    if (L == 2 * kMM - 1) v = ycR;
                                    hR_v = v;
                                }
                                Rz = Rt;
                                gR = gRt;
                            }
                            if (req == kReqTrial && !vis) {
                                ++it;
                                itw = itw == W ? 0 : itw + 1;
                            }
                            E = Et;
                            if (fp64) { E64o = so; E64t = st; }
                            // FP64 regime once either FP32 energy is small (not
                            // when adjusting: U > 0 and no FEASIBLE stop)
                            if (!ADJ && !vis && !fp64 && tau64 > 0.0 && (double)fminf(E, E1t) < tau64) {
                                fp64 = true;
                                req = kReqFp64;          // FP64 energies of x before going on
                                fl |= kDecNext;
                            }
                        }
                        if constexpr (SEQ) {
                            const int nbat = __builtin_amdgcn_readfirstlane(sh.dk.nbat);
                            const bool anm = __builtin_amdgcn_readfirstlane(sh.dk.anm) != 0;
                            if (vend) {
                                // ---- end of a visit: the batch's Gram matrix and
                                // history count are saved, then the next batch
                                kb_v = lane == cb ? k : kb_v;
                                ring_save(cb, lane);
                                int nx = cb + 1;
                                while (nx < nbat && sq.cnt[nx] == 0) ++nx;
                                if (nx >= nbat) {           // outer iteration done
                                    ++it;
                                    gsum_prev = gsum;
                                    // ANM (Alg. 3) by every wave after the barrier
                                    if (anm && anm_tick()) fl |= kDecAnm;
                                    req = kReqTotal;
                                } else {
                                    cb = nx;
                                    ring_load(cb, lane);
                                    k = __builtin_amdgcn_readlane(kb_v, cb);
                                    req = kReqInit;
                                }
                                fl |= kDecNext;
                            } else if (!vis && anm && it > anm_it && !(fl & (kDecNext | kDecStop))) {
                                // one batch: ANM after every iteration; the point
                                // is evaluated again over the lists it leaves
                                anm_it = it;
                                if (anm_tick()) {
                                    fl |= kDecAnm | kDecNext;
                                    req = kReqInit;
                                }
                            }
                        }
                        if (!(fl & (kDecNext | kDecStop))) {
                            // ---- top of an iteration: stop tests, direction
                            // |g| <= g_tol and |g| finite, decided on |g|^2 (no
                            // square root: g_tol_sq is the largest value whose
                            // square root is at most g_tol).  The tests are
                            // selects and the two-loop runs before their outcome
                            // is looked at, so both chains share the issue slots.
                            // A batch visit has no stop test of its own: its
                            // gradient norm joins the outer iteration's sum.
                            const float gg = accept ? lane_value(tot, sGG) : sh.Bring[kG * kRS + 4 * kMM];
                            const float gg0 = fmaxf(gg, 0.f);
                            if (vis) {
                                gsum += sqrtf(gg0);
                                ++nvis;
                                status = 0;
                            } else {
                                const double Eacc = fp64 ? E64o : (double)E;
                                const int itn = itw == W ? 0 : itw + 1;       // (it + 1) mod (W + 1)
                                const bool dtl = ftol > 0.f && it >= W && decreased_too_little(Eacc, itn, ftol);
                                status = (!isfinite(E) || !isfinite(gg0)) ? 6
                                       : (fp64 && E64t < e_feasible)      ? 1
                                       : gg0 <= g_tol_sq                   ? 2
                                       : dtl                               ? 3
                                       : it >= max_iter                    ? 5 : 0;
                                if (lane == itw) ehist = Eacc;                // read above before written
                            }
                            // this lane's row of the updated B in pair order:
                            // contiguous from offset hd in the ring row
                            float Bc[kNB];
                            const int jp = lane < kMM ? lane : lane - kMM;
                            const bool live = lane < 2 * kMM && jp >= kMM - k;
                            float rho_l;
                            {
                                const float *row = &sh.Bring[ring_at(lane < kNB ? lane : kG) * kRS + hd];
#pragma unroll
                                for (int j = 0; j < kMM; ++j) {
                                    Bc[j] = row[j];
                                    Bc[kMM + j] = row[2 * kMM + j];
                                }
                                Bc[kG] = row[4 * kMM - hd];
                                if constexpr (SEQ) {
                                    // 1 / s_j'y_j from the row (no store of it per batch):
                                    // lane j reads <s_j, y_j>, lane 10 + j <y_j, s_j>
                                    rho_l = 1.f / row[lane < kMM ? 2 * kMM + lane : (lane < 2 * kMM ? lane - kMM : 0)];
                                } else {
                                    rho_l = sh.rho[0][ring_at(lane < 2 * kMM ? jp : 0)];
                                }
                            }
                            float cs_v, alph_v, gam;
                            const float gpv = two_loop_core(lane, Bc, live ? rho_l : 0.f, cs_v, alph_v, gam);
                            if (status != 0) {
                                fl |= kDecStop;
                            } else {
                                gp = gpv;
                                if constexpr (ADJ) {
                                    // radius component of the direction
                                    const float cy_v = -gam * alph_v;
                                    float pr = -gam * gR;
#pragma unroll
                                    for (int j = 0; j < kMM; ++j)
                                        pr -= lane_value(cs_v, j) * lane_value(hR_v, j) +
                                              lane_value(cy_v, j) * lane_value(hR_v, kMM + j);
                                    pR = pr;
                                }
                                if (k > 0 && !(gp < 0.f)) {
                                    k = 0;
                                    gp = -gg;
                                    fl |= kDecSteepest;
                                    if constexpr (ADJ) pR = -gR;
                                }
                                if (k > 0) alpha = 1.f;
                                else alpha = 1.f / fmaxf(1.f, sqrtf(gg0));
                                h = 0;
                                req = kReqTrial;
                                if (lane < kMM) {
                                    sh.coef[0][lane] = cs_v;
                                    sh.coef[1][lane] = -gam * alph_v;
                                }
                                if (lane == 0) sh.dec_gam = gam;
                            }
                        }
                    }
                    if (lane == 0) {
                        sh.dec_flags = fl;
                        sh.dec_req = req;
                        sh.dec_fp64 = fp64 ? 1 : 0;
                        sh.dec_alpha = alpha;
                        sh.dec_cb = cb;
                        if constexpr (ADJ) { sh.dec_Rz = Rz; sh.dec_pR = pR; }
                    }
                }
                __syncthreads();                                        // B3
                const int fl = __builtin_amdgcn_readfirstlane(sh.dec_flags);
                req = __builtin_amdgcn_readfirstlane(sh.dec_req);
                fp64 = __builtin_amdgcn_readfirstlane(sh.dec_fp64) != 0;
                alpha = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(
                                                      __builtin_bit_cast(int, sh.dec_alpha)));
                if constexpr (SEQ) cb = __builtin_amdgcn_readfirstlane(sh.dec_cb);
                if constexpr (ADJ) {
                    Rz = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, sh.dec_Rz)));
                    pR = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, sh.dec_pR)));
                }
                if (fl & kDecAccept) {
                    const bool push = (fl & kDecPush) != 0;
#pragma unroll
                    for (int c = 0; c < kCPT; ++c) {
                        // a batch visit's pair belongs to the batch's circles
                        if (push && inb[c]) {
#pragma unroll
                            for (int j = 0; j < kMM - 1; ++j) { S[j][c] = S[j + 1][c]; Y[j][c] = Y[j + 1][c]; }
                            S[kMM - 1][c] = __builtin_bit_cast(double, sc[c]);
                            Y[kMM - 1][c] = __builtin_bit_cast(double, yc[c]);
                        }
                        x[c] = xt[c];
                        g[c] = gt[c];
                    }
                }
                if constexpr (SEQ)
                    if (fl & kDecAnm) anm_compare();                    // every wave
                if (fl & kDecStop) break;
                if (fl & kDecNext) continue;
                // ---- direction p = -(gamma g + sum_j cs_j s_j + cy_j y_j),
                // zero outside the visited batch
                if (fl & kDecSteepest) {
#pragma unroll
                    for (int c = 0; c < kCPT; ++c)
                        p[c] = (!SEQ || !visits || batc_of(c) == cb) ? make_float2(-g[c].x, -g[c].y)
                                                                  : make_float2(0.f, 0.f);
                } else {
                    const float gam = sh.dec_gam;
#pragma unroll
                    for (int c = 0; c < kCPT; ++c) {
                        float px = -gam * g[c].x, py = -gam * g[c].y;
#pragma unroll
                        for (int j = 0; j < kMM; ++j) {
                            const float csj = sh.coef[0][j], cyj = sh.coef[1][j];
                            px -= csj * as_f2(S[j][c]).x + cyj * as_f2(Y[j][c]).x;
                            py -= csj * as_f2(S[j][c]).y + cyj * as_f2(Y[j][c]).y;
                        }
                        p[c] = (!SEQ || !visits || batc_of(c) == cb) ? make_float2(px, py)
                                                                  : make_float2(0.f, 0.f);
                    }
                }
                continue;
            }
            float tot = 0.f;
#pragma unroll
            for (int w = 0; w < kDW; ++w) tot += sh.red[par][w][lane];
            double so = 0.0, st = 0.0;
            if (want64) {
#pragma unroll
                for (int w = 0; w < kDW; ++w) { so += sh.red64[par][w][0]; st += sh.red64[par][w][1]; }
            }
            const float Et = lane_value(tot, sE);
            const float E1t = lane_value(tot, sE1);

            // ================= what the evaluation was for =====================
            if constexpr (SEQ) {
                if (visits && req == kReqTotal) {
                    // ---- top of an outer iteration: stop tests on the whole instance
                    E_tot = Et;
                    E64o = so;
                    E64t = st;
                    const double Eacc = fp64 ? E64o : (double)E_tot;
                    if (!isfinite(E_tot)) { status = 6; break; }
                    if (E64t < A.e_feasible) { status = 1; break; }
                    if (it > 0 && gsum_prev <= A.g_tol) { status = 2; break; }
                    if (A.ftol > 0.f && it >= W && decreased_too_little(Eacc, (it - W) % (W + 1), A.ftol)) { status = 3; break; }
                    if (lane == it % (W + 1)) ehist = Eacc;
                    if (it > 0 && nvis > 0 && nstall == nvis) { status = 4; break; }
                    if (it >= A.max_iter) { status = 5; break; }
                    if (!fp64 && A.tau64 > 0.0 && (double)fminf(E_tot, E1t) < A.tau64) fp64 = true;
                    gsum = 0.f;
                    nvis = 0;
                    nstall = 0;
                    cb = first_b;
                    k = __builtin_amdgcn_readlane(kb_v, cb);
                    req = kReqInit;
                    continue;
                }
            }
            bool accept = false, push = false;
            bool vend = false;     // batch descent: the visit ends with this evaluation
            if (req == kReqTrial) {
                const bool ok = fp64 ? so <= E64o + (double)A.c1 * (double)alpha * (double)gp
                                     : Et <= E + A.c1 * alpha * gp;
                if (ok) {
                    accept = true;
                    const float sy = lane_value(tot, sScYc), yy = lane_value(tot, sYcYc);
                    push = sy > A.eps_curv * yy;
                    vend = SEQ && visits;
                } else {
                    alpha *= 0.5f;
                    if (++h > A.max_halvings) {
                        if (!(SEQ && visits)) { status = 4; break; }   // STALLED
                        vend = true;                                   // the batch stays
                        ++nstall;
                    } else {
                        continue;
                    }
                }
            } else if (req == kReqInit) {
                accept = true;   // g and the g row of B from this evaluation
            } else {             // kReqFp64: FP64 energies of the current point
                E64o = so;
                E64t = st;
            }
            if (accept) {
                gram_update(tot, par, push, lane);
#pragma unroll
                for (int c = 0; c < kCPT; ++c) {
                    if (!DENSE && push && inb[c]) {
#pragma unroll
                        for (int j = 0; j < kMM - 1; ++j) { S[j][c] = S[j + 1][c]; Y[j][c] = Y[j + 1][c]; }
                        S[kMM - 1][c] = __builtin_bit_cast(double, sc[c]);
                        Y[kMM - 1][c] = __builtin_bit_cast(double, yc[c]);
                    }
                    x[c] = xt[c];
                    g[c] = gt[c];
                }
                if (push) k = k + 1 > A.m ? A.m : k + 1;
                if (req == kReqTrial && !(SEQ && visits)) ++it;   // visits: outer iterations
                E = Et;
                if (fp64) { E64o = so; E64t = st; }
                // FP64 regime once either FP32 energy is small: with a contact
                // margin the unit circles can be overlap-free while E (radius
                // rad) still sums (2 mu)^2 over every contact
                if (!(SEQ && visits) && !fp64 && A.tau64 > 0.0 &&
                    (double)fminf(E, E1t) < A.tau64) {
                    fp64 = true;
                    req = kReqFp64;          // FP64 energies of x before going on
                    continue;
                }
            }

            if constexpr (SEQ) {
                if (visits && vend) {
                    // ---- end of a visit (this path's batch mode is the dense
                    // one): record the accepted pair, then the next batch
                    kb_v = lane == cb ? k : kb_v;
                    if (push) dense_record(lane_value(tot, sScYc), sc, yc);
                    int nx = cb + 1;
                    while (nx < A.nbat && sq.cnt[nx] == 0) ++nx;
                    if (nx >= A.nbat) {           // outer iteration done
                        ++it;
                        gsum_prev = gsum;
                        if (A.anm) anm_step();
                        req = kReqTotal;
                        continue;
                    }
                    cb = nx;
                    k = __builtin_amdgcn_readlane(kb_v, cb);
                    req = kReqInit;
                    continue;
                }
                if (!visits && A.anm && it > anm_it) {
                    // one batch: ANM after every iteration; changed lists
                    // re-evaluate the current point over the new lists
                    anm_it = it;
                    if (anm_step()) { req = kReqInit; continue; }
                }
            }

            // ================= top of an iteration: stop tests =================
            const float gg = sh.Bm[cur][kG * kNB + kG];
            const float gn = sqrtf(fmaxf(gg, 0.f));
            if (SEQ && visits) {
                // a visit's first evaluation: its gradient norm joins the sum
                gsum += gn;
                ++nvis;
            } else {
                const double Eacc = fp64 ? E64o : (double)E;
                if (!isfinite(E) || !isfinite(gn)) { status = 6; break; }
                if (fp64 && E64t < A.e_feasible) { status = 1; break; }
                if (gn <= A.g_tol) { status = 2; break; }
                if (A.ftol > 0.f && it >= W && decreased_too_little(Eacc, (it - W) % (W + 1), A.ftol)) { status = 3; break; }
                if (lane == it % (W + 1)) ehist = Eacc;
                if (it >= A.max_iter) { status = 5; break; }
            }

            if constexpr (DENSE) {
                // ================= direction: p = -H_p g (Eq. 8) ==================
                gp = dense_direction();
            } else {
                // ================= direction: two-loop recursion on B ===============
                float cs_v, alph_v, gam;
                gp = two_loop(lane, 0, cs_v, alph_v, gam);
                {
                    const float cy_v = -gam * alph_v;                 // coefficient of y_j at lane j
    #pragma unroll
                    for (int c = 0; c < kCPT; ++c) {
                        float px = -gam * g[c].x, py = -gam * g[c].y;
    #pragma unroll
                        for (int j = 0; j < kMM; ++j) {
                            const float csj = lane_value(cs_v, j), cyj = lane_value(cy_v, j);
                            px -= csj * as_f2(S[j][c]).x + cyj * as_f2(Y[j][c]).x;
                            py -= csj * as_f2(S[j][c]).y + cyj * as_f2(Y[j][c]).y;
                        }
                        p[c] = (!SEQ || !visits || batc_of(c) == cb) ? make_float2(px, py)
                                                                  : make_float2(0.f, 0.f);
                    }
                }
            }
            if (k > 0 && !(gp < 0.f)) {
                k = 0;
                if constexpr (DENSE) dense_reset();
#pragma unroll
                for (int c = 0; c < kCPT; ++c)
                    p[c] = (!SEQ || !visits || batc_of(c) == cb) ? make_float2(-g[c].x, -g[c].y)
                                                              : make_float2(0.f, 0.f);
                gp = -gg;
            }
            if (k > 0) alpha = 1.f;
            else alpha = 1.f / fmaxf(1.f, gn);
            h = 0;
            req = kReqTrial;
        }
        iters_all += it;
        if constexpr (!ADJ) break;
        if (status == 6) break;                  // NONFINITE ends the adjustment
        lam *= 0.5f;
        }   // rounds

        // ---- write back ------------------------------------------------------
#pragma unroll
        for (int c = 0; c < kCPT; ++c)
            if (act[c]) reinterpret_cast<float2 *>(xy)[off + tid + c * kDB] = x[c];
        if (tid == 0) {
            DescentHead r;
            r.status = status;
            r.iters = iters_all;
            r.evals = evals;
            r.rebuilds = rebuilds;
            r.pair_evals = pair_mine;
            // with the radius as a variable, E reports the energy without
            // the penalty (the last lambda was halved once more after the round)
            r.E32 = (ADJ && A.rounds > 0) ? E - 2.f * lam * Rz * Rz : E;
            r.gnorm = sqrtf(fmaxf(SOLO ? sh.Bring[kG * kRS + 4 * kMM] : sh.Bm[cur][kG * kNB + kG], 0.f));
            r.E64 = fp64 ? E64t : -1.0;
            if (SEQ && visits) {
                // outer iterations; whole-instance energies; the sum of the
                // batch gradient norms of the last outer iteration
                r.E32 = E_tot;
                r.gnorm = gsum_prev;
                r.E64 = E64t;
            }
            store_result(out, b, r, sh.cell_evals);
            if constexpr (ADJ) Rout[b] = Rz;
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
    static std::atomic<int> per_cu[kMaxDevices];
    const int cap = current_device_cus() * resident_per_cu(lbfgs_descend_kernel<kModeWhole>, kDB, per_cu);
    return B < cap ? B : cap;
}

hipError_t launch_queue_init(const int32_t *offset, int B, int32_t *queue, hipStream_t s)
{
    queue_init_kernel<<<1, kQB, 0, s>>>(offset, B, queue);
    return hipGetLastError();
}

hipError_t launch_descend(const int32_t *offset, const float *R, const double *R64, float *xy,
                          int B, int64_t total_n, const DescentArgs &a, void *out,
                          int32_t *queue, int grid, hipStream_t s)
{
    queue_init_kernel<<<1, kQB, 0, s>>>(offset, B, queue);
    if (grid < 1) grid = 1;
    lbfgs_descend_kernel<kModeWhole><<<grid, kDB, 0, s>>>(offset, R, R64, xy, B, total_n, a,
                                                          reinterpret_cast<DescentResultDev *>(out),
                                                          queue, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

// The descent's only scratch memory is its work queue (a counter and the
// instance order, B + 1 int32).  For callers that cannot allocate, the
// library keeps one queue per device in a fixed array: kNoAllocMaxInstances
// + 1 words (256 KiB), held by every device the library runs on until the
// process ends.  Host code never passes the array's name to a kernel (in host
// code it is a stand-in, not a device address): the device address comes
// from hipGetSymbolAddress, taken once per device with that device current.
// The queue is set by a kernel at every call (queue_init_kernel), so nothing
// carries over from the previous call; calls that overlap on one device
// share the array and race.
static __device__ __align__(256) int32_t scratch[kNoAllocMaxInstances + 1];

namespace {
std::atomic<int32_t *> g_scratch_ptr[kMaxDevices];

// The array's device address on the current device (looked up once per device).
hipError_t noalloc_queue(int32_t **queue)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    int32_t *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        e = hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev].store(p, std::memory_order_release);   // the same value from any thread
    }
    *queue = p;
    return hipSuccess;
}
}  // namespace

hipError_t launch_descend_noalloc(const int32_t *offset, const float *R, const double *R64,
                                  float *xy, int B, int64_t total_n, const DescentArgs &a,
                                  void *out, int grid, hipStream_t s)
{
    if (B > kNoAllocMaxInstances) return hipErrorInvalidValue;
    int32_t *queue = nullptr;
    const hipError_t e = noalloc_queue(&queue);
    if (e != hipSuccess) return e;
    return launch_descend(offset, R, R64, xy, B, total_n, a, out, queue, grid, s);
}

hipError_t launch_adjust(const int32_t *offset, const float *R, float *xy, int B,
                         int64_t total_n, const DescentArgs &a, float *Rout, void *out,
                         int32_t *queue, int grid, hipStream_t s)
{
    queue_init_kernel<<<1, kQB, 0, s>>>(offset, B, queue);
    if (grid < 1) grid = 1;
    lbfgs_descend_kernel<kModeAdj><<<grid, kDB, 0, s>>>(offset, R, nullptr, xy, B, total_n, a,
                                                        reinterpret_cast<DescentResultDev *>(out),
                                                        queue, Rout, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_seq(const int32_t *offset, const float *R, const double *R64, float *xy, int B,
                      int64_t total_n, const DescentArgs &a, const int32_t *batch_of, void *out,
                      int32_t *queue, int grid, hipStream_t s)
{
    queue_init_kernel<<<1, kQB, 0, s>>>(offset, B, queue);
    if (grid < 1) grid = 1;
    lbfgs_descend_kernel<kModeSeq><<<grid, kDB, 0, s>>>(offset, R, R64, xy, B, total_n, a,
                                                        reinterpret_cast<DescentResultDev *>(out),
                                                        queue, nullptr, batch_of, nullptr);
    return hipGetLastError();
}

hipError_t launch_dense(const int32_t *offset, const float *R, const double *R64, float *xy,
                        int B, int64_t total_n, const DescentArgs &a, const int32_t *batch_of,
                        float *H, void *out, int32_t *queue, int grid, hipStream_t s)
{
    queue_init_kernel<<<1, kQB, 0, s>>>(offset, B, queue);
    if (grid < 1) grid = 1;
    lbfgs_descend_kernel<kModeDense><<<grid, kDB, 0, s>>>(offset, R, R64, xy, B, total_n, a,
                                                          reinterpret_cast<DescentResultDev *>(out),
                                                          queue, nullptr, batch_of, H);
    return hipGetLastError();
}

}  // namespace pecc
