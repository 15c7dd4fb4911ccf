// Persistent L-BFGS descent of the elastic energy at fixed container radius.
//
// Mapping (one workgroup of 1024 threads per instance, n <= 1024):
//   * thread t owns circle t: its position, gradient, search direction and
//     its 2 coordinates of every stored curvature pair (s_j, y_j) live in
//     registers, so the L-BFGS history never leaves the chip;
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

constexpr int kDB = 1024;                 // threads per workgroup
constexpr int kDW = kDB / kWave;          // waves per workgroup
constexpr int kMM = 10;                   // history slots (max m)
constexpr int kNB = 2 * kMM + 1;          // basis size: s_0..s_9, y_0..y_9, g
constexpr int kListCap = 12 * kMaxN;      // neighbor entries held in LDS
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
constexpr int sE = sGG + 6;                                 // trial energy
static_assert(sE < kWave, "fused reduction must fit one slot per lane");

struct DescentShared {
    float2 pos[kMaxN];
    int cell_start[kMaxCells + 1];
    uint16_t cell_circ[kMaxN];
    uint16_t slot_tmp[kMaxN];
    uint16_t list[kListCap];
    uint16_t list_start[kMaxN + 1];
    float red[2][kDW][kWave];
    double red64[2][kDW][2];
    float Bm[2][kNB * kNB];
    int scan_tmp[kDW + 1];
    int flag[2];
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

// Value of reduction slot v for this thread's circle (v is a constant after
// unrolling, so the branches fold away).
__device__ __forceinline__ float slot_value(int v, float2 gt, float2 sc, float2 yc,
                                            const float2 (&S)[kMM], const float2 (&Y)[kMM],
                                            float e)
{
    if (v < kMM) return dot2(gt, S[v]);
    if (v < 2 * kMM) return dot2(gt, Y[v - kMM]);
    if (v < 3 * kMM - 1) return dot2(sc, S[v - 2 * kMM + 1]);
    if (v < 4 * kMM - 2) return dot2(sc, Y[v - (3 * kMM - 1) + 1]);
    if (v < 5 * kMM - 3) return dot2(yc, S[v - (4 * kMM - 2) + 1]);
    if (v < 6 * kMM - 4) return dot2(yc, Y[v - (5 * kMM - 3) + 1]);
    if (v == sGG) return dot2(gt, gt);
    if (v == sScSc) return dot2(sc, sc);
    if (v == sScYc) return dot2(sc, yc);
    if (v == sYcYc) return dot2(yc, yc);
    if (v == sScG) return dot2(sc, gt);
    if (v == sYcG) return dot2(yc, gt);
    if (v == sE) return e;
    return 0.0f;
}

// Reduce-scatter of the 64 slot values over the wave: afterwards lane L
// holds the wave sum of slot L.
__device__ __forceinline__ float wave_reduce_scatter(float2 gt, float2 sc, float2 yc,
                                                     const float2 (&S)[kMM],
                                                     const float2 (&Y)[kMM], float e)
{
    const int lane = threadIdx.x & (kWave - 1);
    float h[32];
    const bool up32 = (lane & 32) != 0;
#pragma unroll
    for (int v = 0; v < 32; ++v) {
        const float a = slot_value(v, gt, sc, yc, S, Y, e);
        const float b = slot_value(v + 32, gt, sc, yc, S, Y, e);
        const float mine = up32 ? b : a, other = up32 ? a : b;
        h[v] = mine + __shfl_xor(other, 32, kWave);
    }
#pragma unroll
    for (int o = 16; o >= 1; o >>= 1) {
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int v = 0; v < o; ++v) {
            const float a = h[v], b = h[v + o];
            const float mine = up ? b : a, other = up ? a : b;
            h[v] = mine + __shfl_xor(other, o, kWave);
        }
    }
    return h[0];
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

__global__ __launch_bounds__(kDB) void lbfgs_descend_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ Rv, float *__restrict__ xy,
    int B, int64_t total_n, DescentArgs A, DescentResultDev *__restrict__ out,
    int32_t *__restrict__ queue)
{
    __shared__ DescentShared sh;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;

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
        const bool act = tid < n;
        const float rad = A.rad, two_r = 2.0f * rad, four_r2 = two_r * two_r;
        const double rad64 = (double)rad, two_r64 = 2.0 * rad64, four_r2_64 = two_r64 * two_r64;
        const double R64 = (double)R;
        const Grid grid = make_grid(R, A.h_req);

        // ---- per-thread state ------------------------------------------------
        float2 x = act ? reinterpret_cast<const float2 *>(xy)[off + tid] : make_float2(0.f, 0.f);
        float2 g = make_float2(0.f, 0.f);
        float2 xr = x;
        float2 S[kMM], Y[kMM];
#pragma unroll
        for (int j = 0; j < kMM; ++j) { S[j] = make_float2(0.f, 0.f); Y[j] = make_float2(0.f, 0.f); }
        int k = 0;                     // valid pairs, slots kMM-k .. kMM-1
        int cur = 0;                   // Bm buffer in use
        int tcount = 0;                // evaluations so far (flag parity)
        bool overflow = false;         // list did not fit: sweep the cell grid
        int half_pairs = 0;            // listed pairs i<j since the last rebuild
        int rebuilds = 0, evals = 0;
        int64_t pair_evals = 0;
        bool fp64 = false;
        double E64o = 0.0, E64t = -1.0;   // FP64 energies (objective / unit circles)
        float E = 0.0f;
        double ehist = 0.0;               // lane w holds the energy of iteration w mod (W+1)
        int status = 0, it = 0;

        for (int q = tid; q < kNB * kNB; q += kDB) { sh.Bm[0][q] = 0.f; sh.Bm[1][q] = 0.f; }
        if (tid == 0) { sh.flag[0] = 1; sh.flag[1] = 0; }
        // (barrier: first thing inside evaluate)

        // ---- neighbor list rebuild at the positions in sh.pos ----------------
        auto rebuild = [&]() {
            bin_circles<kDB>(sh.pos, n, grid, sh.cell_start, sh.cell_circ, sh.slot_tmp,
                             sh.scan_tmp);
            int cnt = 0;
            const float2 pi = act ? sh.pos[tid] : make_float2(0.f, 0.f);
            if (act)
                for_each_candidate(tid, pi, grid, sh.cell_start, sh.cell_circ, [&](int j) {
                    if (near64(pi, sh.pos[j], A.c2)) ++cnt;
                });
            int total;
            const int start = block_exclusive_scan<kDB>(cnt, sh.scan_tmp, &total);
            overflow = total > kListCap;
            half_pairs = total / 2;
            if (act) {
                sh.list_start[tid] = (uint16_t)(overflow ? 0 : start);
                if (!overflow) {
                    int w = start;
                    for_each_candidate(tid, pi, grid, sh.cell_start, sh.cell_circ, [&](int j) {
                        if (near64(pi, sh.pos[j], A.c2)) sh.list[w++] = (uint16_t)j;
                    });
                    for (int a = start + 1; a < w; ++a) {   // ascending j
                        const uint16_t key = sh.list[a];
                        int z = a - 1;
                        while (z >= start && sh.list[z] > key) { sh.list[z + 1] = sh.list[z]; --z; }
                        sh.list[z + 1] = key;
                    }
                }
                xr = pi;
            }
            if (tid == 0) sh.list_start[n] = (uint16_t)(overflow ? 0 : total);
            ++rebuilds;
            __syncthreads();
        };

        // ---- one evaluation at xt: energy, gradient, fused reduction ---------
        // Returns the slot total held by this lane (lane L: slot L); gt gets
        // the trial gradient; e64o/e64t the FP64 energies when fp64.
        auto evaluate = [&](float2 xt, float2 sc, float2 &gt, double &e64o, double &e64t) -> float {
            const int par = tcount & 1;
            if (act) {
                sh.pos[tid] = xt;
                const double dx = (double)xt.x - (double)xr.x, dy = (double)xt.y - (double)xr.y;
                if (dx * dx + dy * dy > A.skin2) sh.flag[par] = 1;
            }
            __syncthreads();                                        // B1
            if (tid == 0) sh.flag[par ^ 1] = 0;
            if (sh.flag[par]) rebuild();
            ++tcount;
            ++evals;
            pair_evals += half_pairs;
            float e = 0.f;
            double eo = 0.0, et = 0.0;
            float gx = 0.f, gy = 0.f;
            if (act) {
                auto pair = [&](int j) {
                    const float2 pj = sh.pos[j];
                    const float dx = xt.x - pj.x, dy = xt.y - pj.y;
                    const float l2 = dx * dx + dy * dy;
                    if (l2 < four_r2) {
                        const float l = sqrtf(l2);
                        const float d = two_r - l;
                        if (j > tid) e += d * d;
                        if (l > 0.f) {
                            const float kf = -2.f * d / l;
                            gx += kf * dx;
                            gy += kf * dy;
                        }
                    }
                    if (fp64 && j > tid) {
                        const double ex = (double)xt.x - (double)pj.x, ey = (double)xt.y - (double)pj.y;
                        const double m2 = ex * ex + ey * ey;
                        if (m2 < four_r2_64) {
                            const double l = sqrt(m2);
                            const double d = two_r64 - l;
                            eo += d * d;
                            if (m2 < 4.0) { const double dt = 2.0 - l; et += dt * dt; }
                        }
                    }
                };
                if (!overflow) {
                    const int a = sh.list_start[tid], z = sh.list_start[tid + 1];
                    for (int q = a; q < z; ++q) pair(sh.list[q]);
                } else {
                    for_each_candidate(tid, xt, grid, sh.cell_start, sh.cell_circ, pair);
                }
                const float rho = sqrtf(xt.x * xt.x + xt.y * xt.y);
                const float d0 = rho + rad - R;
                if (d0 > 0.f) {
                    e += d0 * d0;
                    if (rho > 0.f) {
                        const float kc = 2.f * d0 / rho;
                        gx += kc * xt.x;
                        gy += kc * xt.y;
                    }
                }
                if (fp64) {
                    const double r64 = sqrt((double)xt.x * xt.x + (double)xt.y * xt.y);
                    const double c0 = r64 + rad64 - R64;
                    if (c0 > 0.0) eo += c0 * c0;
                    const double ct = r64 + 1.0 - R64;
                    if (ct > 0.0) et += ct * ct;
                }
                // E sums over every circle: a non-finite position makes it NaN
                if (!(isfinite(xt.x) && isfinite(xt.y))) {
                    e = __builtin_nanf("");
                    eo = et = __builtin_nan("");
                }
            }
            gt = make_float2(gx, gy);
            const float2 yc = make_float2(gx - g.x, gy - g.y);
            const float wsum = wave_reduce_scatter(gt, sc, yc, S, Y, e);
            sh.red[par][wv][lane] = wsum;
            if (fp64) {
                const double wo = wave_sum(eo), wt = wave_sum(et);
                if (lane == 0) { sh.red64[par][wv][0] = wo; sh.red64[par][wv][1] = wt; }
            }
            __syncthreads();                                        // B2
            float tot = 0.f;
#pragma unroll
            for (int w = 0; w < kDW; ++w) tot += sh.red[par][w][lane];
            if (fp64) {
                double so = 0.0, st = 0.0;
#pragma unroll
                for (int w = 0; w < kDW; ++w) { so += sh.red64[par][w][0]; st += sh.red64[par][w][1]; }
                e64o = so;
                e64t = st;
            }
            return tot;
        };

        // ---- Gram-matrix update after an accepted step (every wave) ----------
        auto update_B = [&](float tot, bool push) {
            const int nxt = cur ^ 1;
            // every lane takes part in the shuffles: slot totals sit in all 64 lanes
            const int col = lane < kNB ? lane : 0;
            int ol = 0;
            const int kl = new_basis_kind(col, push, &ol);
#pragma unroll
            for (int a = 0; a < kNB; ++a) {
                int oa = 0;
                const int ka = new_basis_kind(a, push, &oa);
                int sl;
                if (ka == 0 && kl == 0) sl = -1;
                else if (ka == 0) sl = slot_new_old(kl, oa);
                else if (kl == 0) sl = slot_new_old(ka, ol);
                else sl = slot_new_new(ka, kl);
                const float vs = __shfl(tot, sl < 0 ? 0 : sl, kWave);
                if (lane < kNB) {
                    const float vo = sh.Bm[cur][oa * kNB + ol];
                    sh.Bm[nxt][a * kNB + lane] = sl < 0 ? vo : vs;
                }
            }
            cur = nxt;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };

        // ---- initial evaluation ----------------------------------------------
        {
            float2 gt;
            double eo = 0.0, et = 0.0;
            const float tot = evaluate(x, make_float2(0.f, 0.f), gt, eo, et);
            g = gt;
            E = __shfl(tot, sE, kWave);
            update_B(tot, false);
            if (E < (float)A.tau64 && A.tau64 > 0.0) {
                fp64 = true;
                float2 g2;
                const float t2 = evaluate(x, make_float2(0.f, 0.f), g2, eo, et);
                (void)t2;
                E64o = eo;
                E64t = et;
            }
        }

        const int W = A.ftol_window;
        for (;; ++it) {
            const float gg = sh.Bm[cur][kG * kNB + kG];
            const float gn = sqrtf(fmaxf(gg, 0.f));
            const double Eacc = fp64 ? E64o : (double)E;
            if (!isfinite(E) || !isfinite(gn)) { status = 6; break; }
            if (fp64 && E64t < A.e_feasible) { status = 1; break; }
            if (gn <= A.g_tol) { status = 2; break; }
            if (A.ftol > 0.f && it >= W) {
                const double eold = __shfl(ehist, (it - W) % (W + 1), kWave);
                if (eold - Eacc <= (double)A.ftol * eold) { status = 3; break; }
            }
            if (lane == it % (W + 1)) ehist = Eacc;
            if (it >= A.max_iter) { status = 5; break; }

            // ---- direction: two-loop recursion on the Gram matrix -----------
            float Bc[kNB];
#pragma unroll
            for (int a = 0; a < kNB; ++a) Bc[a] = lane < kNB ? sh.Bm[cur][a * kNB + lane] : 0.f;
            float dl = lane == kG ? 1.f : 0.f;
            float alph[kMM], rhoj[kMM];
#pragma unroll
            for (int j = kMM - 1; j >= 0; --j) {
                alph[j] = 0.f;
                rhoj[j] = 0.f;
                if (j >= kMM - k) {
                    const float sy = __shfl(Bc[j], kMM + j, kWave);
                    rhoj[j] = 1.f / sy;
                    const float a = rhoj[j] * wave_sum(dl * Bc[j]);
                    alph[j] = a;
                    if (lane == kMM + j) dl -= a;
                }
            }
            if (k > 0) {
                const float sy = __shfl(Bc[kMM - 1], 2 * kMM - 1, kWave);
                const float yy = __shfl(Bc[2 * kMM - 1], 2 * kMM - 1, kWave);
                dl *= sy / yy;
            }
#pragma unroll
            for (int j = 0; j < kMM; ++j) {
                if (j >= kMM - k) {
                    const float bb = rhoj[j] * wave_sum(dl * Bc[kMM + j]);
                    if (lane == j) dl += alph[j] - bb;
                }
            }
            float gp = -wave_sum(dl * Bc[kG]);
            float2 p;
            {
                const float cg = __shfl(dl, kG, kWave);
                float px = -cg * g.x, py = -cg * g.y;
#pragma unroll
                for (int j = 0; j < kMM; ++j) {
                    const float cs = __shfl(dl, j, kWave), cy = __shfl(dl, kMM + j, kWave);
                    px -= cs * S[j].x + cy * Y[j].x;
                    py -= cs * S[j].y + cy * Y[j].y;
                }
                p = make_float2(px, py);
            }
            if (k > 0 && !(gp < 0.f)) {
                k = 0;
                p = make_float2(-g.x, -g.y);
                gp = -gg;
            }

            // ---- backtracking line search ------------------------------------
            float alpha = k > 0 ? 1.f : 1.f / fmaxf(1.f, gn);
            bool accepted = false;
            float2 xt = x, gt = g;
            float tot = 0.f, Et = E;
            double eo = 0.0, et = 0.0;
            for (int h = 0; h <= A.max_halvings; ++h) {
                xt = make_float2(fmaf(alpha, p.x, x.x), fmaf(alpha, p.y, x.y));
                const float2 sc = make_float2(xt.x - x.x, xt.y - x.y);
                tot = evaluate(xt, sc, gt, eo, et);
                Et = __shfl(tot, sE, kWave);
                bool ok;
                if (fp64) ok = eo <= E64o + (double)A.c1 * (double)alpha * (double)gp;
                else ok = Et <= E + A.c1 * alpha * gp;
                if (ok) { accepted = true; break; }
                alpha *= 0.5f;
            }
            if (!accepted) {
                // restore the accepted positions for the final write-back
                status = 4;
                break;
            }
            // ---- accept: curvature pair, history, Gram matrix ----------------
            const float sy = __shfl(tot, sScYc, kWave), yy = __shfl(tot, sYcYc, kWave);
            const bool push = sy > A.eps_curv * yy;
            update_B(tot, push);
            if (push) {
                const float2 sc = make_float2(xt.x - x.x, xt.y - x.y);
                const float2 yc = make_float2(gt.x - g.x, gt.y - g.y);
#pragma unroll
                for (int j = 0; j < kMM - 1; ++j) { S[j] = S[j + 1]; Y[j] = Y[j + 1]; }
                S[kMM - 1] = sc;
                Y[kMM - 1] = yc;
                k = k + 1 > A.m ? A.m : k + 1;
            }
            x = xt;
            g = gt;
            E = Et;
            if (fp64) { E64o = eo; E64t = et; }
            if (!fp64 && A.tau64 > 0.0 && (double)E < A.tau64) {
                fp64 = true;
                float2 g2;
                const float t2 = evaluate(x, make_float2(0.f, 0.f), g2, eo, et);
                (void)t2;
                E64o = eo;
                E64t = et;
            }
        }

        // ---- write back ------------------------------------------------------
        if (act) reinterpret_cast<float2 *>(xy)[off + tid] = x;
        if (tid == 0) {
            DescentResultDev r;
            r.status = status;
            r.iters = it;
            r.evals = evals;
            r.rebuilds = rebuilds;
            r.pair_evals = pair_evals;
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

hipError_t launch_descend(const int32_t *offset, const float *R, float *xy, int B,
                          int64_t total_n, const DescentArgs &a, void *out, int32_t *queue,
                          int grid, hipStream_t s)
{
    queue_init_kernel<<<1, kQB, 0, s>>>(offset, B, queue);
    if (grid < 1) grid = 1;
    lbfgs_descend_kernel<<<grid, kDB, 0, s>>>(offset, R, xy, B, total_n, a,
                                              reinterpret_cast<DescentResultDev *>(out), queue);
    return hipGetLastError();
}

}  // namespace pecc
