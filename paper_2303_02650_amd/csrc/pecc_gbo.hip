// Geometric batch descent (Alg. 1 with the limited-memory reading of
// Eq. 8-11 and the batch energy of Eq. 7) for batches of instances, one
// persistent launch.
//
// Mapping (one workgroup of 256 threads = 4 waves per instance):
//   * the circles are partitioned once, at the start, into the blocks of a
//     blocks x blocks grid over [-R, R]^2 (computed in FP64 on the input
//     positions); block (bx, by) has colour (bx mod 2) + 2 (by mod 2), so
//     blocks of one colour never touch;
//   * an outer iteration visits the colours 0..3 in turn; inside a colour
//     the 4 waves take its batches, one batch per wave at a time, and run one
//     quasi-Newton iteration each, entirely inside the wave: the batch's
//     circles sit on the lanes (up to 128, two per lane), its curvature
//     history is loaded into registers, its Gram matrix into a wave-private
//     LDS area, and every reduction is a wave reduction -- no workgroup
//     barrier inside a visit;
//   * the other circles are seen at their positions from the start of the
//     colour (the batches of a colour run concurrently); the batch's own
//     trial positions live in a separate LDS array;
//   * neighbor lists (cutoff 2 rad + 2 skin) are rebuilt after a colour once
//     some circle has moved more than skin / 2 from the positions of the
//     last rebuild, so every circle starts a colour within skin / 2 of them.
//     A trial that keeps the batch's circles within skin of those positions
//     is evaluated over the lists; a longer trial (the step of Alg. 1 is not
//     limited) over the cell grid of the last rebuild for the other circles
//     (still within skin / 2 of their cells' positions, so the 3 x 3 cells
//     around the trial position hold every partner closer than 2 rad) and
//     over all of the batch's own circles;
//   * per-batch history (a ring of m pairs) and Gram matrix persist between
//     visits in the caller's workspace (L2-resident per instance).
// Results are bitwise reproducible: membership, list order and every sum
// are functions of the positions only.
#include "pecc_device.hpp"
#include "pecc_host.hpp"
#include "pecc_launch.hpp"
#include "pecc_lbfgs.hpp"

namespace pecc {

constexpr int kGT = 256;                    // threads per workgroup
constexpr int kGW = kGT / kWave;            // waves
constexpr int kGCPB = 2;                    // circles per lane inside a batch
constexpr int kGEll = 24;                   // neighbor slots per circle
constexpr int kMaxGboBatch = kWave * kGCPB; // circles per batch at most
constexpr int kMaxGboBatches = 64;          // blocks x blocks, blocks <= 8

struct GboShared {
    float2 pos[kMaxN];                      // positions at the start of the colour
    float2 tpos[kMaxN];                     // trial positions of visited batches
    float2 npos[kMaxN];                     // positions after the colour
    float2 xref[kMaxN];                     // positions at the last rebuild
    int cell_start[kMaxCells + 1];
    uint16_t cell_circ[kMaxN];
    uint16_t slot_tmp[kMaxN];
    uint16_t list[kGEll][kMaxN];
    uint8_t list_n[kMaxN];
    uint8_t batch_of[kMaxN];
    uint16_t members[kMaxN];                // circles grouped by batch, ascending
    int bstart[kMaxGboBatches + 1];
    uint8_t colour_batches[4][kMaxGboBatches];
    int ncolour[4];
    float Bw[kGW][2][kNB * kNB];            // per-wave Gram matrix, double-buffered
    float totw[kGW][kWave];                 // per-wave slot totals
    uint16_t bsrc[2][kNB * kNB];
    float redf[2][kGW];
    double redd[2][kGW];
    int scan_tmp[kGW + 1];
    int evw[kGW];                           // per-wave evaluation counts at the end
    int flag, over, bad, work;
};

struct GboBatchState {   // in the workspace, per batch
    int k, head;
};

// Workspace of one instance: history S and Y (rings of kMM pairs of up to
// kMaxGboBatch circles), Gram matrices and ring state of every batch.
__host__ __device__ inline size_t gbo_instance_bytes(int nbat)
{
    const size_t b = (size_t)nbat * (2 * (size_t)kMM * kMaxGboBatch * sizeof(float2) +
                                     (size_t)kNB * kNB * sizeof(float) + sizeof(GboBatchState));
    return (b + 255) & ~(size_t)255;
}

template <bool F64>
__global__ __launch_bounds__(kGT) void gbo_descend_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ Rv,
    const double *__restrict__ Rv64, float *__restrict__ xy, int B, int64_t total_n,
    DescentArgs A, int blocks, DescentResultDev *__restrict__ out, int32_t *__restrict__ queue,
    unsigned char *__restrict__ wsb)
{
    __shared__ GboShared sh;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int nbat = blocks * blocks;
    for (int q = tid; q < 2 * kNB * kNB; q += kGT)
        sh.bsrc[q / (kNB * kNB)][q % (kNB * kNB)] = gram_source(q % (kNB * kNB), q >= kNB * kNB);
    const float c2lo = (float)(A.c2 * (1.0 - 1e-5)), c2hi = (float)(A.c2 * (1.0 + 1e-5));

    for (;;) {
        __syncthreads();
        if (tid == 0) sh.work = atomicAdd(&queue[0], 1);
        __syncthreads();
        const int slot = sh.work;
        if (slot >= B) break;
        const int b = queue[1 + slot];
        const int off = offset[b], n = offset[b + 1] - off;
        const float R = Rv[b];
        const double R64 = Rv64 ? Rv64[b] : (double)R;
        auto bad_instance = [&]() {
            if (tid == 0) {
                DescentHead r = {};
                r.status = 7;
                r.E32 = __builtin_nanf("");
                r.gnorm = __builtin_nanf("");
                r.E64 = -1.0;
                store_result(out, b, r, 0);
            }
        };
        if (!(off >= 0 && n >= 0 && n <= kMaxN && (int64_t)off + n <= total_n)) {
            bad_instance();
            continue;
        }
        const float rad = A.rad, two_r = 2.0f * rad, four_r2 = two_r * two_r;
        const double two_r64 = 2.0 * (double)rad, four_r2_64 = two_r64 * two_r64;
        const Grid grid = make_grid(R, A.h_req);
        unsigned char *wsi = wsb + (size_t)b * gbo_instance_bytes(nbat);
        float2 *histS = reinterpret_cast<float2 *>(wsi);
        float2 *histY = histS + (size_t)nbat * kMM * kMaxGboBatch;
        float *gram = reinterpret_cast<float *>(histY + (size_t)nbat * kMM * kMaxGboBatch);
        GboBatchState *bst = reinterpret_cast<GboBatchState *>(gram + (size_t)nbat * kNB * kNB);

        // ---- load, partition (FP64, from the input positions) ------------------
        if (tid == 0) { sh.bad = 0; sh.flag = 1; }
        for (int i = tid; i < n; i += kGT) {
            const float2 p = reinterpret_cast<const float2 *>(xy)[off + i];
            sh.pos[i] = p;
            sh.npos[i] = p;
            const double S = 2.0 * (double)R / blocks;
            const double tx = floor(((double)p.x + (double)R) / S), ty = floor(((double)p.y + (double)R) / S);
            int bx = tx >= 0.0 ? (tx < blocks - 1 ? (int)tx : blocks - 1) : 0;
            int by = ty >= 0.0 ? (ty < blocks - 1 ? (int)ty : blocks - 1) : 0;
            sh.batch_of[i] = (uint8_t)(by * blocks + bx);
        }
        for (int e = tid; e < nbat * kNB * kNB; e += kGT) gram[e] = 0.f;
        for (int p = tid; p < nbat; p += kGT) { bst[p].k = 0; bst[p].head = 0; }
        __syncthreads();
        // members, ascending inside a batch: one thread per batch
        for (int p = tid; p < nbat; p += kGT) {
            int c = 0;
            for (int i = 0; i < n; ++i) c += sh.batch_of[i] == p;
            sh.bstart[p + 1] = c;
        }
        __syncthreads();
        if (tid == 0) {
            sh.bstart[0] = 0;
            for (int p = 0; p < nbat; ++p) {
                sh.bstart[p + 1] += sh.bstart[p];
                if (sh.bstart[p + 1] - sh.bstart[p] > kMaxGboBatch) sh.bad = 1;
            }
            for (int c = 0; c < 4; ++c) sh.ncolour[c] = 0;
            for (int p = 0; p < nbat; ++p) {
                if (sh.bstart[p + 1] == sh.bstart[p]) continue;
                const int c = (p % blocks & 1) + 2 * ((p / blocks) & 1);
                sh.colour_batches[c][sh.ncolour[c]++] = (uint8_t)p;
            }
        }
        __syncthreads();
        for (int p = tid; p < nbat; p += kGT) {
            int w = sh.bstart[p];
            for (int i = 0; i < n; ++i)
                if (sh.batch_of[i] == p) sh.members[w++] = (uint16_t)i;
        }
        __syncthreads();
        if (sh.bad) {   // a batch larger than kMaxGboBatch circles
            bad_instance();
            continue;
        }

        int rebuilds = 0, evals = 0, status = 0, outer = 0;
        int cell_mine = 0;      // this wave's evaluations over the cell grid
        int64_t pair_mine = 0;
        bool overflow = false;
        double ehist = 0.0, E64t = -1.0;
        float Ew = 0.f, gsum = 0.f, gs_all = 0.f;   // gsum: this wave's visits
        const int W = A.ftol_window;

        for (;;) {
            // ---- neighbor lists at sh.pos when flagged ---------------------------
            if (sh.flag) {
                bin_circles<kGT>(sh.pos, n, grid, sh.cell_start, sh.cell_circ, sh.slot_tmp,
                                 sh.scan_tmp);
                for (int cc = tid; cc < grid.nc * grid.nc; cc += kGT) {
                    const int a = sh.cell_start[cc], z = sh.cell_start[cc + 1];
                    for (int q = a + 1; q < z; ++q) {
                        const uint16_t key = sh.cell_circ[q];
                        int t = q - 1;
                        while (t >= a && sh.cell_circ[t] > key) { sh.cell_circ[t + 1] = sh.cell_circ[t]; --t; }
                        sh.cell_circ[t + 1] = key;
                    }
                }
                if (tid == 0) sh.over = 0;
                __syncthreads();
                for (int i0 = 0; i0 < n; i0 += kGT) {
                    const int i = i0 + tid;
                    const bool act = i < n;
                    const float2 q = sh.pos[act ? i : 0];
                    const int bi = sh.batch_of[act ? i : 0];
                    // candidates: the circles of the 3 x 3 cells around q's, in cell
                    // order; three cell rows (start, length), read together, one run
                    int ra[3], rl[3];
                    {
                        const int cx = cell_coord(q.x, grid), cy = cell_coord(q.y, grid);
                        const int y0 = cy > 0 ? cy - 1 : 0, y1 = cy < grid.nc - 1 ? cy + 1 : grid.nc - 1;
                        const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < grid.nc - 1 ? cx + 1 : grid.nc - 1;
#pragma unroll
                        for (int r = 0; r < 3; ++r) {
                            const bool row = act && y0 + r <= y1;
                            const int yy = y0 + r <= y1 ? y0 + r : y0;
                            const int a = sh.cell_start[yy * grid.nc + x0];
                            const int z = sh.cell_start[yy * grid.nc + x1 + 1];
                            ra[r] = row ? a : 0;
                            rl[r] = row ? z - a : 0;
                        }
                    }
                    const int K = rl[0] + rl[1] + rl[2];
                    // the wave walks its longest run, four candidates per step with their
                    // reads in flight; FP32 test outside the +-1e-5 band around the
                    // cutoff, FP64 inside (near_cut), behind one uniform branch
                    const int kmax = wave_max_dpp(K);
                    int m = 0;
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
                            jv[u] = ok[u] ? jj : 0;
                        }
                        float2 pv[4];
                        int bj[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            pv[u] = sh.pos[jv[u]];
                            bj[u] = sh.batch_of[jv[u]];
                        }
                        bool nb[4], band[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const float dx = q.x - pv[u].x, dy = q.y - pv[u].y;
                            const float l2 = dx * dx + dy * dy;
                            const bool cand = ok[u] && jv[u] != i;
                            nb[u] = cand && l2 < c2lo;
                            band[u] = cand && l2 >= c2lo && l2 <= c2hi;
                        }
                        if (__builtin_amdgcn_ballot_w64(band[0] || band[1] || band[2] || band[3])) {
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                if (band[u]) nb[u] = near64(q, pv[u], A.c2);
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (nb[u] && m < kGEll) sh.list[m][i] = (uint16_t)(jv[u] | (bj[u] == bi ? 0x8000 : 0));
                            m += nb[u] ? 1 : 0;
                        }
                    }
                    if (act) {
                        if (m > kGEll) sh.over = 1;
                        sh.list_n[i] = (uint8_t)(m < kGEll ? m : kGEll);
                        sh.xref[i] = q;
                    }
                }
                ++rebuilds;
                if (tid == 0) sh.flag = 0;
                __syncthreads();
                overflow = sh.over != 0;
            }

            // ---- whole-instance energies and the stop tests ------------------------
            {
                float e = 0.f, e1 = 0.f;
                double et = 0.0;
                for (int i = tid; i < n; i += kGT) {
                    const float2 q = sh.pos[i];
                    float ec = 0.f, e1c = 0.f, gx = 0.f, gy = 0.f;
                    double eoc = 0.0, etc = 0.0;
                    auto visit_pair = [&](int j) {
                        if (j <= i) return;
                        const float2 pj = sh.pos[j];
                        pair_term32(q, pj, true, two_r, four_r2, ec, e1c, gx, gy);
                        pair_term64(q, pj, two_r64, four_r2_64, eoc, etc);
                    };
                    if (!overflow) {
                        const int mc = sh.list_n[i];
                        for (int t = 0; t < mc; ++t) visit_pair(sh.list[t][i] & 0x7fff);
                    } else {
                        for_each_candidate(i, q, grid, sh.cell_start, sh.cell_circ, visit_pair);
                    }
                    const float r2 = q.x * q.x + q.y * q.y;
                    const float ir = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
                    const float d0 = fmaxf(r2 * ir + rad - R, 0.f);
                    ec += d0 * d0;
                    const float d01 = fmaxf(d0 - (rad - 1.f), 0.f);
                    e1c += d01 * d01;
                    const double r64 = sqrt((double)q.x * q.x + (double)q.y * q.y);
                    const double ct = r64 + 1.0 - R64;
                    if (ct > 0.0) etc += ct * ct;
                    if (!(isfinite(q.x) && isfinite(q.y))) { ec = e1c = __builtin_nanf(""); etc = __builtin_nan(""); }
                    e += ec;
                    e1 += e1c;
                    et += etc;
                }
                e = wave_sum(e);
                e1 = wave_sum(e1);
                et = wave_sum(et);
                const int par = outer & 1;
                if (lane == 0) {
                    sh.redf[par][wv] = e;
                    sh.redd[par][wv] = et;
                    sh.totw[wv][0] = e1;   // free at this point
                    sh.totw[wv][1] = gsum;
                }
                __syncthreads();
                Ew = 0.f;
                float E1w = 0.f, gs = 0.f;
                double ett = 0.0;
#pragma unroll
                for (int w = 0; w < kGW; ++w) {
                    Ew += sh.redf[par][w];
                    ett += sh.redd[par][w];
                    E1w += sh.totw[w][0];
                    gs += sh.totw[w][1];
                }
                __syncthreads();   // totw is the waves' scratch again below
                gs_all = gs;
                E64t = ett;
                const double Eacc = (double)Ew;
                if (!isfinite(Ew)) { status = 6; break; }
                if (E64t < A.e_feasible) { status = 1; break; }
                if (outer > 0 && gs <= A.g_tol) { status = 2; break; }
                if (A.ftol > 0.f && outer >= W) {
                    const int src = (outer - W) % (W + 1);
                    const long long bits = __builtin_bit_cast(long long, ehist);
                    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), src);
                    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
                    const double eold = __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
                    if (eold - Eacc <= (double)A.ftol * eold) { status = 3; break; }
                }
                if (lane == outer % (W + 1)) ehist = Eacc;
                if (outer >= A.max_iter) { status = 5; break; }
                (void)E1w;
            }

            // ---- one outer iteration: the four colours ---------------------------
            gsum = 0.f;
            for (int colour = 0; colour < 4; ++colour) {
                for (int r = wv; r < sh.ncolour[colour]; r += kGW) {
                    const int p = sh.colour_batches[colour][r];
                    const int m0 = sh.bstart[p], np = sh.bstart[p + 1] - m0;
                    // ---- visit batch p: registers <- its circles and history --
                    GboBatchState st = bst[p];
                    int k = st.k;
                    bool act[kGCPB];
                    int ci[kGCPB];
                    float2 x[kGCPB], g[kGCPB], pd[kGCPB];
                    float2 S[kMM][kGCPB], Y[kMM][kGCPB];
                    float2 *hS = histS + (size_t)p * kMM * kMaxGboBatch;
                    float2 *hY = histY + (size_t)p * kMM * kMaxGboBatch;
#pragma unroll
                    for (int c = 0; c < kGCPB; ++c) {
                        const int q = lane + c * kWave;
                        act[c] = q < np;
                        ci[c] = act[c] ? sh.members[m0 + q] : 0;
                        x[c] = act[c] ? sh.pos[ci[c]] : make_float2(0.f, 0.f);
                        g[c] = make_float2(0.f, 0.f);
                        pd[c] = make_float2(0.f, 0.f);
#pragma unroll
                        for (int j = 0; j < kMM; ++j) {
                            // logical j (newest at kMM-1) is ring slot head - (kMM-1-j)
                            const int sl = (st.head - (kMM - 1 - j) + 2 * kMM) % kMM;
                            const bool valid = act[c] && j >= kMM - k;
                            S[j][c] = valid ? hS[(size_t)sl * kMaxGboBatch + q] : make_float2(0.f, 0.f);
                            Y[j][c] = valid ? hY[(size_t)sl * kMaxGboBatch + q] : make_float2(0.f, 0.f);
                        }
                    }
                    float *Bwc[2] = {sh.Bw[wv][0], sh.Bw[wv][1]};
                    int cur = 0;
                    const float *gp_src = gram + (size_t)p * kNB * kNB;
                    for (int e = lane; e < kNB * kNB; e += kWave) Bwc[0][e] = gp_src[e];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

                    // one evaluation of the batch energy (Eq. 7) at xt: returns the
                    // slot total of this lane; gt gets the batch gradient
                    float Ep = 0.f;
                    double Ep64 = 0.0;
                    auto evaluate = [&](const float2 (&xt)[kGCPB], const float2 (&sc)[kGCPB],
                                        float2 (&gt)[kGCPB], float2 (&yc)[kGCPB], double &e64,
                                        bool far) -> float {
#pragma unroll
                        for (int c = 0; c < kGCPB; ++c)
                            if (act[c]) sh.tpos[ci[c]] = xt[c];
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        float e = 0.f, e1 = 0.f;
                        double ed = 0.0;
                        int pe = 0;
#pragma unroll
                        for (int c = 0; c < kGCPB; ++c) {
                            float gx = 0.f, gy = 0.f;
                            double gxd = 0.0, gyd = 0.0;
                            if (act[c]) {
                                const int i = ci[c];
                                const float2 q = xt[c];
                                auto term_in = [&](int j, bool inb) {
                                    const float2 pj = inb ? sh.tpos[j] : sh.pos[j];
                                    const bool ce = inb ? j < i : true;    // Eq. 7
                                    pe += ce;
                                    if (F64) {
                                        const double dx = (double)q.x - (double)pj.x;
                                        const double dy = (double)q.y - (double)pj.y;
                                        const double l2 = dx * dx + dy * dy;
                                        if (l2 < four_r2_64) {
                                            const double l = sqrt(l2);
                                            const double d = two_r64 - l;
                                            if (ce) ed += d * d;
                                            if (l > 0.0) {
                                                const double kf = -2.0 * d / l;
                                                gxd += kf * dx;
                                                gyd += kf * dy;
                                            }
                                        }
                                    } else {
                                        pair_term32(q, pj, ce, two_r, four_r2, e, e1, gx, gy);
                                    }
                                };
                                auto term = [&](int j) { term_in(j, sh.batch_of[j] == p); };
                                if (far) {
                                    // a circle of the batch left the skin: the other
                                    // circles from the cell grid, the batch's own from
                                    // its member list
                                    for_each_candidate(i, q, grid, sh.cell_start, sh.cell_circ, [&](int j) {
                                        if (sh.batch_of[j] != p) term(j);
                                    });
                                    for (int t = 0; t < np; ++t) {
                                        const int j = sh.members[m0 + t];
                                        if (j != i) term(j);
                                    }
                                } else if (!overflow) {
                                    const int mc = sh.list_n[i];
                                    for (int t = 0; t < mc; ++t) {
                                        const int en = sh.list[t][i];
                                        term_in(en & 0x7fff, (en & 0x8000) != 0);
                                    }
                                } else {
                                    for_each_candidate(i, q, grid, sh.cell_start, sh.cell_circ, term);
                                }
                                if (F64) {
                                    const double r64 = sqrt((double)q.x * q.x + (double)q.y * q.y);
                                    const double d0 = r64 + (double)rad - R64;
                                    if (d0 > 0.0) {
                                        ed += d0 * d0;
                                        if (r64 > 0.0) {
                                            gxd += 2.0 * d0 * q.x / r64;
                                            gyd += 2.0 * d0 * q.y / r64;
                                        }
                                    }
                                    gx = (float)gxd;
                                    gy = (float)gyd;
                                } else {
                                    const float r2 = q.x * q.x + q.y * q.y;
                                    const float ir = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
                                    const float d0 = fmaxf(r2 * ir + rad - R, 0.f);
                                    e += d0 * d0;
                                    const float kc = 2.f * d0 * ir;
                                    gx += kc * q.x;
                                    gy += kc * q.y;
                                }
                                if (!(isfinite(q.x) && isfinite(q.y))) {
                                    e = __builtin_nanf("");
                                    ed = __builtin_nan("");
                                }
                            }
                            gt[c] = make_float2(gx, gy);
                            yc[c] = make_float2(gx - g[c].x, gy - g[c].y);
                        }
                        if (F64) e = (float)ed;
                        e64 = wave_sum(ed);
                        ++evals;
                        cell_mine += (far || overflow) ? 1 : 0;
                        pair_mine += pe;
                        return wave_reduce_scatter<kGCPB>(gt, sc, yc, S, Y, e, e1);
                    };

                    // ---- gradient at the start of the visit (Alg. 1) -----
                    float2 gt[kGCPB], yc[kGCPB], sc0[kGCPB];
#pragma unroll
                    for (int c = 0; c < kGCPB; ++c) sc0[c] = make_float2(0.f, 0.f);
                    double e64 = 0.0;
                    // (every circle starts a colour within skin / 2 of its list
                    // position, so the visit's first point is in range of the lists)
                    float tot = evaluate(x, sc0, gt, yc, e64, false);
                    // slot totals are lane-indexed by lane_slot(); stage them
                    sh.totw[wv][lane_slot(lane)] = tot;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    auto gram_update = [&](bool push) {
                        for (int e = lane; e < kNB * kNB; e += kWave) {
                            const int src = sh.bsrc[push ? 1 : 0][e];
                            Bwc[cur ^ 1][e] = (src & 0x8000) ? sh.totw[wv][src & 0x7fff] : Bwc[cur][src];
                        }
                        cur ^= 1;
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    };
                    gram_update(false);
                    Ep = sh.totw[wv][sE];
                    Ep64 = e64;
#pragma unroll
                    for (int c = 0; c < kGCPB; ++c) g[c] = gt[c];
                    const float gg = Bwc[cur][kG * kNB + kG];
                    const float gn = sqrtf(fmaxf(gg, 0.f));
                    gsum += gn;

                    // ---- direction: two-loop on the batch's Gram matrix -----------
                    float Bc[kNB];
#pragma unroll
                    for (int a2 = 0; a2 < kNB; ++a2) Bc[a2] = lane < kNB ? Bwc[cur][a2 * kNB + lane] : 0.f;
                    // two-loop on the Gram matrix: lane l keeps (B q)_l, the Gram
                    // product of the current q with basis vector l (q = g at the
                    // start), so each step is one readlane and one FMA
                    const int jp = lane < kMM ? lane : lane - kMM;
                    const bool live = lane < 2 * kMM && jp >= kMM - k;
                    float rho_v = 0.f;              // 1 / s_j'y_j at lanes j and kMM + j
                    if (live) rho_v = 1.f / Bwc[cur][(lane < kMM ? kMM + lane : lane - kMM) * kNB + lane];
                    float acc = Bc[kG];
                    float alph_v = 0.f;             // a_j at lanes j and kMM + j
#pragma unroll
                    for (int j = kMM - 1; j >= 0; --j) {
                        const float a = lane_value(rho_v * acc, j);           // rho_j s_j'q
                        if (jp == j) alph_v = a;
                        acc -= a * Bc[kMM + j];
                    }
                    float gam = 1.f;
                    if (k > 0) gam = lane_value(Bc[kMM - 1], 2 * kMM - 1) / lane_value(Bc[2 * kMM - 1], 2 * kMM - 1);
                    acc *= gam;
                    float cs_v = 0.f;               // coefficient of s_j at lane j
#pragma unroll
                    for (int j = 0; j < kMM; ++j) {
                        const float c = lane_value(alph_v - rho_v * acc, kMM + j);   // a_j - rho_j y_j'r
                        if (lane == j) cs_v = c;
                        acc += c * Bc[j];
                    }
                    float gp = -lane_value(acc, kG);                               // g'p = -g'r
                    {
                        float cs[kMM], cy[kMM];
#pragma unroll
                        for (int j = 0; j < kMM; ++j) { cs[j] = lane_value(cs_v, j); cy[j] = -gam * lane_value(alph_v, j); }
#pragma unroll
                        for (int c = 0; c < kGCPB; ++c) {
                            float px = -gam * g[c].x, py = -gam * g[c].y;
#pragma unroll
                            for (int j = 0; j < kMM; ++j) {
                                px -= cs[j] * S[j][c].x + cy[j] * Y[j][c].x;
                                py -= cs[j] * S[j][c].y + cy[j] * Y[j][c].y;
                            }
                            pd[c] = make_float2(px, py);
                        }
                    }
                    if (k > 0 && !(gp < 0.f)) {
                        k = 0;
#pragma unroll
                        for (int c = 0; c < kGCPB; ++c) pd[c] = make_float2(-g[c].x, -g[c].y);
                        gp = -gg;
                    }
                    float alpha = k > 0 ? 1.f : 1.f / fmaxf(1.f, gn);

                    // ---- backtracking line search on E(x_p) ----------------------
                    bool accepted = false, push = false;
                    float2 xt[kGCPB], sc[kGCPB];
                    for (int h = 0; h <= A.max_halvings; ++h) {
                        bool out = false;
#pragma unroll
                        for (int c = 0; c < kGCPB; ++c) {
                            xt[c] = make_float2(fmaf(alpha, pd[c].x, x[c].x), fmaf(alpha, pd[c].y, x[c].y));
                            sc[c] = make_float2(xt[c].x - x[c].x, xt[c].y - x[c].y);
                            if (act[c]) {
                                const float2 rf = sh.xref[ci[c]];
                                const double dx = (double)xt[c].x - (double)rf.x, dy = (double)xt[c].y - (double)rf.y;
                                out |= dx * dx + dy * dy > A.skin2;
                            }
                        }
                        const bool far = __builtin_amdgcn_ballot_w64(out) != 0;
                        tot = evaluate(xt, sc, gt, yc, e64, far);
                        sh.totw[wv][lane_slot(lane)] = tot;
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        const float Et = sh.totw[wv][sE];
                        const bool ok = F64 ? e64 <= Ep64 + (double)A.c1 * (double)alpha * (double)gp
                                            : Et <= Ep + A.c1 * alpha * gp;
                        if (ok) {
                            accepted = true;
                            push = sh.totw[wv][sScYc] > A.eps_curv * sh.totw[wv][sYcYc];
                            break;
                        }
                        alpha *= 0.5f;
                    }
                    if (accepted) {
                        gram_update(push);
                        if (push) {
                            const int sl = (st.head + 1) % kMM;
#pragma unroll
                            for (int c = 0; c < kGCPB; ++c) {
                                const int q = lane + c * kWave;
                                if (act[c]) {
                                    hS[(size_t)sl * kMaxGboBatch + q] = sc[c];
                                    hY[(size_t)sl * kMaxGboBatch + q] = yc[c];
                                }
                            }
                            st.head = sl;
                            k = k + 1 > A.m ? A.m : k + 1;
                        }
#pragma unroll
                        for (int c = 0; c < kGCPB; ++c)
                            if (act[c]) sh.npos[ci[c]] = xt[c];
                    }
                    // ---- persist the batch's Gram matrix and ring ----------------
                    float *gdst = gram + (size_t)p * kNB * kNB;
                    for (int e = lane; e < kNB * kNB; e += kWave) gdst[e] = Bwc[cur][e];
                    if (lane == 0) { st.k = k; bst[p] = st; }
                }
                // ---- end of the colour: commit, maybe rebuild --------------------
                __syncthreads();
                int moved = 0;
                for (int i = tid; i < n; i += kGT) {
                    const float2 q = sh.npos[i];
                    sh.pos[i] = q;
                    const double dx = (double)q.x - (double)sh.xref[i].x, dy = (double)q.y - (double)sh.xref[i].y;
                    moved |= dx * dx + dy * dy > 0.25 * A.skin2;
                }
                if (moved) sh.flag = 1;
                __syncthreads();
                if (sh.flag && colour < 3) {
                    // rebuild between colours (the outer loop rebuilds after colour 3)
                    bin_circles<kGT>(sh.pos, n, grid, sh.cell_start, sh.cell_circ, sh.slot_tmp,
                                     sh.scan_tmp);
                    for (int cc = tid; cc < grid.nc * grid.nc; cc += kGT) {
                        const int a = sh.cell_start[cc], z = sh.cell_start[cc + 1];
                        for (int q = a + 1; q < z; ++q) {
                            const uint16_t key = sh.cell_circ[q];
                            int t = q - 1;
                            while (t >= a && sh.cell_circ[t] > key) { sh.cell_circ[t + 1] = sh.cell_circ[t]; --t; }
                            sh.cell_circ[t + 1] = key;
                        }
                    }
                    if (tid == 0) sh.over = 0;
                    __syncthreads();
                    for (int i0 = 0; i0 < n; i0 += kGT) {
                        const int i = i0 + tid;
                        const bool act = i < n;
                        const float2 q = sh.pos[act ? i : 0];
                        const int bi = sh.batch_of[act ? i : 0];
                        // candidates: the circles of the 3 x 3 cells around q's, in cell
                        // order; three cell rows (start, length), read together, one run
                        int ra[3], rl[3];
                        {
                            const int cx = cell_coord(q.x, grid), cy = cell_coord(q.y, grid);
                            const int y0 = cy > 0 ? cy - 1 : 0, y1 = cy < grid.nc - 1 ? cy + 1 : grid.nc - 1;
                            const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < grid.nc - 1 ? cx + 1 : grid.nc - 1;
#pragma unroll
                            for (int r = 0; r < 3; ++r) {
                                const bool row = act && y0 + r <= y1;
                                const int yy = y0 + r <= y1 ? y0 + r : y0;
                                const int a = sh.cell_start[yy * grid.nc + x0];
                                const int z = sh.cell_start[yy * grid.nc + x1 + 1];
                                ra[r] = row ? a : 0;
                                rl[r] = row ? z - a : 0;
                            }
                        }
                        const int K = rl[0] + rl[1] + rl[2];
                        // the wave walks its longest run, four candidates per step with their
                        // reads in flight; FP32 test outside the +-1e-5 band around the
                        // cutoff, FP64 inside (near_cut), behind one uniform branch
                        const int kmax = wave_max_dpp(K);
                        int m = 0;
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
                                jv[u] = ok[u] ? jj : 0;
                            }
                            float2 pv[4];
                            int bj[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                pv[u] = sh.pos[jv[u]];
                                bj[u] = sh.batch_of[jv[u]];
                            }
                            bool nb[4], band[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const float dx = q.x - pv[u].x, dy = q.y - pv[u].y;
                                const float l2 = dx * dx + dy * dy;
                                const bool cand = ok[u] && jv[u] != i;
                                nb[u] = cand && l2 < c2lo;
                                band[u] = cand && l2 >= c2lo && l2 <= c2hi;
                            }
                            if (__builtin_amdgcn_ballot_w64(band[0] || band[1] || band[2] || band[3])) {
#pragma unroll
                                for (int u = 0; u < 4; ++u)
                                    if (band[u]) nb[u] = near64(q, pv[u], A.c2);
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                if (nb[u] && m < kGEll) sh.list[m][i] = (uint16_t)(jv[u] | (bj[u] == bi ? 0x8000 : 0));
                                m += nb[u] ? 1 : 0;
                            }
                        }
                        if (act) {
                            if (m > kGEll) sh.over = 1;
                            sh.list_n[i] = (uint8_t)(m < kGEll ? m : kGEll);
                            sh.xref[i] = q;
                        }
                    }
                    ++rebuilds;
                    if (tid == 0) sh.flag = 0;
                    __syncthreads();
                    overflow = sh.over != 0;
                }
            }
            // waves' visit-gradient norms, summed in the energy block above
            ++outer;
        }

        // ---- write back ----------------------------------------------------------
        for (int i = tid; i < n; i += kGT) reinterpret_cast<float2 *>(xy)[off + i] = sh.pos[i];
        {
            unsigned long long pm = (unsigned long long)pair_mine;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) pm += __shfl_xor(pm, o, kWave);
            __syncthreads();
            if (lane == 0) sh.redd[0][wv] = __builtin_bit_cast(double, pm);
            __syncthreads();
            pm = 0;
            for (int w = 0; w < kGW; ++w) pm += __builtin_bit_cast(unsigned long long, sh.redd[0][w]);
            pair_mine = (int64_t)pm;
        }
        {
            // every wave's batch evaluations, and those over the cell grid
            __syncthreads();
            if (lane == 0) { sh.scan_tmp[wv] = cell_mine; sh.evw[wv] = evals; }
            __syncthreads();
            cell_mine = 0;
            evals = 0;
            for (int w = 0; w < kGW; ++w) {
                cell_mine += sh.scan_tmp[w];
                evals += sh.evw[w];
            }
        }
        if (tid == 0) {
            DescentHead r;
            r.status = status;
            r.iters = outer;
            r.evals = evals;
            r.rebuilds = rebuilds;
            r.pair_evals = pair_mine;
            r.E32 = Ew;
            r.gnorm = gs_all;
            r.E64 = E64t;
            store_result(out, b, r, cell_mine);
        }
    }
}

size_t gbo_workspace_bytes(int B, int blocks)
{
    return sizeof(int32_t) * ((size_t)B + 1 + 64) + (size_t)B * gbo_instance_bytes(blocks * blocks);
}

int gbo_grid(int B)
{
    const int cus = current_device_cus();
    return B < cus ? B : cus;
}

hipError_t launch_queue_init(const int32_t *offset, int B, int32_t *queue, hipStream_t s);

hipError_t launch_gbo(const int32_t *offset, const float *R, const double *R64, float *xy, int B,
                      int64_t total_n, const DescentArgs &a, int blocks, int sweep_fp64, void *out,
                      void *ws, hipStream_t s)
{
    int32_t *queue = reinterpret_cast<int32_t *>(ws);
    unsigned char *wsb = reinterpret_cast<unsigned char *>(ws) +
                         ((sizeof(int32_t) * ((size_t)B + 1 + 64) + 255) & ~(size_t)255);
    hipError_t e = launch_queue_init(offset, B, queue, s);
    if (e != hipSuccess) return e;
    const int grid = gbo_grid(B);
    if (sweep_fp64)
        gbo_descend_kernel<true><<<grid, kGT, 0, s>>>(offset, R, R64, xy, B, total_n, a, blocks,
                                                      reinterpret_cast<DescentResultDev *>(out), queue, wsb);
    else
        gbo_descend_kernel<false><<<grid, kGT, 0, s>>>(offset, R, R64, xy, B, total_n, a, blocks,
                                                       reinterpret_cast<DescentResultDev *>(out), queue, wsb);
    return hipGetLastError();
}

}  // namespace pecc
