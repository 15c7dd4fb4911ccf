// Device helpers shared by the library's kernels: the uniform cell grid and
// its counting sort in LDS, the FP64 neighbor predicate, wave64 and block
// reductions and scans.  gfx950 only (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pecc {

constexpr int kMaxN = 1024;          // circles per instance
constexpr int kNcMax = 64;           // cells per axis at most
constexpr int kMaxCells = kNcMax * kNcMax;
constexpr int kWave = 64;
// Relative safety on the cell side: (v + R) * (1/h) is rounded in FP32, so
// two points closer than the cutoff could otherwise land two cells apart.
// With at most 64 cells per axis the rounding error of the cell coordinate
// is below 64 * 2^-22; 1e-4 covers it with room to spare.
constexpr float kCellSafety = 1.0e-4f;

// ---------------------------------------------------------------------------
// Cell grid over the square [-R, R]^2.  Cell side h >= cutoff * (1 + safety)
// and h >= 2R / kNcMax (bigger cells when the container is large).  Cell
// coordinates are clamped per axis, which is 1-Lipschitz, so any two points
// closer than the cutoff (also outside the square) sit in adjacent cells.
// ---------------------------------------------------------------------------
struct Grid {
    float lo;      // -R
    float inv_h;   // 1 / h
    int nc;        // cells per axis
};

__device__ __forceinline__ Grid make_grid(float R, float h_req)
{
    Grid g;
    const float span = 2.0f * R;
    float h = h_req;
    if (span / (float)kNcMax > h) h = span / (float)kNcMax;
    float t = span / h;
    int nc = (t >= 1.0f) ? (int)ceilf(fminf(t, (float)kNcMax)) : 1;
    if (nc > kNcMax) nc = kNcMax;
    if (nc < 1) nc = 1;
    g.lo = -R;
    g.inv_h = (h > 0.0f && h < 3.0e38f) ? 1.0f / h : 0.0f;
    g.nc = nc;
    return g;
}

__device__ __forceinline__ int cell_coord(float v, const Grid &g)
{
    const float t = (v - g.lo) * g.inv_h;
    // NaN fails the comparison and lands in cell 0; large values clamp
    return (t >= 0.0f) ? (int)fminf(t, (float)(g.nc - 1)) : 0;
}

__device__ __forceinline__ int cell_of(float2 p, const Grid &g)
{
    return cell_coord(p.y, g) * g.nc + cell_coord(p.x, g);
}

// FP64 neighbor predicate on FP32 coordinates, each operation rounded once:
// dx*dx + dy*dy < c2.  The operators are written here, under contract(off):
// operations inlined from helpers keep the contraction permission of the
// scope they were written in.
__device__ __forceinline__ bool near64(float2 a, float2 b, double c2)
{
#pragma clang fp contract(off)   // each operation rounded on its own, like the oracle
    const double dx = (double)a.x - (double)b.x;
    const double dy = (double)a.y - (double)b.y;
    return dx * dx + dy * dy < c2;
}

// ---------------------------------------------------------------------------
// wave64 reductions and scans
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ int wave_inclusive_scan(int v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one int per thread over the block.  tmp: LDS with at
// least BLOCK/64 + 1 ints.  Returns the exclusive prefix; *total gets the
// block total.  Contains three barriers; every thread must call it.
template <int BLOCK>
__device__ __forceinline__ int block_exclusive_scan(int v, int *tmp, int *total)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int inc = wave_inclusive_scan(v);
    __syncthreads();                 // tmp may still be read by a previous call
    if (lane == kWave - 1) tmp[w] = inc;
    __syncthreads();
    if (w == 0) {
        int t = lane < NW ? tmp[lane] : 0;
        t = wave_inclusive_scan(t);
        if (lane < NW) tmp[lane] = t;   // inclusive prefix of wave totals
    }
    __syncthreads();
    const int base = w > 0 ? tmp[w - 1] : 0;
    *total = tmp[NW - 1];
    return base + inc - v;
}

// Sum of one value per thread over the block, same result in every thread.
// tmp: LDS of BLOCK/64 elements.  Two barriers.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_sum(T v, T *tmp)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    v = wave_sum(v);
    __syncthreads();                 // tmp may still be read by a previous call
    if (lane == 0) tmp[w] = v;
    __syncthreads();
    T s = tmp[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) s += tmp[i];
    return s;
}

template <int BLOCK>
__device__ __forceinline__ double block_max(double v, double *tmp)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) tmp[w] = v;
    __syncthreads();
    double s = tmp[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) s = fmax(s, tmp[i]);
    return s;
}

// ---------------------------------------------------------------------------
// Counting sort of the n circles of one instance into grid cells, in LDS.
//   pos        LDS float2[n]       positions
//   cell_start LDS int[ncell + 1]  out: first slot of each cell
//   cell_circ  LDS uint16[n]       out: local circle indices grouped by cell
//   slot_tmp   LDS uint16[n]       scratch
//   scan_tmp   LDS int[BLOCK/64+1] scratch
// The order inside a cell depends on atomic arrival order; callers that
// need determinism sort what they read out of a cell.  Ends with a barrier.
// ---------------------------------------------------------------------------
template <int BLOCK>
__device__ void bin_circles(const float2 *pos, int n, const Grid &g,
                            int *cell_start, uint16_t *cell_circ, uint16_t *slot_tmp,
                            int *scan_tmp)
{
    const int ncell = g.nc * g.nc;
    for (int c = threadIdx.x; c <= ncell; c += BLOCK) cell_start[c] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += BLOCK) {
        const int c = cell_of(pos[i], g);
        slot_tmp[i] = (uint16_t)atomicAdd(&cell_start[c], 1);
    }
    __syncthreads();
    // exclusive scan over the cell counts: each thread owns a chunk
    constexpr int CH = (kMaxCells + BLOCK - 1) / BLOCK;
    const int c0 = threadIdx.x * CH;
    int loc[CH];
    int s = 0;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int c = c0 + k;
        loc[k] = (c < ncell) ? cell_start[c] : 0;
        s += loc[k];
    }
    int total;
    int run = block_exclusive_scan<BLOCK>(s, scan_tmp, &total);
    // every thread has read its counts before the scan's barriers
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int c = c0 + k;
        if (c < ncell) cell_start[c] = run;
        run += loc[k];
    }
    if (threadIdx.x == 0) cell_start[ncell] = total;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += BLOCK) {
        const int c = cell_of(pos[i], g);
        cell_circ[cell_start[c] + slot_tmp[i]] = (uint16_t)i;
    }
    __syncthreads();
}

// Visit every circle j != i in the 3x3 cells around circle i's cell.
template <typename F>
__device__ __forceinline__ void for_each_candidate(int i, float2 pi, const Grid &g,
                                                   const int *cell_start,
                                                   const uint16_t *cell_circ, F &&f)
{
    const int cx = cell_coord(pi.x, g), cy = cell_coord(pi.y, g);
    const int y0 = cy > 0 ? cy - 1 : 0, y1 = cy < g.nc - 1 ? cy + 1 : g.nc - 1;
    const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < g.nc - 1 ? cx + 1 : g.nc - 1;
    for (int yy = y0; yy <= y1; ++yy) {
        const int rowc = yy * g.nc;
        const int a = cell_start[rowc + x0], b = cell_start[rowc + x1 + 1];
        // cells x0..x1 of one row are contiguous in the sorted order
        for (int k = a; k < b; ++k) {
            const int j = cell_circ[k];
            if (j != i) f(j);
        }
    }
}

// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror & Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011), written from its
// published definition: ten rounds of two 64 x 64 -> 128-bit multiplies, the
// key bumped by two Weyl constants between rounds.
struct U64x4 {
    uint64_t w[4];
};

__device__ __forceinline__ U64x4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    U64x4 o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

}  // namespace pecc
