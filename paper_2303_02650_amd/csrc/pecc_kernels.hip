// Neighbor-list build, list-based energy/gradient sweep and FP64 verify.
//
// One workgroup per instance throughout: an instance (n <= 1024 circles,
// 8 KB of positions) is staged in LDS once and every access after that is
// on chip.
#include "pecc_device.hpp"
#include "pecc_launch.hpp"

#include <type_traits>

namespace pecc {

constexpr int kBuildBlock = 256;

// Positions of one instance into LDS (coalesced float2 loads).
template <int BLOCK>
__device__ __forceinline__ void stage_positions(const float *xy, int off, int n, float2 *pos)
{
    const float2 *src = reinterpret_cast<const float2 *>(xy) + off;
    for (int i = threadIdx.x; i < n; i += BLOCK) pos[i] = src[i];
}

// Circle range of instance b.  False when the offsets are not a valid
// range inside [0, total_n] or the instance has more than kMaxN circles.
__device__ __forceinline__ bool instance_range(const int32_t *offset, int b, int64_t total_n,
                                               int *off, int *n)
{
    const int a = offset[b], e = offset[b + 1];
    *off = a;
    *n = e - a;
    return a >= 0 && e >= a && (int64_t)e <= total_n && e - a <= kMaxN;
}

// True when circles off .. off+n-1 may be written for an invalid instance.
__device__ __forceinline__ bool writable_range(int off, int n, int64_t total_n)
{
    return off >= 0 && n > 0 && (int64_t)off + n <= total_n;
}

// ---------------------------------------------------------------------------
// Build, pass 1: per-circle list length into row[i+1], per-instance total.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBuildBlock) void build_count_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ R,
    const float *__restrict__ xy, int64_t total_n, double c2, float h_req, int full,
    int32_t *__restrict__ row, int64_t *__restrict__ inst_total)
{
    __shared__ float2 pos[kMaxN];
    __shared__ int cell_start[kMaxCells + 1];
    __shared__ uint16_t cell_circ[kMaxN];
    __shared__ uint16_t slot_tmp[kMaxN];
    __shared__ int scan_tmp[kBuildBlock / kWave + 1];
    __shared__ int sum_tmp[kBuildBlock / kWave];

    const int b = blockIdx.x;
    int off, n;
    if (!instance_range(offset, b, total_n, &off, &n)) {
        // not a valid instance: an empty list for each of its circles
        if (writable_range(off, n, total_n))
            for (int i = threadIdx.x; i < n; i += kBuildBlock) row[off + i + 1] = 0;
        if (threadIdx.x == 0) inst_total[b] = 0;
        return;
    }
    stage_positions<kBuildBlock>(xy, off, n, pos);
    __syncthreads();
    const Grid g = make_grid(R[b], h_req);
    bin_circles<kBuildBlock>(pos, n, g, cell_start, cell_circ, slot_tmp, scan_tmp);
    int mine = 0;
    for (int i = threadIdx.x; i < n; i += kBuildBlock) {
        const float2 pi = pos[i];
        int cnt = 0;
        for_each_candidate(i, pi, g, cell_start, cell_circ, [&](int j) {
            if ((full || j > i) && near64(pi, pos[j], c2)) ++cnt;
        });
        row[off + i + 1] = cnt;
        mine += cnt;
    }
    const int tot = block_sum<kBuildBlock>(mine, sum_tmp);
    if (threadIdx.x == 0) inst_total[b] = tot;
}

// Build, pass 2: exclusive scan of the per-instance totals (one workgroup).
constexpr int kScanBlock = 1024;
__global__ __launch_bounds__(kScanBlock) void build_scan_kernel(
    int64_t *__restrict__ inst_total, int B, int64_t total_n,
    int32_t *__restrict__ row, int64_t *__restrict__ num_pairs)
{
    __shared__ int64_t carry_s;
    __shared__ int64_t wsum[kScanBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < B; base += kScanBlock) {
        const int b = base + threadIdx.x;
        const int64_t v = b < B ? inst_total[b] : 0;
        int64_t inc = v;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int64_t t = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += t;
        }
        if (lane == kWave - 1) wsum[w] = inc;
        __syncthreads();
        int64_t before = 0;
        for (int k = 0; k < w; ++k) before += wsum[k];
        int64_t chunk = 0;
        for (int k = 0; k < kScanBlock / kWave; ++k) chunk += wsum[k];
        const int64_t carry = carry_s;
        if (b < B) inst_total[b] = carry + before + inc - v;   // now: base offset
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + chunk;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        num_pairs[0] = carry_s;
        row[0] = 0;
        row[total_n] = (int32_t)(carry_s < 0x7fffffffLL ? carry_s : 0x7fffffffLL);
    }
}

// Build, pass 3: row offsets and the sorted column indices (int32 global
// indices, or uint16 instance-local ones).
template <typename Idx>
__global__ __launch_bounds__(kBuildBlock) void build_fill_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ R,
    const float *__restrict__ xy, int64_t total_n, double c2, float h_req, int full,
    int32_t *__restrict__ row, Idx *__restrict__ col, int64_t capacity,
    const int64_t *__restrict__ inst_base)
{
    constexpr bool kLocal = sizeof(Idx) == 2;
    __shared__ float2 pos[kMaxN];
    __shared__ int cell_start[kMaxCells + 1];
    __shared__ uint16_t cell_circ[kMaxN];
    __shared__ uint16_t slot_tmp[kMaxN];
    __shared__ int scan_tmp[kBuildBlock / kWave + 1];
    __shared__ int cnt_s[kMaxN];
    __shared__ int run_s;

    const int b = blockIdx.x;
    int off, n;
    const bool ok = instance_range(offset, b, total_n, &off, &n);
    const int64_t base = inst_base[b];
    if (!ok) {
        if (writable_range(off, n, total_n))
            for (int i = threadIdx.x; i < n; i += kBuildBlock)
                row[off + i] = (int32_t)(base < 0x7fffffffLL ? base : 0x7fffffffLL);
        return;
    }
    // the counts of pass 1 sit in row[off+1 .. off+n]; read them all first
    for (int i = threadIdx.x; i < n; i += kBuildBlock) cnt_s[i] = row[off + i + 1];
    stage_positions<kBuildBlock>(xy, off, n, pos);
    if (threadIdx.x == 0) run_s = 0;
    __syncthreads();
    // exclusive scan of the counts, kBuildBlock circles at a time
    for (int c0 = 0; c0 < n; c0 += kBuildBlock) {
        const int i = c0 + threadIdx.x;
        const int v = i < n ? cnt_s[i] : 0;
        int tot;
        const int ex = block_exclusive_scan<kBuildBlock>(v, scan_tmp, &tot);
        const int run = run_s;
        __syncthreads();
        if (i < n) cnt_s[i] = run + ex;           // now: local row start
        if (threadIdx.x == 0) run_s = run + tot;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += kBuildBlock) {
        const int64_t r = base + cnt_s[i];
        row[off + i] = (int32_t)(r < 0x7fffffffLL ? r : 0x7fffffffLL);
    }
    const Grid g = make_grid(R[b], h_req);
    bin_circles<kBuildBlock>(pos, n, g, cell_start, cell_circ, slot_tmp, scan_tmp);
    for (int i = threadIdx.x; i < n; i += kBuildBlock) {
        const float2 pi = pos[i];
        const int64_t start = base + cnt_s[i];
        int64_t w = start;
        for_each_candidate(i, pi, g, cell_start, cell_circ, [&](int j) {
            if ((full || j > i) && near64(pi, pos[j], c2)) {
                if (w < capacity) col[w] = (Idx)(kLocal ? j : off + j);
                ++w;
            }
        });
        // insertion sort of the stored part of this row (rows are short)
        const int64_t end = w < capacity ? w : capacity;
        for (int64_t a = start + 1; a < end; ++a) {
            const Idx key = col[a];
            int64_t k = a - 1;
            while (k >= start && col[k] > key) { col[k + 1] = col[k]; --k; }
            col[k + 1] = key;
        }
    }
}

// ---------------------------------------------------------------------------
// Energy and gradient over a list with both orientations (Def. 3.1,
// Def. 3.2), in one of two index forms: int32 global circle indices or
// uint16 instance-local ones (the compact form: 2 bytes per entry, so the
// list costs 4 bytes per pair).  Each thread owns circles and sums their
// pair terms in list order: no atomics.  One workgroup of 256 threads per
// instance; positions (8 KB) and the instance's list segment (when it fits,
// up to 6123 entries) are staged in LDS with coalesced streaming
// (non-temporal) 16-byte loads, the segment held as 16-bit byte offsets into
// the staged positions, so global memory sees each byte once, and the
// gradient leaves with streaming 8-byte stores.  An entry past a row's end
// reads a sentinel that points at a position far outside every container,
// so the pair loop needs no tests of its own.  The LDS footprint (20,464
// bytes) lets eight workgroups (32 waves) stay resident per CU, overlapping
// one instance's loads with another's arithmetic, and each thread walks the
// lists of two circles at once so that their LDS reads overlap.
// ---------------------------------------------------------------------------
constexpr int kSweepBlock = 256;
constexpr int kColLds = 6124;   // 8200 + 2 * 6124 + 16 bytes of LDS fit 8 workgroups per CU
constexpr uint16_t kFarOff = kMaxN * sizeof(float2);   // byte offset of the far position

template <typename Idx>
__global__ __launch_bounds__(kSweepBlock) void energy_grad_full_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ R,
    const float *__restrict__ xy, int64_t total_n, const int32_t *__restrict__ row,
    const Idx *__restrict__ col, int64_t col_len, float rad,
    float *__restrict__ energy, float *__restrict__ grad)
{
    // entries per 16-byte load; a local index needs no offset
    constexpr int kIV = 16 / (int)sizeof(Idx);
    constexpr bool kLocal = sizeof(Idx) == 2;
    __shared__ float2 pos[kMaxN + 1];         // + the far position
    __shared__ uint16_t col_s[kColLds];
    __shared__ float sum_tmp[kSweepBlock / kWave];

    const int b = blockIdx.x;
    int off, n;
    if (!instance_range(offset, b, total_n, &off, &n)) {
        if (threadIdx.x == 0) energy[b] = __builtin_nanf("");
        return;
    }
    // list entries outside [0, col_len) are never read
    const int r0 = row[off], r1 = row[off + n];
    const int len = r1 - r0;
    const bool sane = r0 >= 0 && len >= 0 && (int64_t)r1 <= col_len;
    if (!sane) {
        if (threadIdx.x == 0) energy[b] = __builtin_nanf("");
        return;
    }
    const bool staged = len < kColLds;         // room for the sentinel
    // One batch of streaming loads per thread -- positions as float4 where
    // the instance start is 16-byte aligned, the list segment as int4 -- all
    // issued before the first is used, so the workgroup waits for memory
    // once; then the LDS writes (list entries as 16-bit local indices).
    typedef float v4f __attribute__((ext_vector_type(4)));
    typedef int v4i __attribute__((ext_vector_type(4)));
    constexpr int kPV = (kMaxN / 2 + kSweepBlock - 1) / kSweepBlock;   // float4 per thread
    constexpr int kCV = (kColLds / kIV + kSweepBlock - 1) / kSweepBlock; // 16-byte loads per thread
    const bool pos_al = (reinterpret_cast<uintptr_t>(xy + 2 * (int64_t)off) & 15) == 0;
    const int npv = pos_al ? n / 2 : 0;
    const v4f *psrc = reinterpret_cast<const v4f *>(xy + 2 * (int64_t)off);
    const int mis = (int)((reinterpret_cast<uintptr_t>(col + r0) & 15) / sizeof(Idx));
    const int head = staged ? min(len, (kIV - mis) & (kIV - 1)) : 0;
    const int nv = staged ? (len - head) / kIV : 0;
    const v4i *csrc = reinterpret_cast<const v4i *>(col + r0 + head);
    // unconditional loads (indices clamped into range; the extra lanes'
    // values are dropped below), so nothing waits between them
    v4f pv[kPV];
    v4i cv[kCV];
    if (npv > 0) {
#pragma unroll
        for (int u = 0; u < kPV; ++u) {
            const int k = threadIdx.x + u * kSweepBlock;
            pv[u] = __builtin_nontemporal_load(psrc + (k < npv ? k : 0));
        }
    }
    if (nv > 0) {
#pragma unroll
        for (int u = 0; u < kCV; ++u) {
            const int v = threadIdx.x + u * kSweepBlock;
            cv[u] = __builtin_nontemporal_load(csrc + (v < nv ? v : 0));
        }
    }
    // row bounds of this thread's circles tid + 256 c (indices clamped to n)
    constexpr int kRC = kMaxN / kSweepBlock;
    int rw[kRC + 1];
#pragma unroll
    for (int c = 0; c <= kRC; ++c) {
        const int i = threadIdx.x + c * kSweepBlock;
        rw[c] = row[off + (i < n ? i : n)];
    }
    int rw1[kRC];
#pragma unroll
    for (int c = 0; c < kRC; ++c) {
        const int i = threadIdx.x + c * kSweepBlock + 1;
        rw1[c] = row[off + (i < n ? i : n)];
    }
    // an entry as the byte offset of its position; one outside the
    // instance as the far position (a pair that does not overlap)
    auto put = [&](int k, int v) {
        const int jj = kLocal ? v : v - off;
        col_s[k] = (unsigned)jj < (unsigned)n ? (uint16_t)(jj * (int)sizeof(float2)) : kFarOff;
    };
    if (!pos_al) {
        stage_positions<kSweepBlock>(xy, off, n, pos);
    } else if ((n & 1) && threadIdx.x == 0) {
        pos[n - 1] = reinterpret_cast<const float2 *>(xy)[off + n - 1];
    }
    if (staged) {
        if (threadIdx.x == 0) {
            col_s[len] = kFarOff;                         // sentinel past the last row
            pos[kMaxN] = make_float2(1e18f, 1e18f);       // squared distances stay finite
        }
        if ((int)threadIdx.x < head) put(threadIdx.x, col[r0 + threadIdx.x]);
        for (int k = head + kIV * nv + threadIdx.x; k < len; k += kSweepBlock) put(k, col[r0 + k]);
    }
#pragma unroll
    for (int u = 0; u < kPV; ++u) {
        const int k = threadIdx.x + u * kSweepBlock;
        if (k < npv) reinterpret_cast<float4 *>(pos)[k] = make_float4(pv[u].x, pv[u].y, pv[u].z, pv[u].w);
    }
#pragma unroll
    for (int u = 0; u < kCV; ++u) {
        const int v = threadIdx.x + u * kSweepBlock;
        if (v < nv) {
            const int k = head + kIV * v;
            if constexpr (kLocal) {
                // eight 16-bit entries, low half first
                const int w4[4] = {cv[u].x, cv[u].y, cv[u].z, cv[u].w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    put(k + 2 * q, w4[q] & 0xffff);
                    put(k + 2 * q + 1, (int)((unsigned)w4[q] >> 16));
                }
            } else {
                put(k, cv[u].x); put(k + 1, cv[u].y); put(k + 2, cv[u].z); put(k + 3, cv[u].w);
            }
        }
    }
    __syncthreads();
    const float Rb = R[b];
    const float two_r = 2.0f * rad, four_r2 = two_r * two_r;
    float e = 0.0f;
    const bool g_al = (reinterpret_cast<uintptr_t>(grad) & 7) == 0;
#pragma unroll
    for (int pass = 0; pass < kRC / 2; ++pass) {
      const int i0 = threadIdx.x + 2 * kSweepBlock * pass;
      if (i0 >= n) break;
      // two circles per pass (i0 and i0 + kSweepBlock): their list and
      // position reads overlap; each keeps its own order of terms
      float gxA[2], gyA[2], eiA[2];
      int aA[2], zA[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
          const int i = i0 + h * kSweepBlock;
          gxA[h] = gyA[h] = eiA[h] = 0.f;
          aA[h] = 0; zA[h] = 0;
          if (i < n) {
              int a = rw[2 * pass + h] - r0, z = rw1[2 * pass + h] - r0;
              aA[h] = a < 0 ? 0 : a;
              zA[h] = z > len ? len : z;
          }
      }
      const int span = max(zA[0] - aA[0], zA[1] - aA[1]);
      const float2 piA[2] = {pos[i0], i0 + kSweepBlock < n ? pos[i0 + kSweepBlock] : make_float2(0.f, 0.f)};
      // one pass over the rows, branch-free: an entry past its row or
      // outside the instance is the far position, a pair that does not
      // overlap.  Per pair side: kf' = d / l (the factor -2 of the gradient
      // term is applied to the sums at the end, exactly), and d^2 of every
      // side (each pair counted twice, halved at the end); 1/l from
      // l^2 + FLT_MIN (exactly l^2 above 2^-100), so coincident centres (l =
      // 0, dx = dy = 0) give d = 2 rad and no gradient without a test of
      // their own.
      auto rows_pass = [&](auto staged_c) {
          constexpr bool ST = decltype(staged_c)::value;
#pragma unroll 1
          for (int t = 0; t < span; ++t) {
              float2 pjA[2];
              bool realA[2];
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                  const int k = aA[h] + t;
                  if constexpr (ST) {
                      // past the row: the sentinel at col_s[len]
                      const int off8 = col_s[k < zA[h] ? k : len];
                      pjA[h] = *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(pos) + off8);
                      realA[h] = true;
                  } else {
                      int j = 0xFFFF;
                      if (k < zA[h]) j = kLocal ? (int)col[r0 + k] : col[r0 + k] - off;
                      realA[h] = (unsigned)j < (unsigned)n;
                      pjA[h] = pos[realA[h] ? j : 0];
                  }
              }
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                  const float2 pi = piA[h], pj = pjA[h];
                  const float dx = pi.x - pj.x, dy = pi.y - pj.y;
                  const float l2r = dx * dx + dy * dy;
                  const float l2 = ST || realA[h] ? l2r : four_r2;
                  const float il = __builtin_amdgcn_rsqf(l2 + 1.17549435e-38f);
                  const float d = l2 < four_r2 ? two_r - l2 * il : 0.f;
                  eiA[h] = fmaf(d, d, eiA[h]);
                  const float kf = d * il;
                  gxA[h] = fmaf(kf, dx, gxA[h]);
                  gyA[h] = fmaf(kf, dy, gyA[h]);
              }
          }
      };
      if (staged) rows_pass(std::true_type{});
      else rows_pass(std::false_type{});
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = i0 + h * kSweepBlock;
        if (i >= n) break;
        const float2 pi = piA[h];
        // the sums of the pair sides: gradient times -2, energy halved
        float gx = -2.f * gxA[h], gy = -2.f * gyA[h], ei = 0.5f * eiA[h];
        const float r2 = pi.x * pi.x + pi.y * pi.y;
        const float ir = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
        const float d0 = fmaxf(r2 * ir + rad - Rb, 0.f);
        ei += d0 * d0;
        const float kc = 2.f * d0 * ir;
        gx += kc * pi.x;
        gy += kc * pi.y;
        // E sums over every circle: a non-finite position makes it NaN
        if (!(isfinite(pi.x) && isfinite(pi.y))) ei = __builtin_nanf("");
        e += ei;
        if (grad) {
            if (g_al) {
                typedef float v2f __attribute__((ext_vector_type(2)));
                const v2f t = {gx, gy};
                __builtin_nontemporal_store(t, reinterpret_cast<v2f *>(grad) + (off + i));
            } else {
                __builtin_nontemporal_store(gx, &grad[2 * (int64_t)(off + i)]);
                __builtin_nontemporal_store(gy, &grad[2 * (int64_t)(off + i) + 1]);
            }
        }
      }
    }
    const float tot = block_sum<kSweepBlock>(e, sum_tmp);
    if (threadIdx.x == 0) energy[b] = tot;
}

// ---------------------------------------------------------------------------
// Energy and gradient over a neighbor list that holds each pair once
// (Def. 3.1, Def. 3.2; rows ascending, entries j > i).  One workgroup of 512
// threads per instance, three passes over the list segment staged in LDS:
//   * staging: coalesced streaming (non-temporal) 16-byte loads of the
//     segment, every entry stored as the pair (i, j) of 16-bit local indices
//     (j from the loads, i filled in by the thread that owns row i), so
//     global memory sees each list entry once;
//   * the pair pass, entry-parallel (every thread the same number of
//     pairs): the pair term of Def. 3.1 once per pair, its energy added to
//     the thread's sum and its gradient term for circle i stored in place of
//     the entry; the entry is also counted and placed in circle j's bucket
//     (a counting sort by j in LDS: 16-bit counters two per word, a block
//     scan, a scatter, each bucket then sorted by entry, as the scatter's
//     order depends on atomic arrival);
//   * the gather, one thread per circle: the terms of its partners below it
//     (its bucket, negated: the term for j is minus the term for i, bit for
//     bit) and then above it (its own row), in ascending order of the other
//     circle.  No atomics on the sums, so the result is bitwise
//     reproducible.
// A segment longer than the LDS chunk is taken in consecutive chunks: every
// partner i < j of circle j sits in a row before row j, so a circle's terms
// are still added in ascending order of the other circle.  Four workgroups
// (32 waves) stay resident per CU, overlapping one instance's loads with
// another's on-chip work.
// ---------------------------------------------------------------------------
constexpr int kHalfBlock = 512;
constexpr int kHalfWaves = kHalfBlock / kWave;
constexpr int kHalfChunk = 3024;    // list entries per chunk (a multiple of 8)

union SweepEntry {
    struct { uint16_t j, i; } h;   // staged pair: local indices of the partner and of the row
    uint32_t ij;
    float2 f;                      // after the pair pass: the pair's gradient term for circle i
};

__global__ __launch_bounds__(kHalfBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void energy_grad_half_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ R,
    const float *__restrict__ xy, int64_t total_n, const int32_t *__restrict__ row,
    const int32_t *__restrict__ col, int64_t col_len, float rad,
    float *__restrict__ energy, float *__restrict__ grad)
{
    __shared__ float2 pos[kMaxN];
    __shared__ SweepEntry ent[kHalfChunk];
    __shared__ uint16_t rev[kHalfChunk];        // entries grouped by the higher circle j
    __shared__ uint32_t rcur[kMaxN / 2];    // per circle a 16-bit count / cursor, two per word
    __shared__ int scan_tmp[kHalfWaves];
    __shared__ float sum_tmp[kHalfWaves];

    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    int off, n;
    if (!instance_range(offset, b, total_n, &off, &n)) {
        if (tid == 0) energy[b] = __builtin_nanf("");
        return;
    }
    // list entries outside [0, col_len) are never read
    const int r0 = row[off], r1 = row[off + n];
    const int len = r1 - r0;
    if (!(r0 >= 0 && len >= 0 && (int64_t)r1 <= col_len)) {
        if (tid == 0) energy[b] = __builtin_nanf("");
        return;
    }
    typedef float v4f __attribute__((ext_vector_type(4)));
    typedef int v4i __attribute__((ext_vector_type(4)));
    typedef float v2f __attribute__((ext_vector_type(2)));
    constexpr int kPV = (kMaxN / 2 + kHalfBlock - 1) / kHalfBlock;   // float4 per thread
    constexpr int kCV = (kHalfChunk / 4 + kHalfBlock - 1) / kHalfBlock;  // int4 per thread
    constexpr int kEV = (kHalfChunk + kHalfBlock - 1) / kHalfBlock;      // entries per thread
    constexpr int kRC = kMaxN / kHalfBlock;                           // circles per thread
    const bool pos_al = (reinterpret_cast<uintptr_t>(xy + 2 * (int64_t)off) & 15) == 0;
    const int npv = pos_al ? n / 2 : 0;
    const v4f *psrc = reinterpret_cast<const v4f *>(xy + 2 * (int64_t)off);

    // One batch of streaming loads of the chunk starting at entry c0 (cl
    // entries): a scalar head up to 16-byte alignment, int4 loads, a tail.
    // The int4 loads are unconditional (indices clamped into range, the
    // extra lanes' values dropped when stored), so nothing waits between them.
    v4i cv[kCV];
    int head = 0, nv = 0;
    auto load_chunk = [&](int c0, int cl) {
        const int32_t *src = col + r0 + c0;
        const int mis = (int)((reinterpret_cast<uintptr_t>(src) & 15) >> 2);
        head = min(cl, (4 - mis) & 3);
        nv = (cl - head) >> 2;
        const v4i *csrc = reinterpret_cast<const v4i *>(src + head);
        if (nv > 0) {
#pragma unroll
            for (int u = 0; u < kCV; ++u) {
                const int v = tid + u * kHalfBlock;
                cv[u] = __builtin_nontemporal_load(csrc + (v < nv ? v : 0));
            }
        }
    };
    auto put = [&](int k, int v) {
        const int jj = v - off;
        ent[k].h.j = (unsigned)jj < (unsigned)n ? (uint16_t)jj : (uint16_t)0xFFFF;
    };
    auto store_chunk = [&](int c0, int cl) {
        const int32_t *src = col + r0 + c0;
        if (tid < head) put(tid, src[tid]);
        for (int k = head + 4 * nv + tid; k < cl; k += kHalfBlock) put(k, src[k]);
#pragma unroll
        for (int u = 0; u < kCV; ++u) {
            const int v = tid + u * kHalfBlock;
            if (v < nv) {
                const int k = head + 4 * v;
                put(k, cv[u].x); put(k + 1, cv[u].y); put(k + 2, cv[u].z); put(k + 3, cv[u].w);
            }
        }
    };

    v4f pv[kPV];
    if (npv > 0) {
#pragma unroll
        for (int u = 0; u < kPV; ++u) {
            const int k = tid + u * kHalfBlock;
            pv[u] = __builtin_nontemporal_load(psrc + (k < npv ? k : 0));
        }
    }
    int cl = len < kHalfChunk ? len : kHalfChunk;
    load_chunk(0, cl);
    // row bounds of this thread's circles tid + 512 c, relative to r0
    // (indices clamped to n); rows must be non-decreasing inside [r0, r1]
    int ra[kRC], rz[kRC];
    int bad = 0;
#pragma unroll
    for (int c = 0; c < kRC; ++c) {
        const int i = tid + c * kHalfBlock;
        ra[c] = row[off + (i < n ? i : n)];
        rz[c] = row[off + (i + 1 < n ? i + 1 : n)];
        if (i < n && !(r0 <= ra[c] && ra[c] <= rz[c] && rz[c] <= r1)) bad = 1;
        ra[c] -= r0;
        rz[c] -= r0;
    }
    // the row of every entry of the chunk, from the thread that owns it
    auto fill_rows = [&](int tid, int c0, int cl) {
#pragma unroll
        for (int c = 0; c < kRC; ++c) {
            const int i = tid + c * kHalfBlock;
            const int a = max(ra[c] - c0, 0), z = min(rz[c] - c0, cl);
            for (int k = a; k < z; ++k) ent[k].h.i = (uint16_t)i;
        }
    };
    if (!pos_al) {
        stage_positions<kHalfBlock>(xy, off, n, pos);
    } else if ((n & 1) && tid == 0) {
        pos[n - 1] = reinterpret_cast<const float2 *>(xy)[off + n - 1];
    }
#pragma unroll
    for (int u = 0; u < kPV; ++u) {
        const int k = tid + u * kHalfBlock;
        if (k < npv) reinterpret_cast<float4 *>(pos)[k] = make_float4(pv[u].x, pv[u].y, pv[u].z, pv[u].w);
    }
    store_chunk(0, cl);
    if (!bad) fill_rows(tid, 0, cl);
    for (int q = tid; q < kMaxN / 2; q += kHalfBlock) rcur[q] = 0u;
    if (__syncthreads_or(bad)) {
        if (tid == 0) energy[b] = __builtin_nanf("");
        return;
    }

    const float Rb = R[b];
    const float two_r = 2.0f * rad, four_r2 = two_r * two_r;
    float e = 0.0f;                 // this thread's energy terms
    float gxA[kRC], gyA[kRC];       // gradient of this thread's circles
#pragma unroll
    for (int c = 0; c < kRC; ++c) gxA[c] = gyA[c] = 0.f;
    auto cur16 = [&](int j) -> int { return (int)((rcur[j >> 1] >> ((j & 1) * 16)) & 0xffffu); };

    for (int c0 = 0;;) {
        // an opaque copy of the thread id: addresses and circle indices are
        // recomputed inside the loop instead of being hoisted and kept live
        int tid_l = (int)threadIdx.x;
        asm volatile("" : "+v"(tid_l));
        const int tid = tid_l;
        // ---- count the listed pairs (i < j < n) of every circle j ----------
#pragma unroll
        for (int u = 0; u < kEV; ++u) {
            const int k = tid + u * kHalfBlock;
            if (k < cl) {
                const uint32_t ij = ent[k].ij;
                const int i = (int)(ij >> 16), j = (int)(ij & 0xffffu);
                if (j < n && j > i) atomicAdd(&rcur[j >> 1], 1u << ((j & 1) * 16));
            }
        }
        __syncthreads();
        // exclusive scan: thread t holds the counts of circles 2t and 2t + 1
        // (word t; every count is below kHalfChunk)
        const uint32_t w = rcur[tid];
        const int k0 = (int)(w & 0xffffu), k1 = (int)(w >> 16);
        const int t2 = k0 + k1;
        int inc = t2;                     // inclusive scan over the wave
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int v = __shfl_up(inc, o, kWave);
            if ((tid & (kWave - 1)) >= o) inc += v;
        }
        if ((tid & (kWave - 1)) == kWave - 1) scan_tmp[tid / kWave] = inc;
        __syncthreads();
        int s0 = inc - t2;                // plus the totals of the waves before
#pragma unroll
        for (int q = 0; q < kHalfWaves - 1; ++q) s0 += q < tid / kWave ? scan_tmp[q] : 0;
        rcur[tid] = (uint32_t)s0 | ((uint32_t)(s0 + k0) << 16);
        __syncthreads();
        // ---- the pair pass: every listed pair once --------------------------
#pragma unroll
        for (int u = 0; u < kEV; ++u) {
            const int k = tid + u * kHalfBlock;
            if (k < cl) {
                const uint32_t ij = ent[k].ij;
                const int i = (int)(ij >> 16), j = (int)(ij & 0xffffu);
                float2 f = make_float2(0.f, 0.f);
                if (j < n && j > i) {
                    const float2 pi = pos[i], pj = pos[j];
                    const float dx = pi.x - pj.x, dy = pi.y - pj.y;
                    const float l2 = dx * dx + dy * dy;
                    const bool ov = l2 < four_r2;
                    const float il = (ov && l2 > 0.f) ? __builtin_amdgcn_rsqf(l2) : 0.f;
                    const float d = ov ? two_r - l2 * il : 0.f;
                    e += d * d;
                    const float kf = -2.f * d * il;
                    f = make_float2(kf * dx, kf * dy);
                    const uint32_t sh = (j & 1) * 16;
                    const uint32_t old = atomicAdd(&rcur[j >> 1], 1u << sh);
                    rev[(old >> sh) & 0xffffu] = (uint16_t)k;
                }
                ent[k].f = f;
            }
        }
        __syncthreads();
        // ---- the gather: partners below (bucket), then above (own row) ------
        // cursors now hold bucket ends: circle j's bucket is rev[e(j-1) .. e(j))
        int aA[kRC], nrA[kRC], fA[kRC], totA[kRC];
#pragma unroll
        for (int c = 0; c < kRC; ++c) {
            const int i = tid + c * kHalfBlock;
            aA[c] = i > 0 ? cur16(i - 1) : 0;
            const int z = i < n ? cur16(i) : aA[c];
            nrA[c] = z - aA[c];
            for (int q = aA[c] + 1; q < z; ++q) {        // sort the bucket by entry
                const uint16_t key = rev[q];
                int t = q - 1;
                while (t >= aA[c] && rev[t] > key) { rev[t + 1] = rev[t]; --t; }
                rev[t + 1] = key;
            }
            fA[c] = max(ra[c] - c0, 0);
            const int fz = min(rz[c] - c0, cl);
            totA[c] = nrA[c] + (fz > fA[c] ? fz - fA[c] : 0);
        }
        const int span = max(totA[0], totA[1]);
        for (int t = 0; t < span; ++t) {
            float2 fv[kRC];
            bool below[kRC];
#pragma unroll
            for (int c = 0; c < kRC; ++c) {
                below[c] = t < nrA[c];
                const int k = below[c] ? (int)rev[aA[c] + t] : fA[c] + t - nrA[c];
                fv[c] = t < totA[c] ? ent[k].f : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int c = 0; c < kRC; ++c) {
                if (t < totA[c]) {
                    if (below[c]) { gxA[c] -= fv[c].x; gyA[c] -= fv[c].y; }
                    else { gxA[c] += fv[c].x; gyA[c] += fv[c].y; }
                }
            }
        }
        c0 += cl;
        if (c0 >= len) break;
        // next chunk: every thread has finished with this one
        cl = len - c0 < kHalfChunk ? len - c0 : kHalfChunk;
        __syncthreads();
        load_chunk(c0, cl);
        store_chunk(c0, cl);
        fill_rows(tid, c0, cl);
        for (int q = tid; q < kMaxN / 2; q += kHalfBlock) rcur[q] = 0u;
        __syncthreads();
    }

    // containment terms; a non-finite position makes E NaN
    const bool g_al = (reinterpret_cast<uintptr_t>(grad) & 7) == 0;
#pragma unroll
    for (int c = 0; c < kRC; ++c) {
        const int i = tid + c * kHalfBlock;
        if (i >= n) break;
        const float2 pi = pos[i];
        float gx = gxA[c], gy = gyA[c];
        const float r2 = pi.x * pi.x + pi.y * pi.y;
        const float ir = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
        const float d0 = fmaxf(r2 * ir + rad - Rb, 0.f);
        e += d0 * d0;
        const float kc = 2.f * d0 * ir;
        gx += kc * pi.x;
        gy += kc * pi.y;
        if (!(isfinite(pi.x) && isfinite(pi.y))) e = __builtin_nanf("");
        if (grad) {
            if (g_al) {
                const v2f t = {gx, gy};
                __builtin_nontemporal_store(t, reinterpret_cast<v2f *>(grad) + (off + i));
            } else {
                __builtin_nontemporal_store(gx, &grad[2 * (int64_t)(off + i)]);
                __builtin_nontemporal_store(gy, &grad[2 * (int64_t)(off + i) + 1]);
            }
        }
    }
    const float tot = block_sum<kHalfBlock>(e, sum_tmp);
    if (tid == 0) energy[b] = tot;
}

// ---------------------------------------------------------------------------
// FP64 verify: every pair of the instance once.  Circle i is paired with
// the next floor((n-1)/2) circles cyclically (and, for even n, with i+n/2
// when i < n/2), which visits each unordered pair exactly once and gives
// every thread the same amount of work; the positions sit in LDS twice in
// a row, so partner i + t needs no wrap.  512 threads per instance, partner
// positions read four at a time so that LDS latency overlaps.  No
// contraction: products and sums round as written, like the oracle's.
// With R_tight set it also forms the smallest container of the unit
// circles, rho_max = max_i fl(|c_i| + 1): at any radius R >= rho_max every
// containment term (fl(|c_i| + 1) - R) is <= 0, so the layout is feasible
// there exactly when its pair energy is below tol.  R_tight[b] receives
// rho_max rounded up to FP32 when that holds and the value is below the
// instance's radius, else the instance's FP32 radius; feas_tight[b] is
// feasibility at R_tight[b].
// ---------------------------------------------------------------------------
constexpr int kVerifyBlock = 512;

__global__ __launch_bounds__(kVerifyBlock) void verify_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ R,
    const double *__restrict__ R64, const float *__restrict__ xy, int64_t total_n, double tol,
    double *__restrict__ energy64, double *__restrict__ max_pair,
    double *__restrict__ max_cont, int32_t *__restrict__ feasible, float *__restrict__ R_tight,
    int32_t *__restrict__ feas_tight)
{
#pragma clang fp contract(off)
    __shared__ float2 pos[2 * kMaxN];
    __shared__ double sum_tmp[kVerifyBlock / kWave];

    const int b = blockIdx.x;
    int off, n;
    if (!instance_range(offset, b, total_n, &off, &n)) {
        if (threadIdx.x == 0) {
            if (energy64) energy64[b] = __builtin_nan("");
            if (max_pair) max_pair[b] = __builtin_nan("");
            if (max_cont) max_cont[b] = __builtin_nan("");
            if (feasible) feasible[b] = 0;
            if (R_tight) R_tight[b] = R[b];
            if (feas_tight) feas_tight[b] = 0;
        }
        return;
    }
    {
        const float2 *src = reinterpret_cast<const float2 *>(xy) + off;
        for (int i = threadIdx.x; i < n; i += kVerifyBlock) {
            const float2 v = src[i];
            pos[i] = v;
            pos[i + n] = v;
        }
    }
    __syncthreads();
    const double Rb = R64 ? R64[b] : (double)R[b];
    double sp = 0.0, sc = 0.0, mp = 0.0, mc = 0.0, rm = 0.0;
    const int half = (n - 1) / 2;
    const bool even = (n & 1) == 0;
    for (int i = threadIdx.x; i < n; i += kVerifyBlock) {
        const double xi = pos[i].x, yi = pos[i].y;
        const int extra = (even && i < n / 2) ? 1 : 0;
        const int cnt = half + extra;
        // the overlap branch is rare (never taken once a layout is
        // feasible): a real branch, not a flattened square root per pair
        auto pair = [&](float2 pj) {
            const double dx = xi - (double)pj.x;
            const double dy = yi - (double)pj.y;
            const double l2 = dx * dx + dy * dy;
            if (__builtin_expect(l2 < 4.0, 0)) {
                const double d = 2.0 - sqrt(l2);
                sp = sp + d * d;
                mp = fmax(mp, d);
            }
        };
        int t = 1;
        for (; t + 3 <= cnt; t += 4) {
            float2 pj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) pj[u] = pos[i + t + u];
#pragma unroll
            for (int u = 0; u < 4; ++u) pair(pj[u]);
        }
        for (; t <= cnt; ++t) pair(pos[i + t]);
        const double rho = sqrt(xi * xi + yi * yi);
        rm = fmax(rm, rho + 1.0);
        const double d0 = (rho + 1.0) - Rb;
        if (d0 > 0.0) {
            sc = sc + d0 * d0;
            mc = fmax(mc, d0);
        }
        if (!(isfinite(xi) && isfinite(yi))) sc = __builtin_nan("");
    }
    const double Ep = block_sum<kVerifyBlock>(sp, sum_tmp);
    const double Ec = block_sum<kVerifyBlock>(sc, sum_tmp);
    const double Mp = block_max<kVerifyBlock>(mp, sum_tmp);
    const double Mc = block_max<kVerifyBlock>(mc, sum_tmp);
    const double Rm = R_tight ? block_max<kVerifyBlock>(rm, sum_tmp) : 0.0;
    if (threadIdx.x == 0) {
        const double E = Ep + Ec;
        const bool bad = E != E;     // a non-finite coordinate
        if (energy64) energy64[b] = E;
        if (max_pair) max_pair[b] = bad ? E : Mp;
        if (max_cont) max_cont[b] = bad ? E : Mc;
        if (feasible) feasible[b] = E < tol ? 1 : 0;
        if (R_tight) {
            const float rt = __double2float_ru(Rm);     // smallest FP32 value >= Rm
            const bool use = !bad && n > 0 && Ep < tol && (double)rt < Rb;
            R_tight[b] = use ? rt : R[b];
            if (feas_tight) feas_tight[b] = (use || E < tol) ? 1 : 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
hipError_t launch_build(const int32_t *offset, const float *R, const float *xy, int B,
                        int64_t total_n, double cutoff, float h_req, int format,
                        int32_t *row, void *col, int64_t capacity, int64_t *num_pairs,
                        int64_t *inst_total, hipStream_t s)
{
    const double c2 = cutoff * cutoff;
    const int full = format != kListHalf;
    build_count_kernel<<<B, kBuildBlock, 0, s>>>(offset, R, xy, total_n, c2, h_req, full, row,
                                                 inst_total);
    build_scan_kernel<<<1, kScanBlock, 0, s>>>(inst_total, B, total_n, row, num_pairs);
    if (format == kListLocal16)
        build_fill_kernel<uint16_t><<<B, kBuildBlock, 0, s>>>(
            offset, R, xy, total_n, c2, h_req, full, row, static_cast<uint16_t *>(col), capacity,
            inst_total);
    else
        build_fill_kernel<int32_t><<<B, kBuildBlock, 0, s>>>(
            offset, R, xy, total_n, c2, h_req, full, row, static_cast<int32_t *>(col), capacity,
            inst_total);
    return hipGetLastError();
}

hipError_t launch_energy_grad(const int32_t *offset, const float *R, const float *xy, int B,
                              int64_t total_n, const int32_t *row, const void *col,
                              int64_t col_len, int format, float rad, float *energy, float *grad,
                              hipStream_t s)
{
    if (format == kListHalf)
        energy_grad_half_kernel<<<B, kHalfBlock, 0, s>>>(
            offset, R, xy, total_n, row, static_cast<const int32_t *>(col), col_len, rad, energy, grad);
    else if (format == kListFull)
        energy_grad_full_kernel<int32_t><<<B, kSweepBlock, 0, s>>>(
            offset, R, xy, total_n, row, static_cast<const int32_t *>(col), col_len, rad, energy, grad);
    else
        energy_grad_full_kernel<uint16_t><<<B, kSweepBlock, 0, s>>>(
            offset, R, xy, total_n, row, static_cast<const uint16_t *>(col), col_len, rad, energy, grad);
    return hipGetLastError();
}

hipError_t launch_verify(const int32_t *offset, const float *R, const double *R64,
                         const float *xy, int B, int64_t total_n, double tol, double *e64,
                         double *mp, double *mc, int32_t *feas, hipStream_t s)
{
    verify_kernel<<<B, kVerifyBlock, 0, s>>>(offset, R, R64, xy, total_n, tol, e64, mp, mc, feas,
                                             nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_verify_tighten(const int32_t *offset, const float *R, const double *R64,
                                 const float *xy, int B, int64_t total_n, double tol,
                                 float *R_out, int32_t *feas, hipStream_t s)
{
    verify_kernel<<<B, kVerifyBlock, 0, s>>>(offset, R, R64, xy, total_n, tol, nullptr, nullptr,
                                             nullptr, nullptr, R_out, feas);
    return hipGetLastError();
}

}  // namespace pecc
