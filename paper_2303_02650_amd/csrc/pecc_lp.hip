// Learned proposal for the perturbation step of SED (Sec. 5, Alg. 5): the
// solution-space exploring step relocates a few circles, and a small network
// scores candidate relocations (circle i, destination q) from local features
// so that the best-scored distinct circles are moved.
//
// Kernels
//   features_kernel   8 features per candidate, cell grid of side >= 4 in LDS,
//                     FP64 distances on the FP32 coordinates
//   mlp_forward_kernel    8 -> 64 -> 64 -> 1 erf-GELU network on BF16 MFMA
//   mlp_grad_kernel       forward + backward of the mean BCE-with-logits loss,
//                         per-workgroup partial gradients (MFMA for every
//                         contraction), then grad_reduce_kernel sums them in a
//                         fixed order
//   adam_kernel           Adam on FP32 master weights
//   propose_kernel        top-k distinct circles by score (or the first k
//                         distinct candidates without usable scores) and the
//                         relocated layout
//   accept_kernel         keep the relocated-and-descended layout when its FP64
//                         energy is lower
//
// MFMA (gfx950, v_mfma_f32_16x16x32_bf16), per wave64 lane l, g = l / 16,
// r = l % 16:  A operand  A[r][8g + i],  B operand  B[8g + i][r]  (i < 8),
// result D[4g + i][r] (i < 4).  The network runs with neurons as the M
// dimension and rows (samples) as N, so a layer's result, lane (g, r) holding
// neurons 16t + 4g + i of row r for the four neuron tiles t, is already laid
// out as the next layer's B operand once the K slots are permuted to match:
// K slot (g, i') of chunk c is neuron 16 (2c + i' / 4) + 4g + i' % 4.  The
// weight fragments are read with that permutation, so no data moves between
// lanes.  The forward feeds the features and the first activations as BF16
// high + low pairs (x = hi + lo to about 2^-16), which keeps the logits near
// FP32 accuracy; the features' pair fits in the K slots the 8 inputs leave
// free.  Contractions over rows (weight gradients) go through a per-wave LDS
// stage that transposes rows into the K dimension.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pecc_device.hpp"
#include "pecc_launch.hpp"

namespace pecc {
namespace {

constexpr int kFeat = 8, kHid = 64, kParams = 4801;
constexpr int oW1 = 0, oB1 = 512, oW2 = 576, oB2 = 4672, oW3 = 4736, oB3 = 4800;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Features
// ---------------------------------------------------------------------------
constexpr int kFeatBlock = 256;
constexpr int kFeatChunk = 1024;     // candidates per workgroup
constexpr float kDensRadius = 4.0f;  // widest radius a feature looks at

struct FeatShared {
    float2 pos[kMaxN];
    int cell_start[kMaxCells + 1];
    uint16_t cell_circ[kMaxN];
    uint16_t slot_tmp[kMaxN];
    int scan_tmp[kFeatBlock / 64 + 1];
};

// Overlap energy, neighbor count, boundary gap and density around point p
// over the circles j != skip (the circle that would move is lifted out).
__device__ void feature_quad(const FeatShared &S, const Grid &g, double R, int skip, float2 p,
                             float *f)
{
#pragma clang fp contract(off)   // distances rounded operation by operation, like the oracle
    const double px = (double)p.x, py = (double)p.y;
    double e = 0.0;
    int near = 0, dens = 0;
    for_each_candidate(skip, p, g, S.cell_start, S.cell_circ, [&](int j) {
#pragma clang fp contract(off)
        const double dx = px - (double)S.pos[j].x;
        const double dy = py - (double)S.pos[j].y;
        const double l2 = dx * dx + dy * dy;
        if (l2 < 4.0) {
            const double d = 2.0 - sqrt(l2);
            e = e + d * d;
        }
        near += l2 < 5.29;
        dens += l2 < 16.0;
    });
    const double rho = sqrt(px * px + py * py);
    const double d0 = (rho + 1.0) - R;
    if (d0 > 0.0) e = e + d0 * d0;
    f[0] = (float)(log10(e + 1e-20) / 20.0 + 1.0);
    f[1] = (float)near;
    f[2] = (float)((R - 1.0 - rho) / R);
    f[3] = (float)((double)dens / (16.0 * 3.14159265358979323846));
}

__global__ __launch_bounds__(kFeatBlock) void features_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ Rf,
    const double *__restrict__ R64, const float *__restrict__ xy, int C,
    const int32_t *__restrict__ cand_circle, const float *__restrict__ cand_dest,
    float *__restrict__ feat)
{
    __shared__ FeatShared S;
    const int b = blockIdx.y;
    const int o = offset[b];
    int n = offset[b + 1] - o;
    const bool bad = n < 0 || n > kMaxN;
    if (bad) n = 0;
    const double R = R64 ? R64[b] : (double)Rf[b];
    const float2 *p2 = reinterpret_cast<const float2 *>(xy) + o;
    for (int i = threadIdx.x; i < n; i += kFeatBlock) S.pos[i] = p2[i];
    __syncthreads();
    const Grid g = make_grid(Rf[b], kDensRadius * (1.0f + kCellSafety));
    bin_circles<kFeatBlock>(S.pos, n, g, S.cell_start, S.cell_circ, S.slot_tmp, S.scan_tmp);
    // ascending order inside each cell: every sum runs in a fixed order
    for (int c = threadIdx.x; c < g.nc * g.nc; c += kFeatBlock) {
        const int a = S.cell_start[c], e = S.cell_start[c + 1];
        for (int k = a + 1; k < e; ++k) {
            const uint16_t v = S.cell_circ[k];
            int m = k - 1;
            while (m >= a && S.cell_circ[m] > v) {
                S.cell_circ[m + 1] = S.cell_circ[m];
                --m;
            }
            S.cell_circ[m + 1] = v;
        }
    }
    __syncthreads();
    const int c0 = blockIdx.x * kFeatChunk;
    const int c1 = min(C, c0 + kFeatChunk);
    for (int k = c0 + (int)threadIdx.x; k < c1; k += kFeatBlock) {
        const int64_t gi = (int64_t)b * C + k;
        const int i = cand_circle[gi];
        float f[8];
        if (bad || i < 0 || i >= n) {
#pragma unroll
            for (int q = 0; q < 8; ++q) f[q] = __builtin_nanf("");
        } else {
            feature_quad(S, g, R, i, S.pos[i], f);
            feature_quad(S, g, R, i, reinterpret_cast<const float2 *>(cand_dest)[gi], f + 4);
        }
        float4 *dst = reinterpret_cast<float4 *>(feat + gi * 8);
        dst[0] = make_float4(f[0], f[1], f[2], f[3]);
        dst[1] = make_float4(f[4], f[5], f[6], f[7]);
    }
}

// ---------------------------------------------------------------------------
// Network: weights in LDS as BF16 (round to nearest even of the FP32 master)
// ---------------------------------------------------------------------------
struct NetWeights {
    alignas(16) __bf16 w1[kHid * kFeat];     // [n][k]
    alignas(16) __bf16 w2[kHid * kHid];      // [n][k]
    alignas(16) __bf16 w2t[kHid * kHid];     // [k][n]  (backward)
    float b1[kHid], b2[kHid], w3[kHid];   // w3 holds the BF16 values
    float b3;
};

template <int BLOCK>
__device__ void load_weights(const float *__restrict__ P, NetWeights &W, bool transpose)
{
    for (int k = threadIdx.x; k < kParams; k += BLOCK) {
        const float v = P[k];
        if (k < oB1) {
            W.w1[k] = (__bf16)v;
        } else if (k < oW2) {
            W.b1[k - oB1] = v;
        } else if (k < oB2) {
            const int q = k - oW2;
            W.w2[q] = (__bf16)v;
            if (transpose) W.w2t[(q % kHid) * kHid + q / kHid] = (__bf16)v;
        } else if (k < oW3) {
            W.b2[k - oB2] = v;
        } else if (k < oB3) {
            W.w3[k - oW3] = (float)(__bf16)v;
        } else {
            W.b3 = v;
        }
    }
}

// erf(x) by the rational approximation 7.1.26 of Abramowitz and Stegun
// (Handbook of Mathematical Functions): erf(x) = 1 - (a1 t + ... + a5 t^5)
// exp(-x^2) with t = 1 / (1 + p x) for x >= 0, odd in x; at most 1.5e-7 from
// erf in exact arithmetic, about 6e-7 in FP32 with the hardware reciprocal
// and exponential.  gauss receives the exp(-x^2) it forms.  One reciprocal,
// one exponential and seven FMAs, against the library erff's longer
// piecewise evaluation: the network's 128 activations per row are most of
// its vector work.
__device__ __forceinline__ float erf_as(float x, float &gauss)
{
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float q = fmaf(t, 1.061405429f, -1.453152027f);
    q = fmaf(t, q, 1.421413741f);
    q = fmaf(t, q, -0.284496736f);
    q = fmaf(t, q, 0.254829592f);
    gauss = __expf(-ax * ax);
    return copysignf(fmaf(-t * q, gauss, 1.0f), x);
}

// GELU(t) = t Phi(t) = 0.5 t (1 + erf(t / sqrt 2)) and its derivative
// Phi(t) + t phi(t), phi(t) = exp(-t^2 / 2) / sqrt(2 pi) (the same
// exponential as the erf's).
__device__ __forceinline__ float gelu(float t)
{
    float gs;
    return 0.5f * t * (1.0f + erf_as(t * 0.70710678118654752f, gs));
}

__device__ __forceinline__ float gelu_prime(float t)
{
    float gs;
    const float e = erf_as(t * 0.70710678118654752f, gs);
    return 0.5f * (1.0f + e) + t * 0.39894228040143268f * gs;
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 cat(bf16x4 lo, bf16x4 hi)
{
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

// A fragment of W1 for neuron tile t: row 16t + r, K slots 0..7 (g = 0) and
// again 8..15 (g = 1), which multiply the high and low BF16 parts of x.
__device__ __forceinline__ bf16x8 frag_w1(const NetWeights &W, int t, int g, int r)
{
    const bf16x8 v = *reinterpret_cast<const bf16x8 *>(&W.w1[(16 * t + r) * kFeat]);
    const bf16x8 z = {};
    return g < 2 ? v : z;
}

// A fragment of M (w2 or w2t) for output tile t and K chunk c under the
// permuted K order: slots i' < 4 are columns 32c + 4g + i', slots i' >= 4 are
// columns 32c + 16 + 4g + i' - 4.
__device__ __forceinline__ bf16x8 frag_perm(const __bf16 *M, int t, int c, int g, int r)
{
    const __bf16 *row = M + (16 * t + r) * kHid + 32 * c + 4 * g;
    return cat(*reinterpret_cast<const bf16x4 *>(row), *reinterpret_cast<const bf16x4 *>(row + 16));
}

// B fragments of chunk c from a result held as v[t][i] (neuron 16t + 4g + i):
// hi gets the BF16 rounding, lo the BF16 rounding of the remainder, so that
// hi + lo carries v to about 2^-16 relative.
__device__ __forceinline__ void frag_chunk(const float (&v)[4][4], int c, bf16x8 &hi, bf16x8 &lo)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float x = v[2 * c + h][i];
            const __bf16 xh = (__bf16)x;
            hi[4 * h + i] = xh;
            lo[4 * h + i] = (__bf16)(x - (float)xh);
        }
    }
}

// Single BF16 rounding (the backward contractions).
__device__ __forceinline__ bf16x8 frag_chunk1(const float (&v)[4][4], int c)
{
    bf16x8 b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        b[i] = (__bf16)v[2 * c][i];
        b[4 + i] = (__bf16)v[2 * c + 1][i];
    }
    return b;
}

// B fragment of the input layer: the 8 features of row r, their BF16
// high parts in the slots of g = 0 and the low parts in those of g = 1.
__device__ __forceinline__ bf16x8 frag_x(const float *__restrict__ X, int64_t row, int64_t rows,
                                         int g)
{
    bf16x8 b = {};
    if (g < 2 && row < rows) {
        const float4 *p = reinterpret_cast<const float4 *>(X + row * kFeat);
        const float4 u = p[0], v = p[1];
        const float f[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const __bf16 h = (__bf16)f[i];
            b[i] = g == 0 ? h : (__bf16)(f[i] - (float)h);
        }
    }
    return b;
}

// Forward pass of 16 rows; a1/a2 get the pre-activations (neuron 16t+4g+i of
// this lane's row), h1b the BF16 high parts of h1 as B fragments, h2 the
// second activations; the return value is the logit of row r in every lane.
__device__ __forceinline__ float forward16(const NetWeights &W, bf16x8 xb, int g, int r,
                                           float (&a1)[4][4], float (&a2)[4][4], bf16x8 (&h1b)[2],
                                           float (&h2)[4][4])
{
    float h1[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f32x4 d = mfma(frag_w1(W, t, g, r), xb, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a1[t][i] = d[i] + W.b1[16 * t + 4 * g + i];
            h1[t][i] = gelu(a1[t][i]);
        }
    }
    bf16x8 h1l[2];
    frag_chunk(h1, 0, h1b[0], h1l[0]);
    frag_chunk(h1, 1, h1b[1], h1l[1]);
    float zp = 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bf16x8 w0 = frag_perm(W.w2, t, 0, g, r), w1 = frag_perm(W.w2, t, 1, g, r);
        f32x4 d = mfma(w0, h1b[0], f32x4{0.f, 0.f, 0.f, 0.f});
        d = mfma(w1, h1b[1], d);
        d = mfma(w0, h1l[0], d);
        d = mfma(w1, h1l[1], d);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int nn = 16 * t + 4 * g + i;
            a2[t][i] = d[i] + W.b2[nn];
            h2[t][i] = gelu(a2[t][i]);
            zp += W.w3[nn] * h2[t][i];
        }
    }
    // sum over the four lane groups that share row r
    zp += __shfl_xor(zp, 16);
    zp += __shfl_xor(zp, 32);
    return zp + W.b3;
}

constexpr int kMlpBlock = 256;

__global__ __launch_bounds__(kMlpBlock) void mlp_forward_kernel(const float *__restrict__ P,
                                                                const float *__restrict__ X,
                                                                int64_t rows,
                                                                float *__restrict__ Z)
{
    __shared__ NetWeights W;
    load_weights<kMlpBlock>(P, W, false);
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int64_t waves = (int64_t)gridDim.x * (kMlpBlock / 64);
    const int64_t tiles = (rows + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * (kMlpBlock / 64) + (threadIdx.x >> 6); tile < tiles;
         tile += waves) {
        const int64_t row = tile * 16 + r;
        float a1[4][4], a2[4][4], h2[4][4];
        bf16x8 h1b[2];
        const float z = forward16(W, frag_x(X, row, rows, g), g, r, a1, a2, h1b, h2);
        if (g == 0 && row < rows) Z[row] = z;
    }
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------
struct WaveStage {                    // one per wave: 32 rows of the pair tile
    alignas(16) __bf16 da2[kHid][32];
    alignas(16) __bf16 h1[kHid][32];
    alignas(16) __bf16 da1[kHid][32];
    alignas(16) __bf16 x[16][32];     // features 8..15 stay zero
};

struct GradShared {
    NetWeights W;
    union {
        WaveStage stage[kMlpBlock / 64];
        float sum[kParams + 1];       // workgroup reduction after the row loop
    } u;
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float sum16(float v)   // over the 16 lanes of a group
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// Per workgroup: partial d(sum of row losses)/d params (not yet divided by
// rows) and the partial loss sum, written to part[blockIdx.x][0..kParams].
__global__ __launch_bounds__(kMlpBlock) void mlp_grad_kernel(const float *__restrict__ P,
                                                             const float *__restrict__ X,
                                                             const float *__restrict__ Y,
                                                             int64_t rows,
                                                             float *__restrict__ part)
{
    __shared__ GradShared S;
    load_weights<kMlpBlock>(P, S.W, true);
    const NetWeights &W = S.W;
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    WaveStage &st = S.u.stage[wv];
    for (int k = lane; k < 16 * 32; k += 64) (&st.x[0][0])[k] = (__bf16)0.0f;
    __syncthreads();

    f32x4 gW2[4][4], gW1[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float gW3[4][4] = {}, gB2[4][4] = {}, gB1[4][4] = {};
    float gB3 = 0.0f, lsum = 0.0f;

    const int64_t waves = (int64_t)gridDim.x * (kMlpBlock / 64);
    const int64_t pairs = (rows + 31) / 32;
    for (int64_t pt = (int64_t)blockIdx.x * (kMlpBlock / 64) + wv; pt < pairs; pt += waves) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int64_t row = pt * 32 + 16 * s + r;
            const bool valid = row < rows;
            const bf16x8 xb = frag_x(X, row, rows, g);
            float a1[4][4], a2[4][4], h2[4][4];
            bf16x8 h1b[2];
            const float z = forward16(W, xb, g, r, a1, a2, h1b, h2);
            const float y = valid ? Y[row] : 0.0f;
            const float dz = valid ? 1.0f / (1.0f + __expf(-z)) - y : 0.0f;
            if (g == 0 && valid) {
                lsum += fmaxf(z, 0.0f) - z * y + log1pf(__expf(-fabsf(z)));
                gB3 += dz;
            }
            float da2[4][4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int nn = 16 * t + 4 * g + i;
                    gW3[t][i] += dz * h2[t][i];
                    da2[t][i] = dz * W.w3[nn] * gelu_prime(a2[t][i]);
                    gB2[t][i] += da2[t][i];
                }
            // dh1 = W2^T da2 (same permuted K order as the forward)
            const bf16x8 db0 = frag_chunk1(da2, 0), db1 = frag_chunk1(da2, 1);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                f32x4 d = mfma(frag_perm(W.w2t, t, 0, g, r), db0, f32x4{0.f, 0.f, 0.f, 0.f});
                d = mfma(frag_perm(W.w2t, t, 1, g, r), db1, d);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int nn = 16 * t + 4 * g + i;
                    const float da1 = d[i] * gelu_prime(a1[t][i]);
                    gB1[t][i] += da1;
                    st.da1[nn][16 * s + r] = (__bf16)da1;
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int nn = 16 * t + 4 * g + i;
                    st.da2[nn][16 * s + r] = (__bf16)da2[t][i];
                    st.h1[nn][16 * s + r] = (t & 1) ? h1b[t >> 1][4 + i] : h1b[t >> 1][i];
                }
            if (g == 0) {
#pragma unroll
                for (int f = 0; f < 8; ++f) st.x[f][16 * s + r] = xb[f];
            }
        }
        wave_sync();
        // dW2[n][k] += sum_rows da2[n][row] h1[k][row]; dW1[n][f] likewise with x
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&st.da2[16 * tn + r][8 * g]);
#pragma unroll
            for (int tk = 0; tk < 4; ++tk) {
                const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&st.h1[16 * tk + r][8 * g]);
                gW2[tn][tk] = mfma(a, b, gW2[tn][tk]);
            }
            const bf16x8 a1f = *reinterpret_cast<const bf16x8 *>(&st.da1[16 * tn + r][8 * g]);
            const bf16x8 xf = *reinterpret_cast<const bf16x8 *>(&st.x[r][8 * g]);
            gW1[tn] = mfma(a1f, xf, gW1[tn]);
        }
        wave_sync();
    }

    // ---- workgroup reduction in a fixed order: wave 0 stores, waves 1..3 add
    __syncthreads();                  // the stages are dead; reuse as sum[]
    float *sum = S.u.sum;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            gW3[t][i] = sum16(gW3[t][i]);
            gB2[t][i] = sum16(gB2[t][i]);
            gB1[t][i] = sum16(gB1[t][i]);
        }
    gB3 = sum16(gB3);
    lsum = sum16(lsum);
    for (int w = 0; w < kMlpBlock / 64; ++w) {
        if (wv == w) {
            const bool first = w == 0;
#pragma unroll
            for (int tn = 0; tn < 4; ++tn)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int nn = 16 * tn + 4 * g + i;
#pragma unroll
                    for (int tk = 0; tk < 4; ++tk) {
                        float *q = &sum[oW2 + nn * kHid + 16 * tk + r];
                        *q = first ? gW2[tn][tk][i] : *q + gW2[tn][tk][i];
                    }
                    if (r < kFeat) {
                        float *q = &sum[oW1 + nn * kFeat + r];
                        *q = first ? gW1[tn][i] : *q + gW1[tn][i];
                    }
                    if (r == 0) {
                        float *q3 = &sum[oW3 + nn], *q2 = &sum[oB2 + nn], *q1 = &sum[oB1 + nn];
                        *q3 = first ? gW3[tn][i] : *q3 + gW3[tn][i];
                        *q2 = first ? gB2[tn][i] : *q2 + gB2[tn][i];
                        *q1 = first ? gB1[tn][i] : *q1 + gB1[tn][i];
                    }
                }
            if (lane == 0) {
                sum[oB3] = first ? gB3 : sum[oB3] + gB3;
                sum[kParams] = first ? lsum : sum[kParams] + lsum;
            }
        }
        __syncthreads();
    }
    float *dst = part + (int64_t)blockIdx.x * (kParams + 1);
    for (int k = threadIdx.x; k <= kParams; k += kMlpBlock) dst[k] = sum[k];
}

// grad[k] = (sum over workgroups, in workgroup order) / rows; loss likewise.
__global__ void grad_reduce_kernel(const float *__restrict__ part, int nparts, int64_t rows,
                                   float *__restrict__ grad, float *__restrict__ loss)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > kParams) return;
    float s = 0.0f;
    for (int w = 0; w < nparts; ++w) s += part[(int64_t)w * (kParams + 1) + k];
    const float v = rows > 0 ? s / (float)rows : 0.0f;
    if (k < kParams) {
        grad[k] = v;
    } else if (loss) {
        *loss = v;
    }
}

// ---------------------------------------------------------------------------
// Adam (step counter on the device: t = *step + 1 is used, then stored)
// ---------------------------------------------------------------------------
__global__ void adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, const int32_t *__restrict__ step,
                            AdamArgs a, int count)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int t = *step + 1;
    const float c1 = (float)(1.0 - pow((double)a.b1, (double)t));
    const float c2 = (float)(1.0 - pow((double)a.b2, (double)t));
    const float gk = g[k];
    const float mk = a.b1 * m[k] + (1.0f - a.b1) * gk;
    const float vk = a.b2 * v[k] + (1.0f - a.b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= a.lr * (mk / c1) / (sqrtf(vk / c2) + a.eps);
}

__global__ void step_bump_kernel(int32_t *step) { *step += 1; }

// ---------------------------------------------------------------------------
// Proposal: best candidate per circle by a 64-bit key (score, then lower
// candidate index), bitonic sort of the keys, first k taken.
// ---------------------------------------------------------------------------
constexpr int kPropBlock = 256;

__device__ __forceinline__ uint32_t ordered_bits(float s)
{
    s = s + 0.0f;                                  // -0 -> +0: equal scores tie
    const uint32_t u = __float_as_uint(s);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(kPropBlock) void propose_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ xy, int C,
    const int32_t *__restrict__ cand_circle, const float *__restrict__ cand_dest,
    const float *__restrict__ scores, int k, int32_t *__restrict__ selected,
    float *__restrict__ xy_out)
{
    __shared__ unsigned long long key[kMaxN];
    __shared__ int any_nan;
    const int b = blockIdx.x;
    const int o = offset[b];
    int n = offset[b + 1] - o;
    if (n < 0 || n > kMaxN) n = 0;
    const float2 *src = reinterpret_cast<const float2 *>(xy) + o;
    float2 *dst = reinterpret_cast<float2 *>(xy_out) + o;
    for (int i = threadIdx.x; i < n; i += kPropBlock) dst[i] = src[i];
    for (int i = threadIdx.x; i < kMaxN; i += kPropBlock) key[i] = 0ull;
    if (threadIdx.x == 0) any_nan = 0;
    __syncthreads();
    const int64_t base = (int64_t)b * C;
    if (scores) {
        for (int c = threadIdx.x; c < C; c += kPropBlock)
            if (scores[base + c] != scores[base + c]) any_nan = 1;
    }
    __syncthreads();
    const bool use = scores != nullptr && any_nan == 0;
    for (int c = threadIdx.x; c < C; c += kPropBlock) {
        const int i = cand_circle[base + c];
        if (i < 0 || i >= n) continue;
        const uint32_t hi = use ? ordered_bits(scores[base + c]) : 0x80000000u;
        const unsigned long long kk = ((unsigned long long)hi << 32) | (0xffffffffu - (uint32_t)c);
        atomicMax(&key[i], kk);
    }
    __syncthreads();
    for (int size = 2; size <= kMaxN; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < kMaxN / 2; t += kPropBlock) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const unsigned long long ki = key[i], kj = key[j];
                if ((ki > kj) == up) {
                    key[i] = kj;
                    key[j] = ki;
                }
            }
            __syncthreads();
        }
    }
    // ascending order: the best key is last
    for (int q = threadIdx.x; q < k; q += kPropBlock) {
        const unsigned long long kk = q < kMaxN ? key[kMaxN - 1 - q] : 0ull;
        int32_t c = -1;
        if (kk != 0ull) {
            c = (int32_t)(0xffffffffu - (uint32_t)(kk & 0xffffffffull));
            const int i = cand_circle[base + c];
            dst[i] = reinterpret_cast<const float2 *>(cand_dest)[base + c];
        }
        if (selected) selected[(int64_t)b * k + q] = c;
    }
}

// ---------------------------------------------------------------------------
// Acceptance: keep the new layout of instance b when e_new[b] < e_cur[b].
// ---------------------------------------------------------------------------
constexpr int kAcceptBlock = 256;

__global__ __launch_bounds__(kAcceptBlock) void accept_kernel(
    const int32_t *__restrict__ offset, float *__restrict__ xy_cur, double *__restrict__ e_cur,
    const float *__restrict__ xy_new, const double *__restrict__ e_new,
    int32_t *__restrict__ accepted)
{
    const int b = blockIdx.x;
    const int o = offset[b];
    int n = offset[b + 1] - o;
    if (n < 0 || n > kMaxN) n = 0;
    const double en = e_new[b], ec = e_cur[b];
    const bool take = en < ec;
    __syncthreads();                 // every thread has read e_cur[b]
    if (take) {
        const float2 *src = reinterpret_cast<const float2 *>(xy_new) + o;
        float2 *dst = reinterpret_cast<float2 *>(xy_cur) + o;
        for (int i = threadIdx.x; i < n; i += kAcceptBlock) dst[i] = src[i];
    }
    if (threadIdx.x == 0) {
        if (take) e_cur[b] = en;
        if (accepted) accepted[b] = take ? 1 : 0;
    }
}

int mlp_grid(int64_t rows, int per_wg_rows)
{
    const int64_t need = (rows + per_wg_rows - 1) / per_wg_rows;
    return (int)(need < 1 ? 1 : (need > 256 ? 256 : need));
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_features(const int32_t *offset, const float *R, const double *R64,
                           const float *xy, int B, int C, const int32_t *cand_circle,
                           const float *cand_dest, float *feat, hipStream_t s)
{
    if (B <= 0 || C <= 0) return hipSuccess;
    dim3 grid((C + kFeatChunk - 1) / kFeatChunk, B);
    hipLaunchKernelGGL(features_kernel, grid, dim3(kFeatBlock), 0, s, offset, R, R64, xy, C,
                       cand_circle, cand_dest, feat);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *params, const float *X, int64_t rows, float *Z,
                              hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    // at least two 16-row tiles per wave, at most 4 workgroups per CU
    const int64_t need = (rows + 4 * 32 - 1) / (4 * 32);
    const int grid = (int)(need > 1024 ? 1024 : need);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid), dim3(kMlpBlock), 0, s, params, X, rows, Z);
    return hipGetLastError();
}

size_t mlp_grad_workspace_bytes(int64_t rows)
{
    return (size_t)mlp_grid(rows, 4 * 32) * (kParams + 1) * sizeof(float);
}

hipError_t launch_mlp_grad(const float *params, const float *X, const float *Y, int64_t rows,
                           float *loss, float *grad, void *ws, hipStream_t s)
{
    const int grid = mlp_grid(rows, 4 * 32);
    float *part = static_cast<float *>(ws);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(grid), dim3(kMlpBlock), 0, s, params, X, Y, rows,
                       part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((kParams + 1 + 255) / 256), dim3(256), 0, s, part,
                       grid, rows, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *params, float *m, float *v, const float *grad, int32_t *step,
                       const AdamArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, params, m, v,
                       grad, step, a, kParams);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(step_bump_kernel, dim3(1), dim3(1), 0, s, step);
    return hipGetLastError();
}

hipError_t launch_propose(const int32_t *offset, const float *xy, int B, int C,
                          const int32_t *cand_circle, const float *cand_dest, const float *scores,
                          int k, int32_t *selected, float *xy_out, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(propose_kernel, dim3(B), dim3(kPropBlock), 0, s, offset, xy, C,
                       cand_circle, cand_dest, scores, k, selected, xy_out);
    return hipGetLastError();
}

hipError_t launch_accept(const int32_t *offset, float *xy_cur, double *e_cur, const float *xy_new,
                         const double *e_new, int B, int32_t *accepted, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(accept_kernel, dim3(B), dim3(kAcceptBlock), 0, s, offset, xy_cur, e_cur,
                       xy_new, e_new, accepted);
    return hipGetLastError();
}

}  // namespace pecc
