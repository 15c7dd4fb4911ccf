// Solution-space exploring and descent (SED, Sec. 5, Alg. 5), batched over
// independent chains: one SED iteration of every chain is
//   plan     m_b = max(1, J(E_b)) candidates (J = ceil(-log10 E), capped at
//            M; 0 once the chain's best energy is at or below e_stop), laid
//            out as one packed batch of instances (slot b*M + j, empty when
//            j >= m_b) so that the descent and the FP64 verify of all
//            candidates are single launches;
//   perturb  candidate j of chain b = x_b + r, every coordinate shifted by
//            r in [-0.8, 0.8) drawn from Philox4x64-10 at counter
//            (k / 4, j, iteration, b), key (seed, 0);
//   (descend and verify the candidate batch with the library's calls)
//   select   Eq. 18: the lowest-energy candidate when it beats the chain's
//            current energy, else one drawn with probabilities softmax(J),
//            the uniform from Philox at counter (2^63, 0, iteration, b);
//            the chain's best record follows.
// Philox4x64-10 (philox4x64 in pecc_device.hpp) gives every random number.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pecc_device.hpp"
#include "pecc_launch.hpp"

namespace pecc {
namespace {

// J = ceil(-log10 E) clipped to jmax; E <= 0 (or NaN) gives jmax.
__device__ __forceinline__ int sed_J(double E, int jmax)
{
    if (!(E > 0.0)) return jmax;
    const double j = ceil(-log10(E));
    return j > (double)jmax ? jmax : (int)j;
}

constexpr int kPlanBlock = 1024;

__global__ __launch_bounds__(kPlanBlock) void sed_plan_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ R, const double *__restrict__ R64,
    int B, int M, const double *__restrict__ E_cur, const double *__restrict__ E_best,
    double e_stop, int32_t *__restrict__ m_out, int32_t *__restrict__ cand_offset,
    float *__restrict__ cand_R, double *__restrict__ cand_R64)
{
    __shared__ int scan_tmp[kPlanBlock / kWave + 1];
    const int S = B * M;
    // chunk of consecutive slots per thread, then one block scan
    const int per = (S + kPlanBlock - 1) / kPlanBlock;
    const int s0 = threadIdx.x * per;
    auto slot_n = [&](int c) -> int {
        const int b = c / M, j = c - b * M;
        int n = offset[b + 1] - offset[b];
        if (n < 0 || n > kMaxN) n = 0;
        int m = (E_best[b] <= e_stop) ? 0 : sed_J(E_cur[b], M);
        if (m < 1 && !(E_best[b] <= e_stop)) m = 1;
        return j < m ? n : 0;
    };
    int local = 0;
    for (int c = s0; c < s0 + per && c < S; ++c) local += slot_n(c);
    int total;
    int run = block_exclusive_scan<kPlanBlock>(local, scan_tmp, &total);
    for (int c = s0; c < s0 + per && c < S; ++c) {
        cand_offset[c] = run;
        run += slot_n(c);
        const int b = c / M;
        cand_R[c] = R[b];
        cand_R64[c] = R64 ? R64[b] : (double)R[b];
    }
    if (threadIdx.x == 0) cand_offset[S] = total;
    for (int b = threadIdx.x; b < B; b += kPlanBlock) {
        int m = (E_best[b] <= e_stop) ? 0 : sed_J(E_cur[b], M);
        if (m < 1 && !(E_best[b] <= e_stop)) m = 1;
        m_out[b] = m;
    }
}

constexpr int kPerturbBlock = 256;

// One workgroup per candidate slot; thread t computes Philox blocks t,
// t + 256, ... (4 coordinates each).
__global__ __launch_bounds__(kPerturbBlock) void sed_perturb_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ xy, int M,
    const int32_t *__restrict__ m, const int32_t *__restrict__ cand_offset, uint64_t seed,
    int iter, float *__restrict__ cand_xy)
{
#pragma clang fp contract(off)   // u * 1.6 - 0.8 and x + r rounded step by step
    const int c = blockIdx.x;
    const int b = c / M, j = c - b * M;
    if (j >= m[b]) return;
    const int o = offset[b];
    const int n = cand_offset[c + 1] - cand_offset[c];   // n_b for an active slot
    const float *src = xy + 2 * (int64_t)o;
    float *dst = cand_xy + 2 * (int64_t)cand_offset[c];
    const int blocks = (2 * n + 3) / 4;
    for (int q = threadIdx.x; q < blocks; q += kPerturbBlock) {
        const U64x4 w = philox4x64((uint64_t)q, (uint64_t)(uint32_t)j, (uint64_t)(uint32_t)iter,
                                   (uint64_t)(uint32_t)b, seed, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * q + t;
            if (k < 2 * n) {
                const float u = (float)(w.w[t] >> 40) * 0x1p-24f;
                const float r = u * 1.6f - 0.8f;
                dst[k] = src[k] + r;
            }
        }
    }
}

constexpr int kSelectBlock = 256;

__global__ __launch_bounds__(kSelectBlock) void sed_select_kernel(
    const int32_t *__restrict__ offset, int M, const int32_t *__restrict__ m,
    const int32_t *__restrict__ cand_offset, const float *__restrict__ cand_xy,
    const double *__restrict__ cand_E, uint64_t seed, int iter, float *__restrict__ xy_cur,
    double *__restrict__ E_cur, float *__restrict__ xy_best, double *__restrict__ E_best,
    int32_t *__restrict__ chosen)
{
    __shared__ int pick;
    __shared__ int improve;
    const int b = blockIdx.x;
    const int mb = m[b];
    if (mb <= 0) {
        if (chosen && threadIdx.x == 0) chosen[b] = -1;
        return;
    }
    if (threadIdx.x == 0) {
        const double* Ec = cand_E + (int64_t)b * M;
        const double ecur = E_cur[b];
        int best = 0;
        for (int k = 1; k < mb; ++k)
            if (Ec[k] < Ec[best]) best = k;
        int k_sel = best;
        if (!(Ec[best] < ecur)) {
            // softmax(J) draw; J is recomputed per pass (no per-thread array)
            int jm = -1000000;
            for (int k = 0; k < mb; ++k) {
                const int Jk = sed_J(Ec[k], M);
                jm = Jk > jm ? Jk : jm;
            }
            double tot = 0.0;
            for (int k = 0; k < mb; ++k) tot += exp((double)(sed_J(Ec[k], M) - jm));
            const U64x4 w = philox4x64(1ULL << 63, 0, (uint64_t)(uint32_t)iter,
                                       (uint64_t)(uint32_t)b, seed, 0);
            const double u = (double)(w.w[0] >> 11) * 0x1p-53;
            const double target = u * tot;
            double cdf = 0.0;
            k_sel = mb - 1;
            for (int k = 0; k < mb; ++k) {
                cdf += exp((double)(sed_J(Ec[k], M) - jm));
                if (target < cdf) { k_sel = k; break; }
            }
        }
        const double ek = Ec[k_sel];
        E_cur[b] = ek;
        const int better = ek < E_best[b];
        if (better) E_best[b] = ek;
        pick = k_sel;
        improve = better;
        if (chosen) chosen[b] = k_sel;
    }
    __syncthreads();
    const int c = b * M + pick;
    const int o = offset[b];
    const int n = cand_offset[c + 1] - cand_offset[c];
    const float2 *src = reinterpret_cast<const float2 *>(cand_xy) + cand_offset[c];
    float2 *cur = reinterpret_cast<float2 *>(xy_cur) + o;
    float2 *bst = reinterpret_cast<float2 *>(xy_best) + o;
    for (int i = threadIdx.x; i < n; i += kSelectBlock) {
        const float2 v = src[i];
        cur[i] = v;
        if (improve) bst[i] = v;
    }
}

}  // namespace

hipError_t launch_sed_plan(const int32_t *offset, const float *R, const double *R64, int B, int M,
                           const double *E_cur, const double *E_best, double e_stop,
                           int32_t *m_out, int32_t *cand_offset, float *cand_R, double *cand_R64,
                           hipStream_t s)
{
    hipLaunchKernelGGL(sed_plan_kernel, dim3(1), dim3(kPlanBlock), 0, s, offset, R, R64, B, M,
                       E_cur, E_best, e_stop, m_out, cand_offset, cand_R, cand_R64);
    return hipGetLastError();
}

hipError_t launch_sed_perturb(const int32_t *offset, const float *xy, int B, int M,
                              const int32_t *m, const int32_t *cand_offset, uint64_t seed,
                              int iter, float *cand_xy, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(sed_perturb_kernel, dim3(B * M), dim3(kPerturbBlock), 0, s, offset, xy, M,
                       m, cand_offset, seed, iter, cand_xy);
    return hipGetLastError();
}

hipError_t launch_sed_select(const int32_t *offset, int B, int M, const int32_t *m,
                             const int32_t *cand_offset, const float *cand_xy,
                             const double *cand_E, uint64_t seed, int iter, float *xy_cur,
                             double *E_cur, float *xy_best, double *E_best, int32_t *chosen,
                             hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(sed_select_kernel, dim3(B), dim3(kSelectBlock), 0, s, offset, M, m,
                       cand_offset, cand_xy, cand_E, seed, iter, xy_cur, E_cur, xy_best, E_best,
                       chosen);
    return hipGetLastError();
}

}  // namespace pecc
