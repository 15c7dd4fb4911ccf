// k-batch partitions of the geometric batch optimization (Sec. 4.1): the
// circles of an instance are ordered by a key and cut into k consecutive
// runs, batch p holding floor(n/k) + [p < n mod k] circles.
//   sector   polar angle atan2(y, x) in (-pi, pi], compared exactly: the
//            classes y < 0, (y = 0, x >= 0), y > 0, (y = 0, x < 0) in this
//            order, and inside the first and third class a before b iff
//            x_a y_b - y_a x_b > 0 (FP64 products of FP32 values are exact,
//            so the sign of their difference is exact);
//   annulus  x^2 + y^2 in FP64;
//   fence    x;
//   random   word 0 of Philox4x64-10 at counter (i, instance, 0, 2^62), key
//            (seed, 0).
// Equal keys order by circle index, so the order is strict and total and
// the rank of circle i is the number of circles before it: one workgroup
// per instance counts it against every other circle from LDS (n <= 1024:
// 1e6 comparisons, broadcast reads).
#include "pecc_device.hpp"
#include "pecc_launch.hpp"

namespace pecc {
namespace {

constexpr int kPartBlock = 256;

__device__ __forceinline__ int angle_class(float x, float y)
{
    if (y < 0.f) return 0;
    if (y > 0.f) return 2;
    return x < 0.f ? 3 : 1;
}

// -1: a first, 1: b first, 0: equal keys
template <int KIND>
__device__ __forceinline__ int key_cmp(float2 a, float2 b, int ca, int cb, uint64_t ka,
                                       uint64_t kb)
{
#pragma clang fp contract(off)
    if constexpr (KIND == 0) {
        if (ca != cb) return ca < cb ? -1 : 1;
        if (ca == 1 || ca == 3) return 0;
        const double p = (double)a.x * (double)b.y;
        const double q = (double)a.y * (double)b.x;
        const double cross = p - q;
        return cross > 0.0 ? -1 : (cross < 0.0 ? 1 : 0);
    } else if constexpr (KIND == 1) {
        const double ra = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
        const double rb = (double)b.x * (double)b.x + (double)b.y * (double)b.y;
        return ra < rb ? -1 : (ra > rb ? 1 : 0);
    } else if constexpr (KIND == 2) {
        return a.x < b.x ? -1 : (a.x > b.x ? 1 : 0);
    } else {
        return ka < kb ? -1 : (ka > kb ? 1 : 0);
    }
}

template <int KIND>
__global__ __launch_bounds__(kPartBlock) void partition_kernel(
    const int32_t *__restrict__ offset, const float *__restrict__ xy, int64_t total_n, int k,
    uint64_t seed, int32_t *__restrict__ batch_of)
{
    __shared__ float2 pos[kMaxN];
    __shared__ uint64_t key[kMaxN];
    __shared__ uint8_t cls[kMaxN];
    const int b = blockIdx.x;
    const int off = offset[b], n = offset[b + 1] - off;
    if (!(off >= 0 && n >= 0 && n <= kMaxN && (int64_t)off + n <= total_n)) return;
    for (int i = threadIdx.x; i < n; i += kPartBlock) {
        const float2 p = reinterpret_cast<const float2 *>(xy)[off + i];
        pos[i] = p;
        cls[i] = (uint8_t)angle_class(p.x, p.y);
        if constexpr (KIND == 3)
            key[i] = philox4x64((uint64_t)(uint32_t)i, (uint64_t)(uint32_t)b, 0, 1ULL << 62, seed, 0)
                         .w[0];
    }
    __syncthreads();
    const int q = n / k, rem = n % k, big = rem * (q + 1);
    for (int i = threadIdx.x; i < n; i += kPartBlock) {
        const float2 pi = pos[i];
        const int ci = cls[i];
        const uint64_t ki = KIND == 3 ? key[i] : 0;
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const int c = key_cmp<KIND>(pos[j], pi, cls[j], ci, KIND == 3 ? key[j] : 0, ki);
            rank += (c < 0 || (c == 0 && j < i)) ? 1 : 0;
        }
        batch_of[off + i] = rank < big ? rank / (q + 1) : rem + (rank - big) / q;
    }
}

}  // namespace

hipError_t launch_partition(const int32_t *offset, const float *xy, int B, int64_t total_n,
                            int kind, int k, uint64_t seed, int32_t *batch_of, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    switch (kind) {
    case 0: partition_kernel<0><<<B, kPartBlock, 0, s>>>(offset, xy, total_n, k, seed, batch_of); break;
    case 1: partition_kernel<1><<<B, kPartBlock, 0, s>>>(offset, xy, total_n, k, seed, batch_of); break;
    case 2: partition_kernel<2><<<B, kPartBlock, 0, s>>>(offset, xy, total_n, k, seed, batch_of); break;
    default: partition_kernel<3><<<B, kPartBlock, 0, s>>>(offset, xy, total_n, k, seed, batch_of); break;
    }
    return hipGetLastError();
}

}  // namespace pecc
