// L-BFGS building blocks shared by the descent kernels: the slot layout of
// the fused reduction, DPP wave reductions, the wave reduce-scatter, the
// Gram-matrix update rule, the pair terms and the pre-tested neighbor
// predicate.  gfx950 (wave64) only.
#pragma once
#include "pecc_device.hpp"

namespace pecc {

constexpr int kMM = 10;                   // history slots (max m)
constexpr int kNB = 2 * kMM + 1;          // basis size: s_0..s_9, y_0..y_9, g
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

// Layout-identical mirror of pecc_descent_result, and its first 40 bytes.
struct DescentResultDev {
    int32_t status, iters, evals, rebuilds;
    int64_t pair_evals;
    float E32, gnorm;
    double E64;
    int32_t cell_evals, reserved;
};
struct DescentHead {
    int32_t status, iters, evals, rebuilds;
    int64_t pair_evals;
    float E32, gnorm;
    double E64;
};

// Writes the result of instance b: the head as one struct, then cell_evals
// and the reserved word.  (Kernels build the 40-byte head: a 48-byte local
// struct changes the descent kernel's register allocation -- spills, and in
// one instantiation a misaligned register pair the compiler rejects.)
__device__ __forceinline__ void store_result(DescentResultDev *out, int b, const DescentHead &r,
                                             int cell_evals)
{
    char *o = reinterpret_cast<char *>(out) + (size_t)b * sizeof(DescentResultDev);
    *reinterpret_cast<DescentHead *>(o) = r;
    *reinterpret_cast<int2 *>(o + sizeof(DescentHead)) = make_int2(cell_evals, 0);
}

// The result of an instance that is not descended (status BAD_INSTANCE,
// energies NaN, E64 = -1).  The constants pass through an empty asm so the
// compiler materialises them here, on this rare path, instead of keeping
// them in registers across the whole descent loop.
__device__ __forceinline__ void store_bad_instance(DescentResultDev *out, int b)
{
    float qnan = __builtin_nanf("");
    double m1 = -1.0;
    asm volatile("" : "+v"(qnan), "+v"(m1));
    DescentHead r = {};
    r.status = 7;
    r.E32 = qnan;
    r.gnorm = qnan;
    r.E64 = m1;
    store_result(out, b, r, 0);
}

// History elements: float2, or the same bits held as one 64-bit value (an
// aligned register pair, so that shifting the history moves pairs).
__device__ __forceinline__ float2 as_f2(float2 v) { return v; }
__device__ __forceinline__ float2 as_f2(double v) { return __builtin_bit_cast(float2, v); }

// Value of reduction slot v summed over this thread's circles (v is a
// constant after unrolling, so the branches fold away): one FMA chain over
// the circles' coordinates, started by a product.
template <int CPT, typename HV>
__device__ __forceinline__ float slot_value(int v, const float2 (&gt)[CPT], const float2 (&sc)[CPT],
                                            const float2 (&yc)[CPT],
                                            const HV (&S)[kMM][CPT],
                                            const HV (&Y)[kMM][CPT], float e, float e1)
{
    if (v == sE) return e;
    if (v == sE1) return e1;
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        float2 a, b;
        if (v < kMM) { a = gt[c]; b = as_f2(S[v][c]); }
        else if (v < 2 * kMM) { a = gt[c]; b = as_f2(Y[v - kMM][c]); }
        else if (v < 3 * kMM - 1) { a = sc[c]; b = as_f2(S[v - 2 * kMM + 1][c]); }
        else if (v < 4 * kMM - 2) { a = sc[c]; b = as_f2(Y[v - (3 * kMM - 1) + 1][c]); }
        else if (v < 5 * kMM - 3) { a = yc[c]; b = as_f2(S[v - (4 * kMM - 2) + 1][c]); }
        else if (v < 6 * kMM - 4) { a = yc[c]; b = as_f2(Y[v - (5 * kMM - 3) + 1][c]); }
        else if (v == sGG) { a = gt[c]; b = gt[c]; }
        else if (v == sScSc) { a = sc[c]; b = sc[c]; }
        else if (v == sScYc) { a = sc[c]; b = yc[c]; }
        else if (v == sYcYc) { a = yc[c]; b = yc[c]; }
        else if (v == sScG) { a = sc[c]; b = gt[c]; }
        else { a = yc[c]; b = gt[c]; }   // sYcG
        acc = c == 0 ? a.x * b.x : fmaf(a.x, b.x, acc);
        acc = fmaf(a.y, b.y, acc);
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

__device__ __forceinline__ double lane_value64(double v, int l)
{
    const long long bits = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
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

// Maximum of a non-negative int over the 64 lanes, returned wave-uniform
// (lanes a DPP pattern leaves out read 0, which no value is below).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dppi(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ int wave_max_dpp(int v)
{
    v = max(v, dppi<kDppXor1>(v));
    v = max(v, dppi<kDppXor2>(v));
    v = max(v, dppi<kDppHalfMirror>(v));
    v = max(v, dppi<kDppRowMirror>(v));
    v = max(v, dppi<kDppBcast15, 0xa>(v));
    v = max(v, dppi<kDppBcast31, 0xc>(v));
    return __builtin_amdgcn_readlane(v, 63);
}

// Sum of an int over the 64 lanes (exact), returned wave-uniform.
__device__ __forceinline__ int wave_sum_int(int v)
{
    v += dppi<kDppXor1>(v);
    v += dppi<kDppXor2>(v);
    v += dppi<kDppHalfMirror>(v);
    v += dppi<kDppRowMirror>(v);
    v += dppi<kDppBcast15, 0xa>(v);
    v += dppi<kDppBcast31, 0xc>(v);
    return __builtin_amdgcn_readlane(v, 63);
}

// The same sum for a double: each DPP step moves the two 32-bit halves.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp64(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp64<kDppXor1>(v);
    v += dpp64<kDppXor2>(v);
    v += dpp64<kDppHalfMirror>(v);
    v += dpp64<kDppRowMirror>(v);
    v += dpp64<kDppBcast15, 0xa>(v);
    v += dpp64<kDppBcast31, 0xc>(v);
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Slot held by lane L after wave_reduce_scatter: slot L.
__device__ __forceinline__ int lane_slot(int L) { return L; }

// Half swaps between two registers (gfx950 VALU permutes).  swap32: a keeps
// its lanes 0-31 and receives b's lanes 0-31 in lanes 32-63; b receives a's
// lanes 32-63 in lanes 0-31 and keeps its lanes 32-63.  swap16: the same on
// 16-lane rows (a keeps rows 0, 2 and receives b's rows 0, 2 in rows 1, 3; b
// receives a's rows 1, 3 and keeps its rows 1, 3).  Written as asm because
// the builtins return one register twice in this compiler; the two wait
// states cover a VALU write of either operand just before.
__device__ __forceinline__ void swap32(float &a, float &b)
{
    asm("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}
__device__ __forceinline__ void swap16(float &a, float &b)
{
    asm("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}

// Reduce-scatter of the 64 slot values over the wave: afterwards lane L
// holds the wave sum of slot L.  Each stage halves the values per lane by
// pairing slots that differ in one bit with lanes that differ in the same
// bit: bit 5 and bit 4 by half swaps (slot q and q + 32 swapped between the
// wave halves, then added: one swap and one add per pair), bits 3, 2, 1, 0
// by DPP inside 16-lane rows (row mirror, half mirror, xor 2, xor 1; the lane
// whose bit is set keeps the upper slot).  Slots are produced in groups of
// eight (u + 8k, k = 0..7) that the first three stages consume, so only a
// few values are live at once.
template <int CPT, typename HV>
__device__ __forceinline__ float wave_reduce_scatter(const float2 (&gt)[CPT],
                                                     const float2 (&sc)[CPT],
                                                     const float2 (&yc)[CPT],
                                                     const HV (&S)[kMM][CPT],
                                                     const HV (&Y)[kMM][CPT], float e,
                                                     float e1)
{
    const int lane = threadIdx.x & (kWave - 1);
    const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0, b1 = (lane & 2) != 0;
    const bool b0 = (lane & 1) != 0;
    float h[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        float w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float lo = slot_value(u + 8 * k, gt, sc, yc, S, Y, e, e1);
            float hi = slot_value(u + 8 * k + 32, gt, sc, yc, S, Y, e, e1);
            swap32(lo, hi);
            w[k] = lo + hi;            // lanes 0-31: slot u + 8k, lanes 32-63: + 32
        }
        float v[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            float lo = w[k], hi = w[k + 2];
            swap16(lo, hi);
            v[k] = lo + hi;            // rows 0, 2: slot of w[k]; rows 1, 3: + 16
        }
        h[u] = (b3 ? v[1] : v[0]) + dpp<kDppRowMirror>(b3 ? v[0] : v[1]);
        // keep the streaming order: the next group is not hoisted above here
        __builtin_amdgcn_sched_barrier(0);
    }
    float t4[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) t4[v] = (b2 ? h[v + 4] : h[v]) + dpp<kDppHalfMirror>(b2 ? h[v] : h[v + 4]);
    float t2[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) t2[v] = (b1 ? t4[v + 2] : t4[v]) + dpp<kDppXor2>(b1 ? t4[v] : t4[v + 2]);
    return (b0 ? t2[1] : t2[0]) + dpp<kDppXor1>(b0 ? t2[0] : t2[1]);
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

// Whole-instance descent with B as a ring: the slots that lane l (basis
// vector l in pair order of the UPDATED basis: s_0..s_9, y_0..y_9, g)
// takes its new Gram entries from, as byte addresses for ds_bpermute
// packed in one word: bits 0-7 <g, b_l> without a push, 8-15 <g, b_l>
// with a push, 16-23 <s, b_l> and 24-31 <y, b_l> of the pushed pair.  A
// push renumbers old pair j + 1 as pair j; the new pair is pair 9.
__device__ __forceinline__ uint32_t gram_perm_bytes(int l)
{
    const bool is_g = l >= kG, is_s = l < kMM;
    const int j = is_s ? l : (is_g ? 0 : l - kMM);
    auto slot = [&](int kind, bool push) -> int {   // kind 3: g, 1: s, 2: y
        const bool newp = push && j == kMM - 1;
        const int jo = push ? j + 1 : j;
        if (is_g) return kind == 3 ? sGG : kind == 1 ? sScG : sYcG;
        if (newp) {
            if (kind == 3) return is_s ? sScG : sYcG;
            if (kind == 1) return is_s ? sScSc : sScYc;
            return is_s ? sScYc : sYcYc;
        }
        if (kind == 3) return is_s ? sGS(jo) : sGY(jo);
        if (kind == 1) return is_s ? sSS(jo) : sSY(jo);
        return is_s ? sYS(jo) : sYY(jo);
    };
    return (uint32_t)(4 * slot(3, false)) | ((uint32_t)(4 * slot(3, true)) << 8) |
           ((uint32_t)(4 * slot(1, true)) << 16) | ((uint32_t)(4 * slot(2, true)) << 24);
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

// sqrt(m2) in FP64 from FP32 estimates l32 ~ sqrt(m2) and il ~ 1/sqrt(m2)
// (both 0 when m2 is 0): two Newton steps l <- l + (m2 - l^2) * il / 2, the
// residual formed with one rounding.  With relative errors e of l32 and h
// of il, one step leaves about e^2 / 2 + e h (1e-14 from 1e-7) and the
// second one FP64 rounding: a square root without the FP64 reciprocal
// square root, whose seed is no better than il.
__device__ __forceinline__ double sqrt64_from32(double m2, float l32, float il)
{
    const double h = (double)(0.5f * il);
    double l = (double)l32;
    l = fma(fma(-l, l, m2), h, l);
    l = fma(fma(-l, l, m2), h, l);
    return l;
}

// The list sweep's FP32 pair term of circle i (at q) with circle j (at pj),
// as pair_term32 but with the gradient term divided by -2: gx, gy receive
// (d / l) (c_i - c_j), and the caller multiplies the sum by -2 -- a scaling
// by a power of two, exact, so the result has pair_term32's bits.  Returns
// the FP32 1/l (from max(l^2, FLT_MIN): coincident centres give d = 2 rad
// and a zero term without a test of their own) and l2, the seeds of
// pair_term64s.
__device__ __forceinline__ float pair_term32s(float2 q, float2 pj, bool count_e, float two_r,
                                              float four_r2, float four_r2_band, float &e,
                                              float &e1, float &gx, float &gy, float &l2o,
                                              bool want_e1 = true)
{
    (void)four_r2_band;
    const float dx = q.x - pj.x, dy = q.y - pj.y;
    const float l2 = dx * dx + dy * dy;
    const bool ov = l2 < four_r2;
    // + FLT_MIN: a finite inverse for coincident centres; a no-op (exact)
    // for any l2 above 2^-100
    const float il = __builtin_amdgcn_rsqf(l2 + 1.17549435e-38f);
    const float d = ov ? two_r - l2 * il : 0.f;
    const float dc = count_e ? d : 0.f;       // the overlap if this term counts the pair
    e = fmaf(dc, d, e);
    // the unit-circle energy (wave-uniform want_e1: only its caller's switch
    // into the FP64 regime reads it)
    if (want_e1) {
        const float d1 = fmaxf(dc - (two_r - 2.f), 0.f);
        e1 = fmaf(d1, d1, e1);
    }
    const float kf = d * il;
    gx += kf * dx;
    gy += kf * dy;
    l2o = l2;
    return il;
}

// pair_term64 with the square root from the FP32 seeds (l32 = l2 * il).
__device__ __forceinline__ void pair_term64s(float2 q, float2 pj, float l32, float il,
                                             double two_r64, double four_r2_64, double &eo,
                                             double &et)
{
    const double ex = (double)q.x - (double)pj.x, ey = (double)q.y - (double)pj.y;
    const double m2 = ex * ex + ey * ey;
    if (m2 < four_r2_64) {
        const double l = sqrt64_from32(m2, l32, il);
        const double d = two_r64 - l;
        const double dt = m2 < 4.0 ? 2.0 - l : 0.0;
        eo += d * d;
        et += dt * dt;
    }
}

}  // namespace pecc
