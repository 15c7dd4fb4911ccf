/*
 * pecc_oracle_sed.c -- plain CPU oracle for the solution-space exploring and
 * descent heuristic SED (Sec. 5, Alg. 5) at a fixed container radius.
 *
 * TEST INFRASTRUCTURE ONLY, like the other oracle files: only the test
 * suite, the smoke entry point and the CPU-baseline leg of the benchmark
 * load it; it shares no code with the GPU path.  Build with -O2
 * -ffp-contract=off.
 *
 * Random numbers: both sides draw them from one counter-based generator,
 * Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011), written here from its published definition.
 *   perturbation of chain b, SED iteration i, candidate j: coordinate k of
 *     x (k < 2n) takes word k mod 4 of the block at counter
 *     (k / 4, j, i, b), key (seed, 0); u = (word >> 40) 2^-24 (FP32, exact),
 *     r = u * 1.6 - 0.8 in FP32 (two roundings), x'_k = x_k + r;
 *   selection uniform of chain b, iteration i: word 0 of the block at
 *     counter (2^63, 0, i, b), u = (word >> 11) 2^-53 (FP64, exact).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "pecc_oracle_types.h"

typedef unsigned __int128 u128;

/* Philox4x64 with 10 rounds: two 64x64->128 multiplies per round, the key
 * bumped by the two Weyl constants between rounds. */
void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        const u128 p0 = (u128)M0 * c0, p1 = (u128)M1 * c2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Shift of every coordinate (Alg. 5 perturbation): r_k in [-0.8, 0.8). */
void oracle_sed_shift(int n, uint64_t seed, int32_t chain, int32_t iter, int32_t cand, float *r)
{
    const uint64_t key[2] = { seed, 0 };
    uint64_t w[4];
    for (int k = 0; k < 2 * n; ++k) {
        if ((k & 3) == 0) {
            const uint64_t ctr[4] = { (uint64_t)(k >> 2), (uint64_t)(uint32_t)cand,
                                      (uint64_t)(uint32_t)iter, (uint64_t)(uint32_t)chain };
            oracle_philox4x64(ctr, key, w);
        }
        const float u = (float)(w[k & 3] >> 40) * 0x1p-24f;
        const float scaled = u * 1.6f;
        r[k] = scaled - 0.8f;
    }
}

/* The perturbed layout x + r in FP32, like the positions the GPU keeps. */
void oracle_sed_perturb(int n, const float *xy, uint64_t seed, int32_t chain, int32_t iter,
                        int32_t cand, float *out)
{
    oracle_sed_shift(n, seed, chain, iter, cand, out);
    for (int k = 0; k < 2 * n; ++k) out[k] = xy[k] + out[k];
}

double oracle_sed_uniform(uint64_t seed, int32_t chain, int32_t iter)
{
    const uint64_t key[2] = { seed, 0 };
    const uint64_t ctr[4] = { 1ULL << 63, 0, (uint64_t)(uint32_t)iter, (uint64_t)(uint32_t)chain };
    uint64_t w[4];
    oracle_philox4x64(ctr, key, w);
    return (double)(w[0] >> 11) * 0x1p-53;
}

/* J(x) = ceil(-log10 E(x)) (Sec. 5.2).  E <= 0 has no finite J: returned as
 * the cap `jmax`; every J is clipped to jmax. */
int oracle_sed_J(double E, int jmax)
{
    if (!(E > 0.0)) return jmax;
    const double j = ceil(-log10(E));
    return j > (double)jmax ? jmax : (int)j;
}

/* select(U) of Alg. 5: the lowest-energy candidate when it is below the
 * current energy (lowest index among equal energies), otherwise a candidate
 * drawn with probabilities softmax(J): the first k whose cumulative weight
 * exp(J_k - J_max) exceeds u times the total. */
int oracle_sed_select(int m, const double *E, double E_cur, double u, int jmax)
{
    if (m <= 0) return -1;
    int best = 0;
    for (int k = 1; k < m; ++k)
        if (E[k] < E[best]) best = k;
    if (E[best] < E_cur) return best;
    int J[64];
    int jm = -1000000;
    for (int k = 0; k < m && k < 64; ++k) {
        J[k] = oracle_sed_J(E[k], jmax);
        if (J[k] > jm) jm = J[k];
    }
    double tot = 0.0;
    for (int k = 0; k < m && k < 64; ++k) tot += exp((double)(J[k] - jm));
    const double target = u * tot;
    double cdf = 0.0;
    for (int k = 0; k < m && k < 64; ++k) {
        cdf += exp((double)(J[k] - jm));
        if (target < cdf) return k;
    }
    return (m < 64 ? m : 64) - 1;
}

/* ------------------------------------------------------------------------ */
/* SED (Alg. 5) at a fixed radius with FP64 descents (oracle_descend).       */
/* xy: the random start (2n doubles), replaced by the best layout found.     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t iterations;   /* SED iterations run                               */
    int32_t descents;     /* descents run, the first one included              */
    double E_best;        /* energy of the returned layout                     */
    double E_start;       /* energy after the first descent                    */
} oracle_sed_result;

int oracle_sed(int n, double *xy, double R, const oracle_params *P, int s_iter, int m_max,
               double e_stop, uint64_t seed, int32_t chain, oracle_sed_result *res)
{
    if (m_max < 1 || m_max > 64) return -2;
    const size_t sz = sizeof(double) * 2 * (size_t)(n > 0 ? n : 1);
    double *x = malloc(sz), *best = malloc(sz), *cand = malloc(sz * (size_t)m_max);
    float *r32 = malloc(sizeof(float) * 2 * (size_t)(n > 0 ? n : 1));
    double Ec[64];
    if (!x || !best || !cand || !r32) {
        free(x); free(best); free(cand); free(r32);
        return -1;
    }
    memcpy(x, xy, sz);
    oracle_result r;
    oracle_descend(n, x, R, P, &r, NULL);
    double E = r.E, E_best = r.E;
    memcpy(best, x, sz);
    res->descents = 1;
    res->E_start = E;
    int it = 0;
    for (; it < s_iter; ++it) {
        if (E_best <= e_stop) break;
        int m = oracle_sed_J(E, m_max);
        if (m < 1) m = 1;
        for (int j = 0; j < m; ++j) {
            double *cj = cand + (size_t)j * 2 * n;
            oracle_sed_shift(n, seed, chain, it, j, r32);
            for (int k = 0; k < 2 * n; ++k) cj[k] = x[k] + (double)r32[k];
            oracle_descend(n, cj, R, P, &r, NULL);
            Ec[j] = r.E;
            res->descents += 1;
        }
        const int k = oracle_sed_select(m, Ec, E, oracle_sed_uniform(seed, chain, it), m_max);
        memcpy(x, cand + (size_t)k * 2 * n, sz);
        E = Ec[k];
        if (E < E_best) {
            E_best = E;
            memcpy(best, x, sz);
        }
    }
    memcpy(xy, best, sz);
    res->iterations = it;
    res->E_best = E_best;
    free(x); free(best); free(cand); free(r32);
    return 0;
}
