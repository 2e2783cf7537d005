/*
 * CPU oracle for bulk direct-method stochastic simulation of CWC models.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference the GPU library is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library never does, and the two share no code, headers or tables.
 *
 * What it computes, for every trajectory g = instance*R + replica:
 *   the Gillespie direct method (paper Sec. 2.2: the waiting time is
 *   exponential with the total rate r; reduction e_i is chosen with
 *   probability r_i / r) over the flattened rule/context slots of a CWC
 *   model (paper Sec. 2.3, Fig. "simd": Match / Resolve / Update), with the
 *   propensity of a slot = k * prod binomial(n, m) (paper Sec. 2.2 worked
 *   example and the Match_Populations routine of Fig. "simd").
 *
 * The paper fixes the law but not the random stream or the floating-point
 * order, so this file also follows the project's arithmetic contract (the
 * same contract the GPU library implements on its own):
 *   - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the run
 *     seed, counter = (draw index lo, hi, trajectory lo, hi); one block
 *     per draw;
 *   - u_tau = (m(x0,x1)+1) 2^-53 in (0,1], u_sel = m(x2,x3) 2^-53 in
 *     [0,1), m(a,b) = (a << 21) | (b >> 11);
 *   - ssa_log: argument split u = 2^E f, atanh series, only correctly
 *     rounded + - * /, no fused multiply-add;
 *   - propensities summed in a perfect binary tree over the padded leaf
 *     array (node = left + right), rebuilt from scratch every event here;
 *   - selection: x = u_sel * a0, descend: left if x < L or R == 0, else
 *     x -= L and go right;
 *   - sample k (time k*dt) holds the state after every event at time <= k*dt.
 * Build with -ffp-contract=off and without -ffast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "ssa.h"

/* ---------------------------------------------------------------- Philox */

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {            /* key schedule: Weyl sequence */
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit integer from two 32-bit words. */
static uint64_t m53(uint32_t a, uint32_t b)
{
    return ((uint64_t)a << 21) | (uint64_t)(b >> 11);
}

static const double TWO_M53 = 1.0 / 9007199254740992.0;   /* 2^-53, exact */

double oracle_u_tau(uint32_t x0, uint32_t x1)
{
    return (double)(m53(x0, x1) + 1u) * TWO_M53;
}

double oracle_u_sel(uint32_t x2, uint32_t x3)
{
    return (double)m53(x2, x3) * TWO_M53;
}

/* ----------------------------------------------------------------- log */

/* Bit patterns of the constants (values derived with a 60-digit reference
 * by oracle/constants.py; the test suite re-derives and compares):
 *   SQRT2  = RN(sqrt 2)
 *   LN2_HI = ln 2 rounded to 32 significant bits (so E*LN2_HI is exact)
 *   LN2_LO = RN(ln 2 - LN2_HI)                                          */
static double from_bits(uint64_t b) { double d; memcpy(&d, &b, 8); return d; }
static uint64_t to_bits(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }

#define SQRT2_BITS  0x3FF6A09E667F3BCDull
#define LN2_HI_BITS 0x3FE62E42FF000000ull
#define LN2_LO_BITS 0xBDC718432A1B0E26ull

double oracle_ssa_log(double u)
{
    /* u in [2^-53, 1]: always a positive normal number. */
    uint64_t b = to_bits(u);
    int E = (int)((b >> 52) & 0x7FF) - 1023;
    double f = from_bits((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (f > from_bits(SQRT2_BITS)) {
        f = f * 0.5;
        E = E + 1;
    }
    double s = (f - 1.0) / (f + 1.0);
    double z = s * s;
    /* p(z) = sum_j z^j / (2j+3), j = 0..10, Horner from the top term. */
    double p = 1.0 / 23.0;
    for (int j = 9; j >= 0; --j) {
        double cj = 1.0 / (double)(2 * j + 3);
        p = p * z;
        p = p + cj;
    }
    /* ln f = 2 atanh(s) = 2s + 2 s z p */
    double t = z * p;
    t = s * t;
    double lnf = (2.0 * s) + (2.0 * t);
    double Ed = (double)E;
    double lo = Ed * from_bits(LN2_LO_BITS);
    lo = lo + lnf;
    double hi = Ed * from_bits(LN2_HI_BITS);
    return hi + lo;
}

/* ---------------------------------------------------------- propensity */

/* Number of distinct ways to pick m identical atoms out of n:
 * the binomial coefficient of the paper's Match_Populations routine. */
static uint64_t binom(int64_t n, int m)
{
    if (m == 0) return 1;
    if (n < m) return 0;
    if (m == 1) return (uint64_t)n;
    /* m == 2 */
    return (uint64_t)n * (uint64_t)(n - 1) / 2u;
}

static double leaf_propensity(const oracle_model *M, int leaf,
                              const int32_t *counts, const double *k)
{
    int r = M->leaf_rule[leaf];
    if (r < 0) return 0.0;                       /* padding leaf */
    uint64_t h = 1;
    for (int t = 0; t < 2; ++t) {
        int cell = M->leaf_react[leaf * 4 + 2 * t];
        int m = M->leaf_react[leaf * 4 + 2 * t + 1];
        if (m == 0) continue;
        h = h * binom(counts[cell], m);
    }
    return k[r] * (double)h;
}

/* Heap layout: node 1 is the root, node i has children 2i and 2i+1, the
 * P leaves sit at nodes P..2P-1. */
static void build_tree(const oracle_model *M, const int32_t *counts,
                       const double *k, double *node)
{
    int P = M->n_leaves;
    for (int i = 0; i < P; ++i)
        node[P + i] = leaf_propensity(M, i, counts, k);
    for (int i = P - 1; i >= 1; --i)
        node[i] = node[2 * i] + node[2 * i + 1];
}

static int descend(const oracle_model *M, const double *node, double x)
{
    int P = M->n_leaves;
    int i = 1;
    while (i < P) {
        double L = node[2 * i], R = node[2 * i + 1];
        if (x < L || R == 0.0) {
            i = 2 * i;
        } else {
            x = x - L;
            i = 2 * i + 1;
        }
    }
    return i - P;
}

/* Selection on an explicit leaf vector (exposed for the tests): builds the
 * tree over P leaves and descends with x. */
int oracle_select(const double *leaves, int P, double x, double *a0)
{
    double *node = (double *)malloc(sizeof(double) * (size_t)(2 * P));
    if (!node) return -1;
    for (int i = 0; i < P; ++i) node[P + i] = leaves[i];
    for (int i = P - 1; i >= 1; --i) node[i] = node[2 * i] + node[2 * i + 1];
    oracle_model M;
    memset(&M, 0, sizeof M);
    M.n_leaves = P;
    int j = descend(&M, node, x);
    if (a0) *a0 = node[1];
    free(node);
    return j;
}

/* ------------------------------------------------------------ simulate */

int oracle_simulate(const oracle_model *M, const oracle_run *run,
                    int64_t g0, int64_t g1, oracle_out *out)
{
    const int C = M->n_cells;
    const int K1 = run->n_samples;
    const int P = M->n_leaves;
    int32_t *counts = (int32_t *)malloc(sizeof(int32_t) * (size_t)C);
    double *node = (double *)malloc(sizeof(double) * (size_t)(2 * P));
    if (!counts || !node) { free(counts); free(node); return -1; }
    const uint32_t key[2] = {(uint32_t)run->seed, (uint32_t)(run->seed >> 32)};

    for (int64_t g = g0; g < g1; ++g) {
        int64_t inst = g / run->replicas;
        int64_t o = g - g0;
        const double *k = run->rate_table ? run->rate_table + inst * M->n_rules
                                          : M->rule_k;
        const int32_t *init = run->init_table ? run->init_table + inst * C
                                              : M->init_counts;
        memcpy(counts, init, sizeof(int32_t) * (size_t)C);
        double t = 0.0;
        int64_t e = 0;
        int k_next = 0;
        int status = ORACLE_OK;
        uint64_t digest = 0xcbf29ce484222325ull;     /* FNV-1a offset basis */

        for (;;) {
            build_tree(M, counts, k, node);
            double a0 = node[1];
            uint32_t ctr[4] = {(uint32_t)e, (uint32_t)((uint64_t)e >> 32),
                               (uint32_t)g, (uint32_t)((uint64_t)g >> 32)};
            uint32_t x[4];
            oracle_philox4x32_10(ctr, key, x);
            if (a0 == 0.0) {
                /* absorbing state: nothing can fire any more */
                while (k_next < K1) {
                    if (out->samples)
                        memcpy(out->samples + (o * K1 + k_next) * C, counts,
                               sizeof(int32_t) * (size_t)C);
                    oracle_accumulate(out, inst, k_next, counts, C, K1);
                    ++k_next;
                }
                status = ORACLE_ABSORBED;
                break;
            }
            double u_tau = oracle_u_tau(x[0], x[1]);
            double u_sel = oracle_u_sel(x[2], x[3]);
            double tau = (-oracle_ssa_log(u_tau)) / a0;
            double t_new = t + tau;
            /* right-continuous sampling: sample k is the state after all
             * events at times <= k*dt, i.e. before this event if
             * k*dt < t_new */
            while (k_next < K1 && (double)k_next * run->dt < t_new) {
                if (out->samples)
                    memcpy(out->samples + (o * K1 + k_next) * C, counts,
                           sizeof(int32_t) * (size_t)C);
                oracle_accumulate(out, inst, k_next, counts, C, K1);
                ++k_next;
            }
            if (k_next >= K1) break;                  /* horizon reached */
            double xs = u_sel * a0;
            int j = descend(M, node, xs);
            /* Update: apply the rule's net change at the chosen context */
            int overflow = 0;
            int nd = M->leaf_ndelta[j];
            for (int d = 0; d < nd; ++d) {
                int cell = M->leaf_delta[(j * ORACLE_MAX_DELTA + d) * 2];
                int dv = M->leaf_delta[(j * ORACLE_MAX_DELTA + d) * 2 + 1];
                int64_t v = (int64_t)counts[cell] + dv;
                if (v > (int64_t)run->count_cap) overflow = 1;
            }
            if (overflow) { status = ORACLE_OVERFLOW; break; }
            for (int d = 0; d < nd; ++d) {
                int cell = M->leaf_delta[(j * ORACLE_MAX_DELTA + d) * 2];
                int dv = M->leaf_delta[(j * ORACLE_MAX_DELTA + d) * 2 + 1];
                counts[cell] += dv;
            }
            t = t_new;
            e = e + 1;
            digest = (digest ^ (uint64_t)(uint32_t)j) * 0x100000001b3ull;
            if (run->max_events > 0 && e == run->max_events) {
                status = ORACLE_EVENT_CAP;
                break;
            }
        }
        if (out->final_counts)
            memcpy(out->final_counts + o * C, counts, sizeof(int32_t) * (size_t)C);
        if (out->events) out->events[o] = e;
        if (out->t_final) out->t_final[o] = t;
        if (out->digest) out->digest[o] = digest;
        if (out->status) out->status[o] = (uint8_t)status;
        if (out->n_recorded) out->n_recorded[o] = k_next;
    }
    free(counts);
    free(node);
    return 0;
}

/* Exact integer moments: n, S1 = sum x, S2 = sum x^2 (128-bit). */
void oracle_accumulate(oracle_out *out, int64_t inst, int k,
                       const int32_t *counts, int C, int K1)
{
    if (!out->n) return;
    out->n[inst * K1 + k] += 1;
    for (int c = 0; c < C; ++c) {
        size_t idx = ((size_t)inst * K1 + k) * C + c;
        uint64_t x = (uint64_t)counts[c];
        out->s1[idx] += x;
        unsigned __int128 s2 = ((unsigned __int128)out->s2_hi[idx] << 64) |
                               out->s2_lo[idx];
        s2 += (unsigned __int128)(x * x);
        out->s2_lo[idx] = (uint64_t)s2;
        out->s2_hi[idx] = (uint64_t)(s2 >> 64);
    }
}

void oracle_merge_moments(uint64_t *n_dst, uint64_t *s1_dst, uint64_t *lo_dst,
                          uint64_t *hi_dst, const uint64_t *n_src,
                          const uint64_t *s1_src, const uint64_t *lo_src,
                          const uint64_t *hi_src, int64_t n_rows, int C)
{
    for (int64_t r = 0; r < n_rows; ++r) {
        n_dst[r] += n_src[r];
        for (int c = 0; c < C; ++c) {
            size_t i = (size_t)r * C + c;
            s1_dst[i] += s1_src[i];
            unsigned __int128 a = ((unsigned __int128)hi_dst[i] << 64) | lo_dst[i];
            unsigned __int128 b = ((unsigned __int128)hi_src[i] << 64) | lo_src[i];
            a += b;
            lo_dst[i] = (uint64_t)a;
            hi_dst[i] = (uint64_t)(a >> 64);
        }
    }
}

/* mean = S1/n; var = (n S2 - S1^2) / (n (n-1)), numerator exact in 128 bits
 * then rounded once to double; NaN where fewer than 1 (mean) or 2 (var)
 * trajectories contributed.  Unbiased estimator (divisor n-1). */
void oracle_finalize(const uint64_t *n, const uint64_t *s1, const uint64_t *lo,
                     const uint64_t *hi, int64_t n_rows, int C,
                     double *mean, double *var)
{
    for (int64_t r = 0; r < n_rows; ++r) {
        uint64_t nn = n[r];
        for (int c = 0; c < C; ++c) {
            size_t i = (size_t)r * C + c;
            if (nn == 0) { mean[i] = NAN; var[i] = NAN; continue; }
            mean[i] = (double)s1[i] / (double)nn;
            if (nn < 2) { var[i] = NAN; continue; }
            unsigned __int128 S2 = ((unsigned __int128)hi[i] << 64) | lo[i];
            unsigned __int128 num = (unsigned __int128)nn * S2 -
                                    (unsigned __int128)s1[i] * s1[i];
            unsigned __int128 den = (unsigned __int128)nn * (nn - 1);
            var[i] = (double)num / (double)den;
        }
    }
}
