/* Drives the CPU oracle (oracle/ssa.c) through its whole interface on a
 * small model, for sanitizer builds (AddressSanitizer + UndefinedBehavior-
 * Sanitizer): Lotka-Volterra (X -> 2X, X + Y -> 2Y, Y -> 0; 4 leaves) and a
 * sweep of two rate rows, with every output buffer requested, then the
 * moment merge and finalisation, and the primitives at their edges.
 * Exit status 0 and no sanitizer report = pass. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/ssa.h"

int main(void)
{
    enum { C = 2, P = 4, NR = 3, I = 2, R = 8, K1 = 21 };
    const int32_t leaf_rule[P] = {0, 1, 2, -1};
    int32_t leaf_react[P * 4] = {0};
    int32_t leaf_delta[P * ORACLE_MAX_DELTA * 2] = {0};
    int32_t leaf_ndelta[P] = {0};
    leaf_react[0 * 4 + 0] = 0; leaf_react[0 * 4 + 1] = 1;                /* X     */
    leaf_react[1 * 4 + 0] = 0; leaf_react[1 * 4 + 1] = 1;                /* X + Y */
    leaf_react[1 * 4 + 2] = 1; leaf_react[1 * 4 + 3] = 1;
    leaf_react[2 * 4 + 0] = 1; leaf_react[2 * 4 + 1] = 1;                /* Y     */
    leaf_ndelta[0] = 1; leaf_delta[0 * 32 + 0] = 0; leaf_delta[0 * 32 + 1] = 1;
    leaf_ndelta[1] = 2; leaf_delta[1 * 32 + 0] = 0; leaf_delta[1 * 32 + 1] = -1;
    leaf_delta[1 * 32 + 2] = 1; leaf_delta[1 * 32 + 3] = 1;
    leaf_ndelta[2] = 1; leaf_delta[2 * 32 + 0] = 1; leaf_delta[2 * 32 + 1] = -1;
    const double k[NR] = {1.0, 0.005, 1.0};
    const int32_t init[C] = {300, 300};
    oracle_model M = {C, P, NR, leaf_rule, leaf_react, leaf_delta, leaf_ndelta, k, init};
    const double table[I * NR] = {1.0, 0.005, 1.0, 2.0, 0.01, 2.0};
    const int32_t init_table[I * C] = {300, 300, 0, 5};
    oracle_run run = {7, I, R, table, init_table, 0.25, K1, 2147483647, 0};
    const int G = I * R;
    oracle_out o;
    memset(&o, 0, sizeof o);
    o.samples = calloc((size_t)G * K1 * C, 4);
    o.final_counts = calloc((size_t)G * C, 4);
    o.events = calloc(G, 8);
    o.t_final = calloc(G, 8);
    o.digest = calloc(G, 8);
    o.status = calloc(G, 1);
    o.n_recorded = calloc(G, 4);
    o.n = calloc((size_t)I * K1, 8);
    o.s1 = calloc((size_t)I * K1 * C, 8);
    o.s2_lo = calloc((size_t)I * K1 * C, 8);
    o.s2_hi = calloc((size_t)I * K1 * C, 8);
    if (oracle_simulate(&M, &run, 0, G, &o) != 0) return 2;
    /* a second pass over a sub-range with the caps active */
    oracle_run capped = run;
    capped.count_cap = 305;
    capped.max_events = 50;
    if (oracle_simulate(&M, &capped, 3, 11, &o) != 0) return 3;
    double *mean = calloc((size_t)I * K1 * C, 8), *var = calloc((size_t)I * K1 * C, 8);
    oracle_finalize(o.n, o.s1, o.s2_lo, o.s2_hi, (int64_t)I * K1, C, mean, var);
    uint64_t *n2 = calloc((size_t)I * K1, 8), *s12 = calloc((size_t)I * K1 * C, 8);
    uint64_t *lo2 = calloc((size_t)I * K1 * C, 8), *hi2 = calloc((size_t)I * K1 * C, 8);
    oracle_merge_moments(n2, s12, lo2, hi2, o.n, o.s1, o.s2_lo, o.s2_hi, (int64_t)I * K1, C);
    /* primitives at their edges */
    const uint32_t ctr[4] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu};
    const uint32_t key[2] = {0xffffffffu, 0xffffffffu};
    uint32_t x[4];
    oracle_philox4x32_10(ctr, key, x);
    volatile double acc = oracle_ssa_log(1.0) + oracle_ssa_log(0x1p-53) +
                          oracle_u_tau(0u, 0u) + oracle_u_tau(~0u, ~0u) +
                          oracle_u_sel(0u, 0u) + oracle_u_sel(~0u, ~0u);
    const double leaves[8] = {0.0, 1.0, 0.0, 0.0, 2.0, 0.0, 0.0, 3.0};
    double a0 = 0.0;
    int j = oracle_select(leaves, 8, 0.0, &a0) + oracle_select(leaves, 8, 5.999, &a0) +
            oracle_select(leaves, 8, 6.0, &a0);
    (void)acc;
    printf("ok %d %lld %d\n", j, (long long)o.events[0], (int)o.status[5]);
    free(o.samples); free(o.final_counts); free(o.events); free(o.t_final); free(o.digest);
    free(o.status); free(o.n_recorded); free(o.n); free(o.s1); free(o.s2_lo); free(o.s2_hi);
    free(mean); free(var); free(n2); free(s12); free(lo2); free(hi2);
    return 0;
}
