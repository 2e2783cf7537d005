/*
 * CPU oracle interface.  TEST INFRASTRUCTURE ONLY: loaded by the test suite,
 * the smoke check and the benchmark's CPU-baseline leg, never by the GPU
 * library.  The flattened model tables are produced by oracle/cwc.py.
 */
#ifndef CWC_ORACLE_SSA_H
#define CWC_ORACLE_SSA_H
#include <stdint.h>

#define ORACLE_MAX_DELTA 16

enum { ORACLE_OK = 0, ORACLE_ABSORBED = 1, ORACLE_OVERFLOW = 2,
       ORACLE_EVENT_CAP = 3 };

typedef struct {
    int32_t n_cells;          /* C */
    int32_t n_leaves;         /* P, a power of two */
    int32_t n_rules;
    const int32_t *leaf_rule;   /* [P] rule index, -1 = padding leaf */
    const int32_t *leaf_react;  /* [P][2][2] (cell, multiplicity); m = 0 unused */
    const int32_t *leaf_delta;  /* [P][ORACLE_MAX_DELTA][2] (cell, net change) */
    const int32_t *leaf_ndelta; /* [P] */
    const double *rule_k;       /* [n_rules] model kinetic constants */
    const int32_t *init_counts; /* [C] model initial multiplicities */
} oracle_model;

typedef struct {
    uint64_t seed;
    int64_t n_instances;
    int64_t replicas;
    const double *rate_table;   /* [I][n_rules] or NULL */
    const int32_t *init_table;  /* [I][C] or NULL */
    double dt;
    int32_t n_samples;          /* K + 1 */
    int32_t count_cap;
    int64_t max_events;         /* 0 = none */
} oracle_run;

typedef struct {              /* every pointer may be NULL; rows indexed g-g0 */
    int32_t *samples;         /* [g][K+1][C] */
    int32_t *final_counts;    /* [g][C] */
    int64_t *events;
    double *t_final;
    uint64_t *digest;
    uint8_t *status;
    int32_t *n_recorded;
    uint64_t *n;              /* [I][K+1]        */
    uint64_t *s1;             /* [I][K+1][C]     */
    uint64_t *s2_lo, *s2_hi;  /* [I][K+1][C]     */
} oracle_out;

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]);
double oracle_u_tau(uint32_t x0, uint32_t x1);
double oracle_u_sel(uint32_t x2, uint32_t x3);
double oracle_ssa_log(double u);
int oracle_select(const double *leaves, int P, double x, double *a0);
int oracle_simulate(const oracle_model *M, const oracle_run *run,
                    int64_t g0, int64_t g1, oracle_out *out);
void oracle_accumulate(oracle_out *out, int64_t inst, int k,
                       const int32_t *counts, int C, int K1);
void oracle_merge_moments(uint64_t *n_dst, uint64_t *s1_dst, uint64_t *lo_dst,
                          uint64_t *hi_dst, const uint64_t *n_src,
                          const uint64_t *s1_src, const uint64_t *lo_src,
                          const uint64_t *hi_src, int64_t n_rows, int C);
void oracle_finalize(const uint64_t *n, const uint64_t *s1, const uint64_t *lo,
                     const uint64_t *hi, int64_t n_rows, int C,
                     double *mean, double *var);
#endif
