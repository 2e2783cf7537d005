/*
 * CPU oracle for general CWC models (compartment creation, dissolution and
 * deletion; patterns two levels deep).  TEST INFRASTRUCTURE ONLY: loaded by
 * the test suite, the smoke check and the benchmark's CPU-baseline leg.
 */
#ifndef CWC_ORACLE_GCWC_H
#define CWC_ORACLE_GCWC_H
#include <stdint.h>

#include "ssa.h"

#define GORACLE_MAX_COMP 64
#define GORACLE_MAX_SPECIES 32

enum { GORACLE_NONE = 0, GORACLE_CREATE = 1, GORACLE_DISSOLVE = 2, GORACLE_DELETE = 3 };

typedef struct {
    int32_t n_species, n_labels, max_comp;
    const int32_t *has_wrap;                    /* [n_labels] */
    int32_t n_init;                             /* initial compartments, [0] = top */
    const int32_t *init_label, *init_parent;    /* [n_init] (parent of top = -1) */
    const int32_t *init_wrap, *init_content;    /* [n_init][NS] */
    int32_t n_rules;
    const int32_t *rule_depth;                  /* [R] 0, 1 or 2 */
    const int32_t *rule_labels;                 /* [R][3] context, child, grandchild */
    const int32_t *rule_lhs, *rule_rhs;         /* [R][5][NS]: regions context content,
                                                   child wrap, child content,
                                                   grandchild wrap, grandchild content */
    const int32_t *rule_action, *rule_level;    /* [R] GORACLE_*, level it acts on */
    const int32_t *rule_new_label;              /* [R] create */
    const int32_t *rule_new_wrap, *rule_new_content;  /* [R][NS] create */
    const int32_t *rule_release_wrap;           /* [R] dissolve */
    const double *rule_k;                       /* [R] */
} goracle_model;

int goracle_layout(const goracle_model *M, int *PL, int *Np, int32_t *rule_at);
int goracle_n_obs(const goracle_model *M);
/* out: samples / final_counts hold the observables; final_term (may be
 * NULL): [g][max_comp][3 + 2 NS] alive, label, parent, wrap, content. */
int goracle_simulate(const goracle_model *M, const oracle_run *run, int64_t g0, int64_t g1,
                     oracle_out *out, int32_t *final_term);
#endif
