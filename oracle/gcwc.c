/*
 * CPU oracle for general CWC models: compartments created, dissolved and
 * deleted at run time, patterns that reach two levels below the context.
 *
 * TEST INFRASTRUCTURE ONLY.  Loaded by the test suite, the smoke check and
 * the benchmark's CPU-baseline leg, never by the GPU library; the two share
 * no code.  Random numbers, uniforms, ssa_log, the tree and the descent
 * are those of ssa.c (same contract).
 *
 * The term (paper Sec. 2.1): a multiset of atoms and compartments
 * (wrap atoms | content)^label, nested.  It is held as a pool of max_comp
 * compartment slots; slot 0 is the top level and never goes away; every
 * other live slot has a parent slot.  A new compartment takes the lowest
 * free slot.
 *
 * A rule ell: P -> O (paper Sec. 2.1) is applied in the content of a
 * compartment of its context label; its pattern may name a child
 * compartment of a given label (its wrap atoms, its content atoms; the
 * rest of each is the pattern's variable x / X), and inside that child a
 * grandchild of a given label (depth 2).  A match is the tuple
 * (context, child, grandchild); its *anchor* is the deepest compartment the
 * pattern names, which determines the match (a compartment has one parent),
 * so every live slot holds one match per rule anchored at its label.  The
 * rate of a match is k times the product, over the pattern's atoms (a, m)
 * in each region, of binomial(n_a, m) (Sec. 2.2; Match_Populations of
 * Fig. "simd"); summing a rule over its matching compartments is the
 * paper's count_compartments factor (Fig. "simd", Match).
 *
 * Update ("delete P_sigma ... add O_sigma", Fig. "simd"): the net change of
 * atoms in each named region, then the rule's structural action:
 *   create   a new compartment (label, wrap atoms, content atoms) inside
 *            the context (level 0), the child (1) or the grandchild (2);
 *   dissolve the child (level 1) or grandchild (2): its content atoms, its
 *            wrap atoms if the rule releases them, and its compartments
 *            pass to its parent's content (O binds X outside the wrap);
 *   delete   the child or grandchild with everything inside it.
 * An event that would exceed the count cap, or create a compartment with
 * no free slot, is not applied and ends the trajectory (OVERFLOW).
 *
 * Leaf layout: slot-major; the block of slot s lists the rules anchored at
 * label(s) in ascending rule index, padded to PL = next power of two of
 * the longest such list; the slot count is padded to a power of two.  A
 * model without structural actions whose compartments of one label all
 * have parents of one label has exactly the fixed-tree layout of ssa.c.
 *
 * Observables (samples, statistics, final state): per label, in label
 * order, the content atom totals over its live compartments, the wrap atom
 * totals (labels with a wrap), and the number of live compartments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "gcwc.h"
#include "ssa.h"

#define MAXC GORACLE_MAX_COMP
#define MAXS GORACLE_MAX_SPECIES

enum { REG_CTX = 0, REG_CW = 1, REG_CC = 2, REG_GW = 3, REG_GC = 4 };

typedef struct {
    uint8_t alive[MAXC];
    int32_t label[MAXC], parent[MAXC];
    int32_t wrap[MAXC][MAXS], content[MAXC][MAXS];
} pool_t;

static int next_pow2(int n)
{
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

static int anchor_label(const goracle_model *M, int r)
{
    return M->rule_labels[r * 3 + M->rule_depth[r]];
}

int goracle_layout(const goracle_model *M, int *PL, int *Np, int32_t *rule_at)
{
    /* rule_at: [n_labels][PL] rule index or -1 (caller sizes it n_labels*64) */
    int longest = 1;
    for (int l = 0; l < M->n_labels; ++l) {
        int n = 0;
        for (int r = 0; r < M->n_rules; ++r) n += anchor_label(M, r) == l;
        if (n > longest) longest = n;
    }
    *PL = next_pow2(longest);
    *Np = next_pow2(M->max_comp);
    if (rule_at) {
        for (int l = 0; l < M->n_labels; ++l) {
            int n = 0;
            for (int p = 0; p < *PL; ++p) rule_at[l * *PL + p] = -1;
            for (int r = 0; r < M->n_rules; ++r)
                if (anchor_label(M, r) == l) rule_at[l * *PL + n++] = r;
        }
    }
    return *Np * *PL;
}

int goracle_n_obs(const goracle_model *M)
{
    int n = 0;
    for (int l = 0; l < M->n_labels; ++l) n += M->n_species * (M->has_wrap[l] ? 2 : 1) + 1;
    return n;
}

static void observe(const goracle_model *M, const pool_t *T, int32_t *obs)
{
    const int NS = M->n_species;
    int o = 0;
    for (int l = 0; l < M->n_labels; ++l) {
        int64_t cont[MAXS] = {0}, wr[MAXS] = {0}, cnt = 0;
        for (int s = 0; s < M->max_comp; ++s) {
            if (!T->alive[s] || T->label[s] != l) continue;
            ++cnt;
            for (int a = 0; a < NS; ++a) {
                cont[a] += T->content[s][a];
                wr[a] += T->wrap[s][a];
            }
        }
        for (int a = 0; a < NS; ++a) obs[o++] = (int32_t)cont[a];
        if (M->has_wrap[l])
            for (int a = 0; a < NS; ++a) obs[o++] = (int32_t)wr[a];
        obs[o++] = (int32_t)cnt;
    }
}

static uint64_t binom(int64_t n, int m)
{
    if (m == 0) return 1;
    if (n < m) return 0;
    if (m == 1) return (uint64_t)n;
    return (uint64_t)n * (uint64_t)(n - 1) / 2u;     /* m == 2 */
}

/* The match of rule r anchored at slot s: (ctx, child, grandchild) slots,
 * or 0 if the compartments above s do not carry the pattern's labels. */
static int match_of(const goracle_model *M, const pool_t *T, int r, int s, int m[3])
{
    const int depth = M->rule_depth[r];
    const int32_t *lab = M->rule_labels + r * 3;
    m[0] = m[1] = m[2] = -1;
    int z = s;
    for (int lv = depth; lv >= 0; --lv) {
        if (z < 0 || !T->alive[z] || T->label[z] != lab[lv]) return 0;
        m[lv] = z;
        z = lv > 0 ? T->parent[z] : z;
    }
    return 1;
}

static int32_t *region(pool_t *T, const int m[3], int reg)
{
    switch (reg) {
    case REG_CTX: return T->content[m[0]];
    case REG_CW: return T->wrap[m[1]];
    case REG_CC: return T->content[m[1]];
    case REG_GW: return T->wrap[m[2]];
    default: return T->content[m[2]];
    }
}

static double leaf_rate(const goracle_model *M, const pool_t *T, int r, int s, const double *k)
{
    int m[3];
    if (!match_of(M, T, r, s, m)) return 0.0;
    const int NS = M->n_species;
    uint64_t h = 1;
    for (int reg = 0; reg <= 2 * M->rule_depth[r]; ++reg)
        for (int a = 0; a < NS; ++a) {
            const int mult = M->rule_lhs[(r * 5 + reg) * NS + a];
            if (mult) h *= binom(region((pool_t *)T, m, reg)[a], mult);
        }
    return k[r] * (double)h;
}

static void free_slot(pool_t *T, int z)
{
    T->alive[z] = 0;
    T->label[z] = -1;
    T->parent[z] = -1;
    memset(T->wrap[z], 0, sizeof T->wrap[z]);
    memset(T->content[z], 0, sizeof T->content[z]);
}

/* Applies rule r at match m to T; returns 0, or 1 if the result would
 * exceed the cap or needs a slot the pool does not have (T unchanged). */
static int apply(const goracle_model *M, pool_t *T, int r, const int m[3], int64_t cap)
{
    const int NS = M->n_species;
    pool_t U = *T;
    for (int reg = 0; reg <= 2 * M->rule_depth[r]; ++reg) {
        int32_t *v = region(&U, m, reg);
        for (int a = 0; a < NS; ++a)
            v[a] += M->rule_rhs[(r * 5 + reg) * NS + a] - M->rule_lhs[(r * 5 + reg) * NS + a];
    }
    const int act = M->rule_action[r], lv = M->rule_level[r];
    if (act == GORACLE_CREATE) {
        int z = -1;
        for (int s = 1; s < M->max_comp; ++s)
            if (!U.alive[s]) { z = s; break; }
        if (z < 0) return 1;
        U.alive[z] = 1;
        U.label[z] = M->rule_new_label[r];
        U.parent[z] = m[lv];
        for (int a = 0; a < NS; ++a) {
            U.wrap[z][a] = M->rule_new_wrap[r * NS + a];
            U.content[z][a] = M->rule_new_content[r * NS + a];
        }
    } else if (act == GORACLE_DISSOLVE) {
        const int z = m[lv], p = U.parent[z];
        for (int a = 0; a < NS; ++a) {
            U.content[p][a] += U.content[z][a];
            if (M->rule_release_wrap[r]) U.content[p][a] += U.wrap[z][a];
        }
        for (int s = 0; s < M->max_comp; ++s)
            if (U.alive[s] && U.parent[s] == z) U.parent[s] = p;
        free_slot(&U, z);
    } else if (act == GORACLE_DELETE) {
        uint8_t gone[MAXC] = {0};
        gone[m[lv]] = 1;
        for (int changed = 1; changed;) {      /* close under "parent is gone" */
            changed = 0;
            for (int s = 0; s < M->max_comp; ++s)
                if (U.alive[s] && !gone[s] && U.parent[s] >= 0 && gone[U.parent[s]]) {
                    gone[s] = 1;
                    changed = 1;
                }
        }
        for (int s = 0; s < M->max_comp; ++s)
            if (gone[s]) free_slot(&U, s);
    }
    /* counts compared as unsigned 32-bit values: a sum that wrapped past
     * 2^31 - 1 is above any cap as well */
    for (int s = 0; s < M->max_comp; ++s) {
        if (!U.alive[s]) continue;
        for (int a = 0; a < NS; ++a)
            if ((uint32_t)U.wrap[s][a] > (uint32_t)cap || (uint32_t)U.content[s][a] > (uint32_t)cap)
                return 1;
    }
    *T = U;
    return 0;
}

static void record(oracle_out *out, const goracle_model *M, const pool_t *T, int64_t o,
                   int64_t inst, int k, int K1, int C, int32_t *obs)
{
    observe(M, T, obs);
    if (out->samples) memcpy(out->samples + (o * K1 + k) * C, obs, sizeof(int32_t) * (size_t)C);
    oracle_accumulate(out, inst, k, obs, C, K1);
}

int goracle_simulate(const goracle_model *M, const oracle_run *run, int64_t g0, int64_t g1,
                     oracle_out *out, int32_t *final_term)
{
    if (M->max_comp < 1 || M->max_comp > MAXC || M->n_species > MAXS) return -1;
    const int NS = M->n_species, C = goracle_n_obs(M), K1 = run->n_samples;
    int PL, Np;
    int32_t *rule_at = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M->n_labels * 64 + 1));
    const int P = goracle_layout(M, &PL, &Np, rule_at);
    double *node = (double *)malloc(sizeof(double) * (size_t)(2 * P));
    int32_t *obs = (int32_t *)malloc(sizeof(int32_t) * (size_t)C);
    pool_t *T = (pool_t *)malloc(sizeof(pool_t));
    if (!rule_at || !node || !obs || !T) {
        free(rule_at); free(node); free(obs); free(T);
        return -1;
    }
    const uint32_t key[2] = {(uint32_t)run->seed, (uint32_t)(run->seed >> 32)};
    for (int64_t g = g0; g < g1; ++g) {
        const int64_t inst = g / run->replicas, o = g - g0;
        const double *k = run->rate_table ? run->rate_table + inst * M->n_rules : M->rule_k;
        memset(T, 0, sizeof *T);
        for (int s = 0; s < MAXC; ++s) { T->label[s] = -1; T->parent[s] = -1; }
        for (int i = 0; i < M->n_init; ++i) {
            T->alive[i] = 1;
            T->label[i] = M->init_label[i];
            T->parent[i] = M->init_parent[i];
            for (int a = 0; a < NS; ++a) {
                T->wrap[i][a] = M->init_wrap[i * NS + a];
                T->content[i][a] = M->init_content[i * NS + a];
            }
        }
        double t = 0.0;
        int64_t e = 0;
        int kn = 0, status = ORACLE_OK;
        uint64_t digest = 0xcbf29ce484222325ull;
        for (;;) {
            /* Match: every leaf, then the tree (node i = 2i + 2i+1) */
            for (int s = 0; s < Np; ++s)
                for (int p = 0; p < PL; ++p) {
                    double a = 0.0;
                    if (s < M->max_comp && T->alive[s]) {
                        const int r = rule_at[T->label[s] * PL + p];
                        if (r >= 0) a = leaf_rate(M, T, r, s, k);
                    }
                    node[P + s * PL + p] = a;
                }
            for (int i = P - 1; i >= 1; --i) node[i] = node[2 * i] + node[2 * i + 1];
            const double a0 = node[1];
            uint32_t ctr[4] = {(uint32_t)e, (uint32_t)((uint64_t)e >> 32), (uint32_t)g,
                               (uint32_t)((uint64_t)g >> 32)};
            uint32_t x[4];
            oracle_philox4x32_10(ctr, key, x);
            if (a0 == 0.0) {
                while (kn < K1) record(out, M, T, o, inst, kn++, K1, C, obs);
                status = ORACLE_ABSORBED;
                break;
            }
            const double tau = (-oracle_ssa_log(oracle_u_tau(x[0], x[1]))) / a0;
            const double t_new = t + tau;
            while (kn < K1 && (double)kn * run->dt < t_new) record(out, M, T, o, inst, kn++, K1, C, obs);
            if (kn >= K1) break;
            /* Resolve: descend the tree */
            double xs = oracle_u_sel(x[2], x[3]) * a0;
            int i = 1;
            while (i < P) {
                const double L = node[2 * i], R = node[2 * i + 1];
                if (xs < L || R == 0.0) {
                    i = 2 * i;
                } else {
                    xs = xs - L;
                    i = 2 * i + 1;
                }
            }
            const int j = i - P, s = j / PL, r = rule_at[T->label[s] * PL + j % PL];
            int m[3];
            match_of(M, T, r, s, m);
            /* Update */
            if (apply(M, T, r, m, (int64_t)run->count_cap)) {
                status = ORACLE_OVERFLOW;
                break;
            }
            t = t_new;
            e += 1;
            digest = (digest ^ (uint64_t)(uint32_t)j) * 0x100000001b3ull;
            if (run->max_events > 0 && e == run->max_events) {
                status = ORACLE_EVENT_CAP;
                break;
            }
        }
        observe(M, T, obs);
        if (out->final_counts) memcpy(out->final_counts + o * C, obs, sizeof(int32_t) * (size_t)C);
        if (out->events) out->events[o] = e;
        if (out->t_final) out->t_final[o] = t;
        if (out->digest) out->digest[o] = digest;
        if (out->status) out->status[o] = (uint8_t)status;
        if (out->n_recorded) out->n_recorded[o] = kn;
        if (final_term) {
            const int W = 3 + 2 * NS;
            int32_t *row = final_term + o * (int64_t)M->max_comp * W;
            for (int z = 0; z < M->max_comp; ++z) {
                row[z * W + 0] = T->alive[z];
                row[z * W + 1] = T->label[z];
                row[z * W + 2] = T->parent[z];
                for (int a = 0; a < NS; ++a) {
                    row[z * W + 3 + a] = T->wrap[z][a];
                    row[z * W + 3 + NS + a] = T->content[z][a];
                }
            }
        }
    }
    free(rule_at);
    free(node);
    free(obs);
    free(T);
    return 0;
}
