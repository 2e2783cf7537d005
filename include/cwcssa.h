/*
 * cwcssa -- bulk stochastic simulation of Calculus of Wrapped Compartments
 * (CWC) models on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only; no C++ exceptions cross it.  Every
 * call returns a cwc_status (CWC_OK = 0, errors < 0); the message of the
 * last error on the calling thread is available from cwc_last_error().
 *
 * What the library computes (Aldinucci et al., "On Designing Multicore-aware
 * Simulators for Biological Systems", PDP 2011):
 *   - the CWC term/rule model of Sec. 2.1 restricted to a fixed compartment
 *     tree: every compartment holds a content multiset and, if its label has
 *     one, a wrap multiset; rules rewrite the content of a compartment, or
 *     the content of a compartment together with the wrap and content of one
 *     of its children;
 *   - the stochastic semantics of Sec. 2.2: a rule's rate in a context is the
 *     kinetic constant times the number of distinct reactant combinations
 *     (product of binomial coefficients, the a a b b -> rate 4k example);
 *   - Gillespie's direct method (Sec. 2.2 two-step procedure; Sec. 2.3
 *     Match / Resolve / Update loop), run independently for every replica of
 *     every instance of a parameter sweep (Sec. 3.1.2, Sec. 5.2);
 *   - trajectories sampled at fixed simulation times and reduced across
 *     replicas into mean and variance per sample time, on line (Sec. 3,
 *     Fig. "simout"; Sec. 5.2 schema iii).
 *
 * Random stream and arithmetic (fixed so that results are reproducible
 * bit for bit, independent of batch size, execution form or tuning):
 *   - draw e of trajectory g: Philox4x32-10, key = (seed lo, seed hi),
 *     counter = (e lo, e hi, g lo, g hi); g = instance * R + replica;
 *   - u_tau = (m(x0,x1) + 1) 2^-53, u_sel = m(x2,x3) 2^-53 with
 *     m(a,b) = (a << 21) | (b >> 11);
 *   - tau = -ssa_log(u_tau) / a0 (ssa_log: exponent split plus an atanh
 *     series, correctly rounded + - * / only, no FMA contraction);
 *   - propensities in a perfect binary tree over the leaf array (slot blocks
 *     per compartment, each padded to a power of two, compartments padded to
 *     a power of two); node = left + right in binary64;
 *   - selection: x = u_sel * a0; at each node go left if x < L or R == 0,
 *     otherwise x -= L and go right;
 *   - sample k (time k*dt) holds the state after every event at time
 *     <= k*dt; the draw that crosses the last sample time is discarded.
 */
#ifndef CWCSSA_H
#define CWCSSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CWC_ABI_VERSION 2u

typedef int32_t cwc_status;
#define CWC_OK             0
#define CWC_E_INVALID     -1   /* malformed argument or model            */
#define CWC_E_UNSUPPORTED -2   /* outside the supported CWC fragment      */
#define CWC_E_NOMEM       -3   /* arena / device memory / budget too small */
#define CWC_E_DEVICE      -4   /* HIP runtime error                       */
#define CWC_E_NOTREADY    -5   /* results requested before completion     */
#define CWC_E_COMPILE     -6   /* kernel generation / compilation failed  */

/* Per-trajectory terminal status (data, not an error). */
#define CWC_REPLICA_OK        0   /* reached the last sample time            */
#define CWC_REPLICA_ABSORBED  1   /* total rate 0: remaining samples filled  */
#define CWC_REPLICA_OVERFLOW  2   /* an event would push a count above cap;
                                     the pre-event state is final, samples
                                     from then on are not contributed        */
#define CWC_REPLICA_EVENT_CAP 3   /* max_events applied; samples from then on
                                     are not contributed                     */

/* Pattern regions of a rule (Sec. 2.1: a rule is applied to the content of
 * a compartment of its label; a pattern may also name one child
 * compartment's wrap and content). */
#define CWC_REGION_PARENT 0   /* content of the compartment the rule runs in */
#define CWC_REGION_WRAP   1   /* wrap of the child compartment               */
#define CWC_REGION_CHILD  2   /* content of the child compartment            */

/* Execution forms. */
#define CWC_MODE_PLAIN      0  /* grid covers every trajectory, natural
                                  order                                     */
#define CWC_MODE_PERSISTENT 1  /* instances taken longest-first (Sec. 5.2
                                  schema ii), launch replayed from a HIP
                                  graph; a grid smaller than the run drains
                                  a work queue (idle lanes claim the next
                                  items), a grid that holds every
                                  trajectory runs without one, the
                                  hardware dispatcher starting blocks in
                                  that order as others finish             */

typedef struct cwc_ctx cwc_ctx;
typedef struct cwc_model cwc_model;
typedef struct cwc_run cwc_run;
typedef struct cwc_server cwc_server;
typedef struct cwc_stream cwc_stream;

/* --------------------------------------------------------------- basics */

/* Returns CWC_ABI_VERSION of the loaded library. */
uint32_t cwc_abi_version(void);

/* Message of the last failed call on this thread ("" if none).  Valid until
 * the next library call on the same thread. */
const char *cwc_last_error(void);

/* ------------------------------------------------------------- context */

/* Creates a context on HIP device `device` (the simulation engine of
 * Sec. 2.3, here one GPU running many instances at once, Sec. 3.1.2).
 *   arena, arena_bytes: optional caller-owned device buffer (e.g. a torch
 *     tensor's storage) from which all run buffers are sub-allocated; the
 *     library never frees it.  NULL/0: the library allocates device memory
 *     itself with hipMalloc.
 * Errors: CWC_E_INVALID (bad device), CWC_E_DEVICE. */
cwc_status cwc_ctx_create(int device, void *arena, size_t arena_bytes,
                          cwc_ctx **out);
void cwc_ctx_destroy(cwc_ctx *ctx);

/* --------------------------------------------------------------- model */

typedef struct {
    int32_t region;    /* CWC_REGION_*                         */
    int32_t species;   /* atom index, 0 <= species < n_species */
    int32_t mult;      /* multiplicity >= 1                    */
} cwc_term;

typedef struct {
    int32_t parent_type;   /* label l of "l: P -> O" (Sec. 2.1)            */
    int32_t child_type;    /* -1: content-only rule; else the child label  */
    int32_t n_lhs;         /* terms of the pattern P                       */
    const cwc_term *lhs;
    int32_t n_rhs;         /* terms of O                                   */
    const cwc_term *rhs;
    double k;              /* kinetic constant (Sec. 2.2), finite, > 0     */
} cwc_rule;

/* A CWC model with a fixed compartment tree.  Compartments are listed in
 * preorder; compartment 0 is the top level (parent -1) and every other
 * compartment's parent has a smaller index.  Count cells are ordered by
 * compartment; each compartment contributes n_species content cells, then
 * n_species wrap cells if its label has a wrap.
 * Supported fragment (else CWC_E_UNSUPPORTED): total reactant order <= 2
 * per rule (mass action up to bimolecular), no compartment creation or
 * dissolution, patterns of depth <= 1 (a rule reaches at most one child). */
typedef struct {
    int32_t n_species;
    int32_t n_types;
    int32_t n_comp;
    const int32_t *type_has_wrap;  /* [n_types] 0/1                        */
    const int32_t *comp_type;      /* [n_comp]                             */
    const int32_t *comp_parent;    /* [n_comp]                             */
    const int32_t *init_counts;    /* [n_cells] initial multiplicities     */
    int32_t n_rules;
    const cwc_rule *rules;         /* [n_rules]                            */
} cwc_model_desc;

typedef struct {
    int32_t n_cells;     /* C                                              */
    int32_t n_slots;     /* (rule, context) pairs                          */
    int32_t n_leaves;    /* P, power of two                                */
    int32_t p_local;     /* leaves per compartment block                   */
    int32_t n_rules;
    int32_t layout;      /* 0 = lane per replica, 1 = wave per replica     */
    double alg_slots_per_event;  /* algorithmic VALU issue slots of one
                                    applied event (roofline work unit):
                                    Philox4x32-10 (its key schedule, the
                                    same in every lane, is scalar work and
                                    not counted) + uniforms + log + time
                                    (195), selection (1 + 5 log2 P), update
                                    (2 per changed cell), re-evaluation of
                                    the slots whose reactants changed and of
                                    their tree paths, averaged over slots  */
} cwc_model_info;

/* Validates and flattens `d` into rule/context slots (Sec. 2.1: the terms
 * and rules of a model; Sec. 2.3: a rule is matched once per compartment of
 * its label, each match a propensity), generates the model's device code and compiles it for the context's device (compiled code is
 * cached on disk by content hash).  `d` is copied; the caller keeps it.
 * Errors: CWC_E_INVALID (bad indices, k <= 0 or not finite, negative
 * counts, non-preorder tree), CWC_E_UNSUPPORTED, CWC_E_COMPILE. */
cwc_status cwc_model_create(cwc_ctx *ctx, const cwc_model_desc *d,
                            cwc_model **out);
cwc_status cwc_model_get_info(const cwc_model *m, cwc_model_info *info);
/* Copies the generated device source (NUL-terminated) into buf if it fits;
 * *len receives the required size including the NUL. */
cwc_status cwc_model_source(const cwc_model *m, char *buf, size_t cap,
                            size_t *len);
void cwc_model_destroy(cwc_model *m);
/* Host-only: validates and flattens `d` and fills `info` (no device, no
 * compilation). */
cwc_status cwc_model_describe(const cwc_model_desc *d, cwc_model_info *info);
/* Host-only: flattens and validates `d` and returns the generated device
 * source (as cwc_model_source) without a device or a compilation. */
cwc_status cwc_codegen(const cwc_model_desc *d, char *buf, size_t cap,
                       size_t *len);

/* ------------------------------------------------------- general models */

/* General CWC terms (paper Sec. 2.1): compartments are created, dissolved
 * and deleted while a trajectory runs, and a rule's pattern may name a
 * child compartment of its context and a grandchild inside that child.
 * The term is held as a pool of max_comp compartment slots (one wavefront
 * lane each, so max_comp <= 64): the initial compartments take slots 0..n-1
 * in preorder (slot 0 the top level, which never goes away), a new
 * compartment the lowest free slot.  Each live slot anchors one match per
 * rule whose deepest named label is its label; the match's rate is k times
 * the product of binomial(n, m) over the pattern's atoms (total order <=
 * 2), and summing a rule over its matching compartments is the paper's
 * count_compartments (Fig. "simd", Match).  Leaves are slot-major, the
 * rules anchored at a label in ascending index, padded to a power of two;
 * slots padded to a power of two.  The outputs ("cells") are observables:
 * per label in label order, the content atom totals over its live
 * compartments, the wrap atom totals (labels with a wrap), the number of
 * live compartments.  An event that would exceed count_cap or needs a slot
 * the pool does not have is not applied: status OVERFLOW. */

#define CWC_ACT_NONE     0
#define CWC_ACT_CREATE   1   /* a compartment in the context (level 0), the
                                child (1) or the grandchild (2)           */
#define CWC_ACT_DISSOLVE 2   /* the child (1) or grandchild (2): its content
                                atoms and compartments (and its wrap atoms
                                with release_wrap) pass to its parent    */
#define CWC_ACT_DELETE   3   /* the child or grandchild with its content  */

typedef struct {
    int32_t label;
    int32_t parent;            /* index in the list (preorder); -1 for [0]  */
    const int32_t *wrap;       /* [n_species] or NULL (none)                */
    const int32_t *content;    /* [n_species] or NULL (none)                */
} cwc_gcomp;

typedef struct {
    int32_t context;           /* label of the compartment whose content the
                                  rule rewrites                              */
    int32_t child;             /* label of a child it names, or -1          */
    int32_t grandchild;        /* label of a compartment inside that child,
                                  or -1 (needs child)                        */
    int32_t n_lhs;
    const cwc_term *lhs;       /* region 0 context content, 1 child wrap,
                                  2 child content, 3 grandchild wrap,
                                  4 grandchild content                       */
    int32_t n_rhs;
    const cwc_term *rhs;       /* atoms the rule puts back (same regions)   */
    int32_t action;            /* CWC_ACT_*                                 */
    int32_t level;             /* see CWC_ACT_*                             */
    int32_t new_label;         /* create: the new compartment's label ...   */
    const int32_t *new_wrap;   /* ... its wrap [n_species] or NULL ...      */
    const int32_t *new_content;/* ... and content [n_species] or NULL       */
    int32_t release_wrap;      /* dissolve: wrap atoms join the parent      */
    double k;                  /* kinetic constant > 0                      */
} cwc_grule;

typedef struct {
    int32_t n_species;         /* 1..32                                     */
    int32_t n_labels;          /* 1..16                                     */
    const int32_t *has_wrap;   /* [n_labels]                                */
    int32_t max_comp;          /* 1..64 compartment slots                   */
    int32_t n_comp;            /* initial compartments, 1..max_comp         */
    const cwc_gcomp *comps;    /* [n_comp], preorder                        */
    int32_t n_rules;           /* 0..64                                     */
    const cwc_grule *rules;    /* [n_rules]                                 */
} cwc_gmodel_desc;

/* Validates `d` (copied), generates the general engine's model header and
 * compiles it for the context's device.  The model is used like any other
 * with cwc_run_submit (plain or persistent form, one wavefront per
 * trajectory; lanes_per_replica 0 or 64; rate tables allowed, init_table
 * must be NULL, the initial term is the model's; want_traj keeps the
 * observables [K+1][C][G]) and cwc_run_fetch_term, and in streamed runs
 * and the server (time-sliced, each trajectory's term checkpointed in
 * device memory between slices; cwc_stream_fetch_term,
 * cwc_server_fetch_term).  Errors: CWC_E_INVALID (indices,
 * rates, counts, regions beyond the pattern, non-preorder term),
 * CWC_E_UNSUPPORTED (max_comp > 64, order > 2), CWC_E_COMPILE. */
cwc_status cwc_gmodel_create(cwc_ctx *ctx, const cwc_gmodel_desc *d,
                             cwc_model **out);
/* Host-only: validates `d` and returns the generated model header plus the
 * engine source (as cwc_model_source), no device. */
cwc_status cwc_gcodegen(const cwc_gmodel_desc *d, char *buf, size_t cap,
                        size_t *len);

/* ----------------------------------------------------------------- run */

typedef struct {
    int32_t block_size;        /* threads per block, multiple of 64; 0 = auto */
    int32_t waves_per_simd;    /* persistent grid: requested waves per SIMD
                                  (1..16; 0 = 2).  More than fit wait for the
                                  hardware dispatcher; a grid that holds every
                                  trajectory runs without the queue, its items
                                  still claimed longest-first               */
    int32_t refill_chunk;      /* persistent, lane layout: 1 = each idle lane
                                  claims one item from the global queue;
                                  >= 64 = a wavefront claims this many
                                  consecutive items at once and its idle lanes
                                  take them first; 0 = auto (64); 2..63 are
                                  rejected with CWC_E_INVALID                 */
    int32_t lanes_per_replica; /* 1 (lane layout), 2 (pair: two lanes per
                                  trajectory, each holding half of the
                                  propensity tree; models with >= 2 leaves),
                                  4 (quad: four lanes, a quarter each; models
                                  with >= 4 leaves; run forms only, serving
                                  uses 1 or 2) or 64 (wave layout); 0 = auto.
                                  Other values, or a group of more lanes
                                  than the model has leaves:
                                  CWC_E_UNSUPPORTED                         */
    int32_t sample_slots;      /* lane layout: sampling-buffer depth, i.e. the
                                  accumulator rows each wavefront keeps in
                                  LDS before writing moments back; a power of
                                  two, at most 64; 0 = auto (16).  Results do
                                  not depend on it.                           */
} cwc_tuning;

typedef struct {
    uint64_t seed;
    int64_t n_instances;            /* I >= 1                                   */
    int64_t replicas_per_instance;  /* R >= 1; G = I * R trajectories           */
    const double *rate_table;       /* host [I][n_rules] or NULL (model k)      */
    const int32_t *init_table;      /* host [I][n_cells] or NULL (model init)   */
    double dt;                      /* sample spacing > 0                       */
    int32_t n_samples;              /* K + 1 >= 1 sample times k*dt             */
    int32_t mode;                   /* CWC_MODE_*                               */
    int32_t want_traj;              /* keep samples [K+1][C][G]                 */
    int32_t want_digest;            /* keep an FNV-1a digest of fired leaves    */
    int32_t count_cap;              /* > 0; typically INT32_MAX                 */
    int64_t max_events;             /* per trajectory; 0 = unlimited            */
    const cwc_tuning *tuning;       /* NULL = library choice                    */
} cwc_run_desc;

/* Enqueues a run on `hip_stream` (a hipStream_t; NULL = the null stream):
 * G = I x R independent simulations by the direct method (Sec. 2.2 and
 * 2.3), the replicas of one model or the instances of a parameter sweep
 * (Sec. 3.1.2), each sampled at t_k = k dt and reduced on line into
 * per-sample moments (Sec. 3, Sec. 5.2 schema iii).
 * Host tables are copied before return.  Buffers come from the context's
 * arena (CWC_E_NOMEM if it is too small) or from hipMalloc.
 * Errors: CWC_E_INVALID, CWC_E_NOMEM, CWC_E_DEVICE. */
cwc_status cwc_run_submit(cwc_ctx *ctx, const cwc_model *m,
                          const cwc_run_desc *d, void *hip_stream,
                          cwc_run **out);
/* Re-enqueues the same run (same inputs, same buffers; results are
 * overwritten with identical values, each trajectory's random stream being
 * fixed by (seed, trajectory, draw): Sec. 2.2's draws made reproducible).  In persistent mode the launch
 * sequence is replayed from a captured HIP graph.  On another stream the
 * relaunch first waits for the previous launch to end. */
cwc_status cwc_run_relaunch(cwc_run *r, void *hip_stream);
/* Completion of the launch sequence (Sec. 5.2: the instances' results
 * gathered once every instance has reached its end time): query sets
 * *done to 1 or 0 without blocking; wait blocks until the end.  Errors:
 * CWC_E_DEVICE if the launch failed. */
cwc_status cwc_run_query(cwc_run *r, int *done);
cwc_status cwc_run_wait(cwc_run *r);
/* Waits at most `timeout_s` seconds (a host-side watchdog): CWC_OK once
 * the launch has ended, CWC_E_NOTREADY if it is still running (it keeps
 * running; wait again or destroy the run after it ends), CWC_E_DEVICE if
 * it failed. */
cwc_status cwc_run_wait_for(cwc_run *r, double timeout_s);
/* Device time of the last launch of the simulation kernel (HIP events on
 * the run's stream), and of the whole launch sequence. */
cwc_status cwc_run_elapsed(cwc_run *r, float *sim_ms, float *total_ms);
/* Name of the simulation kernel the run dispatches (NUL-terminated) copied
 * into buf if it fits; *len receives the required size including the NUL.
 * The persistent form runs a "*_persistent_*" kernel when its grid drains
 * the queue and a "*_plain_*" kernel (items still in longest-first order)
 * when its grid already holds every trajectory.  Valid from submission on. */
cwc_status cwc_run_kernel_name(const cwc_run *r, char *buf, size_t cap, size_t *len);

/* On-line statistics (Sec. 3 and Fig. "simout": mean and variance of the
 * instances' states at each sample time; Sec. 5.2 schema iii).
 * Statistics per (instance, sample, cell): mean and unbiased variance
 * (NaN where fewer than 1 / 2 trajectories contributed) and the number of
 * contributing trajectories per (instance, sample).  Layout [I][K+1][C] and
 * [I][K+1].  Any pointer may be NULL.  dst_is_device: destinations are
 * device pointers.  CWC_E_NOTREADY before completion. */
cwc_status cwc_run_fetch_stats(cwc_run *r, double *mean, double *var,
                               int64_t *n, int dst_is_device);
/* The reduction's exact state (Sec. 5.2 schema iii, the partial sums the
 * statistics are computed from): S1 = sum x, S2 = sum x^2 split as
 * s2_hi32 * 2^32 + s2_lo32 (each an exact uint64 sum), layout [I][K+1][C]. */
cwc_status cwc_run_fetch_moments(cwc_run *r, uint64_t *s1, uint64_t *s2_hi32,
                                 uint64_t *s2_lo32, int64_t *n,
                                 int dst_is_device);
/* Sampled trajectories (paper Sec. 3: states at fixed simulation times,
 * the simulator's primary output beside the on-line statistics).  Layout
 * [K+1][C][G] int32, trajectory fastest: cell c of sample k of trajectory g
 * is dst[(k * C + c) * G + g] (the kernels write it in place, so lanes that
 * record the same sample write neighbouring words).  Requires want_traj;
 * entries of samples at or after a trajectory's n_recorded are unspecified.
 * dst is caller-owned, G * (K+1) * C int32, host or device memory
 * (dst_is_device).  Errors: CWC_E_NOTREADY before completion, CWC_E_INVALID
 * for a run submitted without want_traj. */
cwc_status cwc_run_fetch_trajectories(cwc_run *r, int32_t *dst,
                                      int dst_is_device);
/* General models: each trajectory's final term, [G][max_comp][3 + 2 NS]
 * int32 rows (alive 0/1, label or -1, parent slot or -1, wrap atoms [NS],
 * content atoms [NS]); free slots hold 0, -1, -1 and zeros.  CWC_E_INVALID
 * for a fixed-tree model. */
cwc_status cwc_run_fetch_term(cwc_run *r, int32_t *dst, int dst_is_device);
/* Per trajectory [G] (each instance's end state, Sec. 2.3: the loop ends
 * at the end time, when no rule applies, or at a cap): applied events,
 * terminal status, digest (0 unless want_digest), final simulation time,
 * number of recorded samples, final counts [G][C].  Any pointer may be
 * NULL; caller-owned destinations (dst_is_device as above).  Errors:
 * CWC_E_NOTREADY before completion. */
cwc_status cwc_run_fetch_counters(cwc_run *r, int64_t *events,
                                  uint8_t *status, uint64_t *digest,
                                  double *t_final, int32_t *n_recorded,
                                  int32_t *final_counts, int dst_is_device);
/* Releases the run's device buffers (arena regions or hipMalloc'd memory)
 * after waiting for its launch to end; NULL is ignored. */
void cwc_run_destroy(cwc_run *r);

/* ------------------------------------------------- run without allocation */

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * simulation as cwc_run_submit (same kernels, bit-identical results), but
 * the run's intermediate state -- exact moment accumulators, recorded-count
 * histogram, queue cursor -- lives in a device array of
 * CWC_NOALLOC_SCRATCH_BYTES that the library holds statically on every GPU
 * it runs on (until the process ends), and the call allocates and frees
 * nothing: it enqueues fill kernels, the simulation kernel and the two
 * finalisation kernels on `hip_stream` and returns.  Synchronise the stream
 * before reading the outputs.
 *   d: as cwc_run_submit, except that rate_table ([I][n_rules] f64) and
 *      init_table ([I][n_cells] i32) are DEVICE pointers (or NULL: the
 *      model's own), their values are not checked (kinetic constants must be
 *      finite and > 0, counts in [0, count_cap]), want_traj must be 0,
 *      instances run in natural order, and tuning NULL means the library's
 *      defaults (the stored autotuner table is not read).  The model's code
 *      for the requested layout must already be loaded (it is for the
 *      model's default layout; another layout is loaded by one
 *      cwc_run_submit in it).
 *   o: caller-owned device outputs, every pointer set: mean/var [I][K+1][C]
 *      f64, n [I][K+1] i64, per trajectory events i64, status u8, digest
 *      u64, t_final f64, n_recorded i32 [G], final_counts [G][C] i32.
 * The scratch array is shared by every call on one GPU: calls whose work
 * overlaps on the device (different streams or threads) race on it; calls
 * on one stream are ordered and safe.
 * Errors: CWC_E_INVALID (as cwc_run_submit, a missing output, want_traj, a
 * layout not loaded), CWC_E_NOMEM when 24 x I x (K+1) x C + 8 x I x (K+2)
 * bytes (each part rounded up to 256) plus 256 exceed the scratch array,
 * CWC_E_DEVICE. */
#define CWC_NOALLOC_SCRATCH_BYTES (32u << 20)

typedef struct {
    double *mean;
    double *var;
    int64_t *n;
    int64_t *events;
    uint8_t *status;
    uint64_t *digest;
    double *t_final;
    int32_t *n_recorded;
    int32_t *final_counts;
} cwc_run_outputs;

cwc_status cwc_run_into(cwc_ctx *ctx, const cwc_model *m, const cwc_run_desc *d,
                        const cwc_run_outputs *o, void *hip_stream);

/* -------------------------------------------------------- streamed runs */

/* Bounded-memory execution of a run in windows of sample points (paper
 * Sec. 5.2: schema ii time-slices instances at constant simulation time,
 * stopping and restarting them under a scheduler with predictive
 * heuristics from their history; schema iii reduces a running window of
 * all trajectories on line while later parts are produced, so the reduced
 * part leaves memory).  The K+1 sample points are cut into windows of
 * `window` points; each window is one time-sliced launch that advances
 * every unfinished trajectory to just before the window's end and suspends
 * it to a device checkpoint; the window's rows of exact moments are then
 * finalised and handed out while the next window already runs.  Device
 * memory is O(G C + I window C), independent of K.  Wavefronts are
 * dispatched heaviest first: by total propensity at t = 0 for the first
 * window, then by the events their trajectories applied in the previous
 * window.  Every trajectory, statistic and counter equals that of
 * cwc_run_submit on the same descriptor bit for bit. */

/* d: as cwc_run_submit, except want_traj must be 0 (statistics only), mode
 * is ignored and tuning is read only for lanes_per_replica (0 = two lanes
 * per trajectory where the model has two leaves, else one; 1, 2, or 64 for
 * one wavefront per trajectory).  window >= 1 sample points (clamped to
 * K+1).  Host tables are copied.  The first window is enqueued on
 * hip_stream before return.  Errors: as cwc_run_submit; CWC_E_UNSUPPORTED
 * for want_traj or another lanes_per_replica. */
cwc_status cwc_stream_open(cwc_ctx *ctx, const cwc_model *m,
                           const cwc_run_desc *d, int32_t window,
                           void *hip_stream, cwc_stream **out);
/* Waits for the next window, returns its first sample index in *k0 and its
 * number of sample points in *rows (0 once every window has been
 * returned), and copies its statistics: mean and var [I][rows][C] f64
 * (NaN where fewer than 1 / 2 trajectories contributed) and n [I][rows]
 * i64 contributing trajectories.  Destinations are caller-owned host
 * memory, or device memory with dst_is_device; any may be NULL.  Before it
 * returns, the following window is already enqueued. */
cwc_status cwc_stream_next(cwc_stream *s, int32_t *k0, int32_t *rows,
                           double *mean, double *var, int64_t *n,
                           int dst_is_device);
typedef struct {
    size_t device_bytes;     /* device memory the stream holds               */
    int32_t window;          /* sample points per window                     */
    int32_t n_windows;
    int32_t windows_done;    /* windows returned by cwc_stream_next          */
    float last_window_ms;    /* simulation time of the last window returned  */
    char kernel[48];         /* the time-sliced kernel the windows launch    */
} cwc_stream_info_t;
cwc_status cwc_stream_info(const cwc_stream *s, cwc_stream_info_t *info);
/* Per-trajectory results (as cwc_run_fetch_counters), once every window has
 * been returned; CWC_E_NOTREADY before. */
cwc_status cwc_stream_fetch_counters(cwc_stream *s, int64_t *events,
                                     uint8_t *status, uint64_t *digest,
                                     double *t_final, int32_t *n_recorded,
                                     int32_t *final_counts,
                                     int dst_is_device);
/* General models: each trajectory's final term, as cwc_run_fetch_term,
 * once every window has been returned.  Errors: CWC_E_NOTREADY before,
 * CWC_E_INVALID for a fixed-tree model. */
cwc_status cwc_stream_fetch_term(cwc_stream *s, int32_t *dst, int dst_is_device);
/* Waits for enqueued work and releases the stream's device memory. */
void cwc_stream_destroy(cwc_stream *s);

/* ------------------------------------------------------------ autotuner */

/* Times candidate launch shapes for this model and run -- lanes per
 * trajectory (1, 2, 4 or a wavefront, as the model fits), block size (64,
 * 128, 256), in persistent mode requested wavefronts per SIMD (16, 8, 4, 2,
 * 1), then the sampling-buffer depth and the refill chunk --
 * on the run's own inputs with the horizon shortened so that the whole
 * search takes about `budget_s` seconds, and returns the fastest in *out.
 * The choice is stored in a tuning table on disk (the library's cache
 * directory), keyed by the model's generated code, the run's mode, whether
 * it has a rate table, and log2 of its trajectory count; cwc_run_submit
 * uses a stored entry when the descriptor's tuning is NULL.  Results never
 * depend on the tuning.  Errors: as cwc_run_submit. */
cwc_status cwc_autotune(cwc_ctx *ctx, const cwc_model *m, const cwc_run_desc *d,
                        double budget_s, cwc_tuning *out);

/* ------------------------------------------------------------- serving */

/* Continuous batching (paper Sec. 5.2 schema ii: instances as objects that
 * can be stopped and restarted, time-sliced, scheduled on line).  A server
 * owns a device pool of `hbm_budget` bytes, four device streams and a
 * scheduler thread: jobs waiting in the queue are admitted (FIFO) when a job
 * slot and pool memory are free; a stream with no work in flight takes the
 * ready jobs of one model (oldest first, up to about half the device's
 * wavefronts) and runs one slice launch that advances every unfinished
 * trajectory of those jobs by at most `slice_events` draws, suspending the
 * rest to a device checkpoint; when a slice ends, jobs whose trajectories
 * have all finished get their statistics finalised, the others become ready
 * again.  Jobs therefore join and leave while others are on the GPU, and
 * streams advance independently.  A job's trajectories and statistics are
 * bit-identical to the same run submitted alone (counter-based stream).
 * Job memory stays on the device until cwc_server_release. */

#define CWC_JOB_QUEUED 0
#define CWC_JOB_ACTIVE 1
#define CWC_JOB_DONE   2

typedef struct {
    int32_t state;        /* CWC_JOB_*                                    */
    int32_t n_ticks;      /* slice launches the job took part in          */
    double t_submit;      /* seconds since server creation                */
    double t_admit;
    double t_done;        /* results ready (statistics finalised)         */
    int64_t events;       /* applied events (valid once done)             */
    int64_t bytes;        /* device memory held                           */
} cwc_job_info;

typedef struct {
    int64_t jobs_submitted, jobs_done, ticks;
    int64_t events;              /* applied events of finished jobs       */
    int64_t pool_bytes, pool_used, pool_peak;
    double busy_s;               /* wall time with a slice in flight      */
} cwc_server_stats;

/* hbm_budget: device bytes for the pool (from the context's arena or
 * hipMalloc).  max_active: job slots (1..1024).  slice_events: draws per
 * trajectory per tick (>= 1).  Errors: CWC_E_INVALID, CWC_E_NOMEM. */
cwc_status cwc_server_create(cwc_ctx *ctx, size_t hbm_budget, int32_t max_active,
                             int64_t slice_events, cwc_server **out);
/* Scheduling (paper Sec. 5.2 schema ii: slices at constant simulation
 * time; dispatching guided by predictive heuristics from the instances'
 * history).  slice_samples > 0: a slice also ends, for each trajectory,
 * before it records its slice_samples-th sample point of the slice, so a
 * job advances by equal spans of simulation time per slice (0: slices are
 * bounded by slice_events draws only); it applies to jobs admitted after
 * the call.  policy CWC_SCHED_FIFO: an idle stream takes the oldest ready
 * job's model group; CWC_SCHED_PREDICTED: jobs that have had no slice
 * first (in arrival order), then the job whose predicted remaining time --
 * remaining slices (sample points left / slice_samples) times its mean
 * slice wall time so far -- is longest (FIFO while slice_samples is 0).
 * CWC_SCHED_RESIDENT (paper Sec. 5.2: the farm's workers take instances
 * from one stream of tasks as they become free): no slices; each model
 * group (model, layout, rate-table use) has a queue of (job, trajectory)
 * items in coherent host memory, published as jobs are admitted, and
 * resident kernels of that group -- on eight streams of the server's own,
 * launched when items wait unclaimed -- keep claiming items and running
 * them to their end while new jobs arrive; a kernel's wavefront leaves
 * after 2 ms without an item, and the kernel that completes a job's last
 * item reports the job's id to the host.  (Every stream of the server,
 * slice and resident, has a hardware queue of its own.)  slice_events and slice_samples do not apply;
 * a job takes at most 2^18 items (wavefront-sized runs of trajectories).
 * The switch to or from CWC_SCHED_RESIDENT needs a server with no queued
 * or active job.  Results never depend on the policy.  Errors:
 * CWC_E_INVALID. */
#define CWC_SCHED_FIFO      0
#define CWC_SCHED_PREDICTED 1
#define CWC_SCHED_RESIDENT  2
cwc_status cwc_server_set_policy(cwc_server *s, int32_t slice_samples, int32_t policy);
/* Queues a job (never blocks).  Tables are copied.  mode and tuning of `d`
 * are ignored (the server's time-sliced or resident form is used).
 * CWC_E_NOMEM if the job alone exceeds the pool; CWC_E_INVALID as
 * cwc_run_submit; CWC_E_UNSUPPORTED for a resident-policy job of more than
 * 2^18 items. */
cwc_status cwc_server_submit(cwc_server *s, const cwc_model *m, const cwc_run_desc *d,
                             uint64_t *job_id);
/* Ids of jobs completed since the last poll (each reported once). */
cwc_status cwc_server_poll(cwc_server *s, uint64_t *done_ids, int32_t max, int32_t *n_done);
cwc_status cwc_server_job_info(cwc_server *s, uint64_t job, cwc_job_info *info);
/* As cwc_run_fetch_stats / cwc_run_fetch_counters for a completed job. */
cwc_status cwc_server_fetch_stats(cwc_server *s, uint64_t job, double *mean, double *var,
                                  int64_t *n, int dst_is_device);
cwc_status cwc_server_fetch_counters(cwc_server *s, uint64_t job, int64_t *events,
                                     uint8_t *status, uint64_t *digest, double *t_final,
                                     int32_t *n_recorded, int32_t *final_counts,
                                     int dst_is_device);
/* General models: a completed job's final terms, as cwc_run_fetch_term.
 * Errors: as cwc_server_fetch_counters; CWC_E_INVALID for a fixed-tree
 * model's job. */
cwc_status cwc_server_fetch_term(cwc_server *s, uint64_t job, int32_t *dst,
                                 int dst_is_device);
/* Frees a completed job's device memory; its id becomes invalid. */
cwc_status cwc_server_release(cwc_server *s, uint64_t job);
/* Blocks until no job is queued or active, or timeout_s elapses
 * (CWC_E_NOTREADY). */
cwc_status cwc_server_wait_idle(cwc_server *s, double timeout_s);
cwc_status cwc_server_get_stats(cwc_server *s, cwc_server_stats *st);
/* Stops the scheduler after the current tick and frees everything. */
void cwc_server_destroy(cwc_server *s);

/* --------------------------------------------------------------- stats */

/* Realignment onto the sample grid (paper Sec. 5.2 schema i: fixed-step
 * sampling simplifies the on-line reduction; trajectories recorded at
 * other times can be realigned while buffered).  Host function, no device.
 * times[n] non-decreasing, values[n][n_cells]: a piecewise-constant,
 * right-continuous trajectory (values[i] holds from times[i] on).  For
 * k = 0..n_samples-1, out[k][c] = values[j][c] with j the last index whose
 * times[j] <= k * dt (k * dt formed as the kernels form sample times), or
 * `fill` where no record precedes k * dt.  A trajectory the library
 * sampled on a grid of step dt / m realigned onto step dt gives the run on
 * step dt bit for bit.  Errors: CWC_E_INVALID (sizes, NULL arrays, dt not
 * finite and > 0, times NaN or decreasing). */
cwc_status cwc_realign(const double *times, const int32_t *values, int64_t n,
                       int32_t n_cells, double dt, int32_t n_samples,
                       int32_t fill, int32_t *out);

/* Confidence bands of the on-line statistics (paper Sec. 5.2 schema iii:
 * the reduction reports mean, variance and a confidence interval per
 * sample time).  Host function, no device: for each row r (an (instance,
 * sample) pair with n[r] trajectories) and cell c,
 *   half_width[r][c] = t_{(1+level)/2, n[r]-1} * sqrt(var[r][c] / n[r]),
 * the half-width of the two-sided Student-t interval around the mean at
 * the given level (0.9 for the paper's 90 % band); NaN where n[r] < 2.
 * var/half_width: [rows][n_cells] host arrays; n: [rows].  The t quantile
 * is accurate to about 1e-12 relative.  Errors: CWC_E_INVALID. */
cwc_status cwc_stats_confidence(const double *var, const int64_t *n, int64_t rows,
                                int32_t n_cells, double level, double *half_width);

/* Finalises exact moments into mean/var on the device (the same routine the
 * runs use).  All pointers are device pointers; rows = I*(K+1).
 * n[row] trajectories; s1/s2_hi32/s2_lo32 [row][C]. */
cwc_status cwc_stats_finalize(cwc_ctx *ctx, const int64_t *n,
                              const uint64_t *s1, const uint64_t *s2_hi32,
                              const uint64_t *s2_lo32, int64_t rows,
                              int32_t n_cells, double *mean, double *var,
                              void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* CWCSSA_H */
