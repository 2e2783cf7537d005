// Device engine, lane-per-replica layout: every lane of a wavefront runs
// its own trajectory of Gillespie's direct method over a CWC model whose
// slot structure has been compiled into the model section that precedes
// this file.  The model section defines CWC_C (cells), CWC_P (leaves),
// CWC_NR (rules) and statement macros over named scalar variables, so the
// whole per-lane state (counts, rates, propensity tree) lives in registers
// with no indexed arrays:
//   CWC_DECL_K / CWC_LOAD_K(ptr)       rate variables k<r>
//   CWC_DECL_STATE                     counts n<c>, tree nodes a<i>
//   CWC_LOAD_COUNTS(ptr) / CWC_STORE_COUNTS(ptr)
//   CWC_TREE                           leaves k * prod C(n, m), node sums
//   CWC_ROOT                           the root value (total propensity a0)
//   CWC_DESCEND(x, j)                  selection descent -> leaf index j
//   CWC_APPLY(j, cap, ovf)             net change of leaf j, in place, and
//                                      whether a count exceeds the cap
//   CWC_UNDO() / CWC_REDO()            take that change back / apply it again
//   CWC_STAGE(ptr, stride)             counts -> ptr[c * stride]
// and, for the two-lane (pair) layout, over the slots z<k> a lane keeps
// (the four-lane quad layout's CWC_QUAD_* likewise, with CWC_QUAD_PART):
//   CWC_PAIR_STATE / CWC_PAIR_DECL / CWC_PAIR_SETUP   slots; rates K<i>
//                                      and half tree q<i>; change table
//   CWC_PAIR_LOAD_COUNTS(ptr, h) / CWC_PAIR_STORE_COUNTS(ptr, h)
//   CWC_PAIR_STAGE(col0, h)            the lane's cells -> col0[c * 64]
//   CWC_PAIR_TREE(h) / CWC_PAIR_HALF / CWC_PAIR_DESCEND(x, j)
//   CWC_PAIR_APPLY_MX(j, mx) / CWC_PAIR_UNDO() / CWC_PAIR_REDO()
//
// One event (paper Sec. 2.3, Match / Resolve / Update):
//   Resolve  - one Philox4x32-10 block keyed by the run seed at counter
//              (event, trajectory) gives u_tau and u_sel; tau = -ln(u_tau)/a0
//              (Sec. 2.2 step 1); samples whose time precedes the event are
//              emitted; x = u_sel * a0 selects a leaf of the propensity tree
//              (Sec. 2.2 step 2: slot i with probability a_i / a0);
//   Update   - the chosen rule's net change is applied at its context;
//   Match    - (first, each iteration) every slot's propensity
//              k * prod C(n, m) and the tree are computed from the counts,
//              all in registers.
// Sampled states are reduced on line into exact integer moments per
// (instance, sample, cell) with 64-bit atomics (Sec. 5.2 schema iii).
//
// Requires engine_common.h (Philox4x32-10, uniforms, ssa_log).

// On-line reduction of sampled states (paper Sec. 5.2 schema iii): exact
// 64-bit sums of x and of x^2 per (instance, sample, cell); x^2 is split in
// 32-bit halves so no sum wraps for fewer than 2^32 trajectories.
//
// Each wavefront keeps a direct-mapped cache of accumulator rows in LDS
// (p.nslot rows, a power of two: the sampling-buffer depth), tagged by
// (instance, sample): a lane that records sample k of instance i adds its
// counts into slot h(i, k) with LDS atomics when the tag matches; otherwise
// one lane at a time writes the slot's row back to the global sums (device
// atomics) and re-tags it.  Rows are written back when the wavefront
// finishes.  Lanes of one instance record the same samples at nearby
// times, so a row can collect several trajectories before it is written
// back.  h maps the consecutive samples of one instance to consecutive
// slots and scatters instances over the slots.  All sums are exact
// integers: the result does not depend on the order or on the depth.
// Sampled trajectories are kept [sample][cell][trajectory], trajectory
// fastest: cell c of sample k of local trajectory lg sits at
// (k * C + c) * G + lg, so the lanes of a wavefront that record the same
// sample write neighbouring words of each cell row.  The pointer to
// (k, cell 0, lg); cell c is c * G further on.  A streamed run keeps only
// the rows of its current window: sample k is row k - k_base.
// Accumulator row of sample kn of instance inst: [I][KR] rows, row 0 being
// sample k_base (KR = K + 1 and k_base = 0 unless the run is streamed).
#define CWC_ROW(p, inst, kn) ((i64)(inst) * (i64)(p).KR + (i64)((kn) - (p).k_base))

#define CWC_TRAJ_AT(p, lg, kn)                                                \
    ((p).traj ? (p).traj + (i64)((kn) - (p).k_base) * (i64)CWC_C * (p).G + (lg) : (i32 *)0)

struct cwc_acc {
    unsigned long long *tag;   // [nslot]  accumulator row (CWC_ROW), ~0 = empty
    unsigned long long *s1;    // [nslot][C]
    unsigned long long *s2;    // [nslot][C] low 32-bit halves of x^2
    int mask;                  // nslot - 1
};

__device__ __forceinline__ int cwc_acc_slot(const cwc_acc &a, i64 inst, i32 kn)
{
    return (int)(((u32)kn + (((u32)inst * 0x9E3779B1u) >> 26)) & (u32)a.mask);
}

// keeps the compiler from moving LDS accesses across this point; the
// hardware executes one wavefront's LDS instructions in order
__device__ __forceinline__ void cwc_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void cwc_acc_init(const cwc_acc &a)
{
    const int lane = __lane_id();
    const int n = a.mask + 1;
    for (int i = lane; i < n; i += 64) a.tag[i] = ~0ull;
    for (int i = lane; i < n * CWC_C; i += 64) {
        a.s1[i] = 0ull;
        a.s2[i] = 0ull;
    }
    cwc_lds_order();
}

// write slot `sl` back to the global sums (one lane) and empty it
__device__ __forceinline__ void cwc_acc_flush_slot(const cwc_kparams &p, const cwc_acc &a, int sl)
{
    const unsigned long long key = a.tag[sl];
    if (key == ~0ull) return;
    const i64 row = (i64)key * (i64)CWC_C;
    unsigned long long *r1 = a.s1 + sl * CWC_C, *r2 = a.s2 + sl * CWC_C;
    // eight cells at a time: their loads are issued together
    constexpr int B = CWC_C < 8 ? CWC_C : 8;
#pragma unroll 1
    for (int c0 = 0; c0 < CWC_C; c0 += B) {
        unsigned long long x[B], q[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int c = c0 + i < CWC_C ? c0 + i : CWC_C - 1;
            x[i] = r1[c];
            q[i] = r2[c];
        }
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int c = c0 + i;
            if (c < CWC_C) {
                if (x[i]) atomicAdd(p.s1 + row + c, x[i]);
                if (q[i]) atomicAdd(p.s2_lo32 + row + c, q[i]);
                r1[c] = 0ull;
                r2[c] = 0ull;
            }
        }
    }
    a.tag[sl] = ~0ull;
}

// lanes of the calling (possibly partial) set record their staged state
__device__ __forceinline__ void cwc_emit_moments(const cwc_kparams &p, const cwc_acc &a,
                                                 const i32 *col, i64 inst, i32 kn, i32 *tr)
{
    const unsigned long long key = (unsigned long long)CWC_ROW(p, inst, kn);
    if (p.n_rows) atomicAdd(p.n_rows + key, 1ull);
    const int sl = cwc_acc_slot(a, inst, kn);
    unsigned long long *r1 = a.s1 + sl * CWC_C, *r2 = a.s2 + sl * CWC_C;
    bool pending = true;
    for (;;) {
        cwc_lds_order();
        if (pending && a.tag[sl] == key) {
#pragma unroll 4
            for (int c = 0; c < CWC_C; ++c) {
                const i32 v = col[c * 64];
                const u64 x = (u64)(u32)v;
                const u64 q = x * x;
                atomicAdd(r1 + c, x);
                atomicAdd(r2 + c, q & 0xFFFFFFFFull);
                if (q >> 32) atomicAdd(p.s2_hi32 + key * (u64)CWC_C + c, q >> 32);
                if (tr) tr[(i64)c * p.G] = v;
            }
            pending = false;
        }
        cwc_lds_order();
        // one lane whose slot holds another row writes it back and claims it
        const u64 want = __ballot(pending);
        if (!want) break;
        const int leader = __ffsll((long long)want) - 1;
        if (__lane_id() == leader) {
            cwc_acc_flush_slot(p, a, sl);
            a.tag[sl] = key;
        }
    }
}

__device__ __forceinline__ void cwc_acc_flush_all(const cwc_kparams &p, const cwc_acc &a)
{
    cwc_lds_order();
    if (__lane_id() == 0) {
        for (int sl = 0; sl <= a.mask; ++sl) cwc_acc_flush_slot(p, a, sl);
    }
}

// ------------------------------------------------------------- per-lane state
// The statement macros below operate on the locals declared by
// CWC_LANE_LOCALS; they are shared by the run-to-completion kernels and the
// time-sliced kernel of the serving form.
//
// The event loop is software-pipelined: the draw of event e (E = -ln u_tau,
// U = u_sel) is ready when the iteration starts, and the draw of event e+1
// is computed in the same straight-line block as event e's propensities,
// waiting time, selection and (in place) update, so the independent
// integer (Philox) and floating-point (tree, division, descent) chains
// overlap.  The update stands unless something rare happens -- a sample
// time is crossed, the state is absorbing, a count would exceed the cap,
// or the event cap is reached -- in which case the slow path takes it
// back and handles the event in the order the direct method defines.

#define CWC_GROUP_LOCALS                                                      \
    const double INF = __longlong_as_double(0x7FF0000000000000ll);            \
    /* dynamic LDS (sized by the host): per wavefront a staging area      \
       [cell][lane] i32, then per wavefront the accumulator cache: nslot   \
       tags, then nslot x C sums of x, then nslot x C sums of x^2 (u64) */  \
    extern __shared__ __align__(16) unsigned char cwc_lds[];                  \
    const int wv_ = (int)(threadIdx.x >> 6);                                  \
    i32 *const col = (i32 *)cwc_lds + wv_ * (CWC_C * 64) + (threadIdx.x & 63); \
    cwc_acc acc;                                                              \
    {                                                                         \
        const int ns_ = p.nslot;                                              \
        unsigned long long *b_ = (unsigned long long *)(cwc_lds +             \
            (blockDim.x >> 6) * (CWC_C * 64 * 4)) + wv_ * ns_ * (1 + 2 * CWC_C); \
        acc.tag = b_;                                                         \
        acc.s1 = b_ + ns_;                                                    \
        acc.s2 = b_ + ns_ + ns_ * CWC_C;                                      \
        acc.mask = ns_ - 1;                                                   \
    }                                                                         \
    cwc_acc_init(acc);                                                        \
    CWC_DECL_K;                                                               \
    CWC_DECL_STATE;                                                           \
    double t = 0.0, t_next = 0.0;   /* current time, next sample time */      \
    u64 e = 0, dig = 0;             /* applied events (= next draw), digest */ \
    i64 g = 0, lg = 0, inst = 0;    /* global / local id, instance */         \
    i32 kn = 0;                     /* next sample index */                   \
    i32 kstop = p.k_stop;           /* suspend before recording this one */   \
    double E = 0.0, U = 0.0;        /* draw e: -ln(u_tau), u_sel */           \
    (void)INF;
// the lane and quad layouts' locals: the group locals and the per-leaf
// change table in LDS
#define CWC_LANE_LOCALS                                                       \
    CWC_GROUP_LOCALS;                                                         \
    CWC_DT_SETUP

// time-sliced kernels: a slice of p.k_slice sample points (constant
// simulation time) ends before the trajectory records sample kn + k_slice
#define CWC_SLICE_STOP()                                                      \
    do {                                                                      \
        if (p.k_slice > 0 && (long long)kn + p.k_slice < (long long)p.k_stop) \
            kstop = kn + p.k_slice;                                           \
    } while (0)

// draw e of trajectory g
#define CWC_DRAW(ee, EO, UO)                                                  \
    do {                                                                      \
        u32 x0_, x1_, x2_, x3_;                                               \
        cwc_philox((u32)(ee), (u32)((ee) >> 32), (u32)g, (u32)((u64)g >> 32), \
                   (u32)p.seed, (u32)(p.seed >> 32), x0_, x1_, x2_, x3_);     \
        (EO) = -cwc_ssa_log(cwc_u_open0(x0_, x1_));                           \
        (UO) = cwc_u_open1(x2_, x3_);                                         \
    } while (0)

// identify trajectory lg of the run (instance, global id, rates)
#define CWC_IDENT(LG, SHARED_K)                                               \
    do {                                                                      \
        lg = (LG);                                                            \
        inst = (i64)((u32)lg / (u32)p.R);                                     \
        g = p.g_base + lg;                                                    \
        if (!(SHARED_K)) {                                                    \
            const double *kr_ = p.rates + (i64)p.rate_stride * inst;          \
            CWC_LOAD_K(kr_);                                                  \
        }                                                                     \
    } while (0)

// start the identified trajectory from the run's initial state
#define CWC_START()                                                           \
    do {                                                                      \
        { const i32 *ini_ = p.init + (i64)p.init_stride * inst;               \
          CWC_LOAD_COUNTS(ini_); }                                            \
        t = 0.0; t_next = 0.0; e = 0; kn = 0;                                 \
        dig = 0xcbf29ce484222325ull;                                          \
        CWC_DRAW(e, E, U);                                                    \
    } while (0)

// emit sample kn of the current state and move to the next sample time
#define CWC_EMIT()                                                            \
    do {                                                                      \
        i32 *tr_ = CWC_TRAJ_AT(p, lg, kn); \
        CWC_STAGE(col, 64);                                                   \
        cwc_emit_moments(p, acc, col, inst, kn, tr_);                         \
        kn += 1;                                                              \
        t_next = (kn < p.K1) ? (double)kn * p.dt : INF;                       \
    } while (0)

// one draw and, unless the trajectory ends, one applied event
#define CWC_STEP(st)                                                          \
    do {                                                                      \
        CWC_TREE;                       /* Match: propensities of the state */ \
        const double a0_ = CWC_ROOT;                                          \
        const double tn_ = t + E / a0_; /* Resolve: time of the event */      \
        double x_ = U * a0_;            /* Resolve: which slot */             \
        i32 j_;                                                               \
        CWC_DESCEND(x_, j_);                                                  \
        CWC_APPLY(j_, p.cap, ovf_);     /* Update, undone on the slow path */ \
        const u64 e1_ = e + 1;                                                \
        double E1_, U1_;                                                      \
        CWC_DRAW(e1_, E1_, U1_);        /* next draw, independent */          \
        const bool slow_ = (a0_ == 0.0) | (t_next < tn_) | ovf_ |             \
                           (e1_ == (u64)p.max_events);                        \
        if (!slow_) {                                                         \
            t = tn_; e = e1_; E = E1_; U = U1_;                               \
            if (p.want_digest) dig = (dig ^ (u64)(u32)j_) * 0x100000001b3ull; \
        } else if (a0_ == 0.0) {                                              \
            /* absorbing state: remaining samples hold the current counts */  \
            CWC_UNDO();                                                       \
            while (kn < p.K1 && kn < kstop) CWC_EMIT();                    \
            (st) = kn < p.K1 ? CWC_ST_WINDOW : CWC_ST_ABSORBED;               \
        } else {                                                              \
            CWC_UNDO();                                                       \
            while (t_next < tn_ && kn < kstop) CWC_EMIT();                 \
            if (t_next < tn_) {                                               \
                (st) = CWC_ST_WINDOW;   /* the window's last sample is done */ \
            } else if (kn >= p.K1) {                                          \
                (st) = CWC_ST_OK;       /* this draw lies past the horizon */ \
            } else if (ovf_) {                                                \
                (st) = CWC_ST_OVERFLOW;                                       \
            } else {                                                          \
                CWC_REDO();                                                   \
                t = tn_; e = e1_; E = E1_; U = U1_;                           \
                if (p.want_digest) dig = (dig ^ (u64)(u32)j_) * 0x100000001b3ull; \
                if (e == (u64)p.max_events) (st) = CWC_ST_EVENT_CAP;          \
            }                                                                 \
        }                                                                     \
    } while (0)

// terminal outputs of the trajectory
#define CWC_FINISH(st)                                                        \
    do {                                                                      \
        { i32 *fc_ = p.final_counts + lg * (i64)CWC_C; CWC_STORE_COUNTS(fc_); } \
        CWC_FINISH_REST(st);                                                  \
    } while (0)
// the per-trajectory results other than the final counts
#define CWC_FINISH_REST(st)                                                   \
    do {                                                                      \
        p.events[lg] = (i64)e;                                                \
        p.t_final[lg] = t;                                                    \
        p.digest[lg] = p.want_digest ? dig : 0ull;                            \
        p.status[lg] = (unsigned char)(st);                                   \
        p.n_recorded[lg] = kn;                                                \
        if (p.rec_hist) atomicAdd(p.rec_hist + inst * (i64)(p.K1 + 1) + kn, 1ull); \
    } while (0)

// Queue claim of the persistent forms, called by the whole wavefront when
// some of its lane groups (G lanes per trajectory: 1, 2 or 4) need a new
// item; `want` is the ballot of the lanes that do.  The wanting groups take
// the next unclaimed items in lane order with at most one queue atomic per
// wavefront.  With chunked claims (p.chunk >= 64) they drain the
// wavefront's window [w_next, w_end) first and claim a new chunk only when
// it runs short, so a wavefront works on few instances at a time and its
// accumulator rows fill up.  Returns this lane's item (for the wanting
// lanes; >= p.G once the queue is exhausted).
template <int G>
__device__ __forceinline__ i64 cwc_claim(const cwc_kparams &p, u64 want, i64 &w_next, i64 &w_end)
{
    const u64 firsts = G == 1 ? want
                              : want & (G == 2 ? 0x5555555555555555ull : 0x1111111111111111ull);
    const int cnt = __popcll(firsts);
    const int lane = __lane_id();
    const int leader = __ffsll((long long)want) - 1;
    const int rank = __popcll(firsts & ((1ull << (lane & ~(G - 1))) - 1ull));
    i64 item;
    if (p.chunk <= 1) {
        u64 base = 0;
        if (lane == leader) base = atomicAdd(p.cursor, (u64)cnt);
        base = __shfl(base, leader);
        item = (i64)base + rank;
    } else {
        const i64 avail = w_end - w_next;   /* >= 0 */
        if (avail >= cnt) {
            item = w_next + rank;
            w_next += cnt;
        } else {
            // cnt - avail <= 64 <= chunk: one new chunk suffices
            u64 base = 0;
            if (lane == leader) base = atomicAdd(p.cursor, (u64)p.chunk);
            base = __shfl(base, leader);
            const i64 nb = (i64)base;
            item = rank < avail ? w_next + rank : nb + (rank - avail);
            w_end = nb + p.chunk < p.G ? nb + p.chunk : p.G;
            w_next = nb + (cnt - avail);
            if (w_next > w_end) w_next = w_end;
        }
    }
    return item;
}

template <bool PERSIST, bool SHARED_K>
__device__ __forceinline__ void cwc_lane_main(const cwc_kparams &p)
{
    CWC_LANE_LOCALS;
    if (SHARED_K) { CWC_LOAD_K(p.rates); }

    // begin the trajectory of claimed item `item`
#define CWC_BEGIN(item)                                                       \
    do {                                                                      \
        i64 lg0_ = (item);                                                    \
        if (p.order) {                                                        \
            const u32 grp_ = (u32)(item) / (u32)p.R;                          \
            const u32 rep_ = (u32)(item) - grp_ * (u32)p.R;                   \
            lg0_ = (i64)p.order[grp_] * p.R + rep_;                           \
        }                                                                     \
        CWC_IDENT(lg0_, SHARED_K);                                            \
        CWC_START();                                                          \
    } while (0)

    const i64 tid = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    bool active = tid < p.G;
    bool live = active;             // persistent form: may still receive work
    // persistent form with chunked claims: the wavefront's window of
    // claimed, not yet started items [w_next, w_end) (wave-uniform)
    i64 w_next = 0, w_end = 0;
    if (active) CWC_BEGIN(tid);
    for (;;) {
        if (PERSIST) {
            // lanes whose trajectory ended take the next unclaimed items
            const u64 want = __ballot(live && !active);
            if (want) {
                const i64 item = cwc_claim<1>(p, want, w_next, w_end);
                if (live && !active) {
                    if (item < p.G) {
                        CWC_BEGIN(item);
                        active = true;
                    } else {
                        live = false;
                    }
                }
            }
            if (!__any(live)) break;
        } else {
            if (!__any(active)) break;
        }
        if (!active) continue;
        int st = CWC_ST_RUNNING;
        CWC_STEP(st);
        if (st != CWC_ST_RUNNING) {
            CWC_FINISH(st);
            active = false;
        }
    }
    cwc_acc_flush_all(p, acc);
#undef CWC_BEGIN
}

// Time-sliced form (serving): the launch covers many jobs of this model;
// wavefront w works on job wave_job[w], trajectories wave_first[w] + lane.
// A trajectory resumes from its checkpoint (or starts), runs at most
// `budget` draws, then either finishes or is suspended back to its
// checkpoint.  The counter-based random stream makes the split invisible:
// the trajectory is identical to an uninterrupted run.
// Resident form (RESIDENT): the wavefront claims items (job, first
// trajectory) from the host's queue instead, runs each to its end and
// counts it toward its job, until the queue is closed or stays empty.
template <bool SHARED_K, bool RESIDENT>
__device__ __forceinline__ void cwc_lane_slice(const cwc_kparams *jobs, const int *wave_job,
                                               const long long *wave_first, long long budget,
                                               const cwc_rq &q)
{
    const int w = (int)((blockIdx.x * (u64)blockDim.x + threadIdx.x) >> 6);
    // the resident form's LDS layout takes the queue's accumulator depth,
    // the same for every job of the kernel
    cwc_kparams pr{};
    pr.nslot = q.nslot;
    pr.k_stop = 0x7FFFFFFF;
    const cwc_kparams &p = RESIDENT ? pr : jobs[wave_job[w]];
    CWC_LANE_LOCALS;
    // one item: trajectories first + lane of job p; returns how many of
    // them the item finished
    auto item = [&](const cwc_kparams &p, i64 first, long long budget) -> u32 {
        kstop = p.k_stop;
        if (SHARED_K) { CWC_LOAD_K(p.rates); }
        const i64 my = first + (i64)(threadIdx.x & 63);
        bool active = my < p.G && p.ck_state[my] != 2;
        if (active) {
            CWC_IDENT(my, SHARED_K);
            if (p.ck_state[my] == 0) {
                CWC_START();
            } else {
                { const i32 *ck_ = p.ck_counts + lg * (i64)CWC_C; CWC_LOAD_COUNTS(ck_); }
                t = p.ck_t[lg];
                e = p.ck_e[lg];
                dig = p.ck_dig[lg];
                kn = p.ck_kn[lg];
                t_next = (kn < p.K1) ? (double)kn * p.dt : INF;
                CWC_DRAW(e, E, U);
            }
            CWC_SLICE_STOP();
        }
        bool fin = false;
        long long n = 0;
        while (__any(active)) {
            if (!active) continue;
            int st = CWC_ST_RUNNING;
            CWC_STEP(st);
            ++n;
            if (st != CWC_ST_RUNNING && st != CWC_ST_WINDOW) {
                CWC_FINISH(st);
                p.ck_state[lg] = 2;
                if (!RESIDENT) atomicAdd(p.done_count, 1ull);
                fin = true;
                active = false;
            } else if (st == CWC_ST_WINDOW || n == budget) {
                { i32 *ck_ = p.ck_counts + lg * (i64)CWC_C; CWC_STORE_COUNTS(ck_); }
                p.ck_t[lg] = t;
                p.ck_e[lg] = e;
                p.ck_dig[lg] = dig;
                p.ck_kn[lg] = kn;
                p.ck_state[lg] = 1;
                active = false;
            }
        }
        cwc_acc_flush_all(p, acc);
        return (u32)__popcll(__ballot(fin));
    };
    if (!RESIDENT) {
        item(p, wave_first[w], budget);
        return;
    }
    __shared__ cwc_kparams rq_kp[4];                  // per wavefront of the block
    cwc_kparams &jp = rq_kp[threadIdx.x >> 6];
    int slot;
    i64 first, job;
    while (cwc_rq_claim(q, slot, first, job)) {
        cwc_rq_params(&jp, jobs + slot);
        const u32 n = item(jp, first, 0x7FFFFFFFFFFFFFFFll);
        cwc_rq_finish(q, jp, slot, job, n);
    }
}

extern "C" __global__ void __launch_bounds__(256)
cwc_lane_plain_shared(cwc_kparams p) { cwc_lane_main<false, true>(p); }
extern "C" __global__ void __launch_bounds__(256)
cwc_lane_plain_table(cwc_kparams p) { cwc_lane_main<false, false>(p); }
extern "C" __global__ void __launch_bounds__(256)
cwc_lane_persistent_shared(cwc_kparams p) { cwc_lane_main<true, true>(p); }
extern "C" __global__ void __launch_bounds__(256)
cwc_lane_persistent_table(cwc_kparams p) { cwc_lane_main<true, false>(p); }
extern "C" __global__ void __launch_bounds__(256)
cwc_lane_slice_shared(const cwc_kparams *jobs, const int *wave_job, const long long *wave_first,
                      long long budget)
{ cwc_lane_slice<true, false>(jobs, wave_job, wave_first, budget, cwc_rq{}); }
extern "C" __global__ void __launch_bounds__(256)
cwc_lane_slice_table(const cwc_kparams *jobs, const int *wave_job, const long long *wave_first,
                     long long budget)
{ cwc_lane_slice<false, false>(jobs, wave_job, wave_first, budget, cwc_rq{}); }
extern "C" __global__ void __launch_bounds__(256)
cwc_lane_resident_shared(const cwc_kparams *jobs, cwc_rq q)
{ cwc_lane_slice<true, true>(jobs, nullptr, nullptr, 0, q); }
extern "C" __global__ void __launch_bounds__(256)
cwc_lane_resident_table(const cwc_kparams *jobs, cwc_rq q)
{ cwc_lane_slice<false, true>(jobs, nullptr, nullptr, 0, q); }

#ifdef CWC_PAIR
// ------------------------------------------------------------ pair layout
// Two lanes per trajectory (lane bit h): lane h holds half h of the
// propensity tree (leaves [h*B, (h+1)*B)), both hold the counts.  Per event:
// each lane builds its half; the root is its half plus the partner's (one
// DPP swap; the sum is the same in both lanes); both take the root decision,
// then each descends its own half and the lane holding the chosen half
// supplies the leaf index; both apply the change.  The draws are shared:
// on even iterations of the wavefront lane 1 computes the draw of the next
// event and lane 0 the one after, so Philox and ssa_log run every other
// iteration; the event of an even iteration uses lane 0's draw, of an odd
// one lane 1's.  Every pair of a wavefront follows this parity, so the draw
// code is wavefront-uniform.  Results are those of the lane layout bit for
// bit: the same tree, the same descent, the same draws per event.

// Values of the pair's lanes (DPP quad permutations; both lanes of a pair
// are always active together, so every source lane is live): the value of
// lane 0 of the pair ([0,0,2,2]) and of lane 1 ([1,1,3,3]), in both lanes.
template <int CTRL>
__device__ __forceinline__ int cwc_pair_dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double cwc_pair_dpp(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = cwc_pair_dpp_i<CTRL>((int)b);
    const int hi = cwc_pair_dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
#define CWC_PAIR_LO 0xA0
#define CWC_PAIR_HI 0xF5
#define CWC_PAIR_SWAP 0xB1

// Both lanes take the pair's two fresh draws: lane 1's (the next event,
// an odd iteration) into Eo/Uo, lane 0's (the one after, an even
// iteration) into E/U.
#define CWC_PAIR_SPREAD(EN, UN)                                               \
    do {                                                                      \
        Eo = cwc_pair_dpp<CWC_PAIR_HI>(EN);                                   \
        Uo = cwc_pair_dpp<CWC_PAIR_HI>(UN);                                   \
        E = cwc_pair_dpp<CWC_PAIR_LO>(EN);                                    \
        U = cwc_pair_dpp<CWC_PAIR_LO>(UN);                                    \
    } while (0)

// Locals of the pair kernels: the group locals, the lane's count slots,
// the lane's rates and half tree, and its change table in LDS.
#define CWC_PAIR_LOCALS                                                       \
    CWC_GROUP_LOCALS;                                                         \
    CWC_PAIR_STATE;                                                           \
    CWC_PAIR_DECL;                                                            \
    CWC_PAIR_SETUP

// Every lane of a group (pair or quad; STAGE its staging macro) writes the
// counts it keeps into the group's lane 0's staging column, in place for
// lane 0 to record the sample.
#define CWC_GROUP_STAGE_ALL(STAGE)                                            \
    do {                                                                      \
        i32 *c0_ = col - h_;                                                  \
        STAGE(c0_, h_);                                                       \
        cwc_lds_order();                                                      \
    } while (0)

// terminal outputs: each lane of a group writes the counts it keeps
// (STORE its count-row macro), lane 0 the rest
#define CWC_GROUP_FINISH(st, STORE)                                           \
    do {                                                                      \
        { i32 *fc_ = p.final_counts + lg * (i64)CWC_C;                        \
          STORE(fc_, h_); }                                                   \
        if (h_ == 0) CWC_FINISH_REST(st);                                     \
    } while (0)

// One step of a pair (the locals of the pair kernels, CWC_PEMIT and h_ in
// scope): the event of this iteration -- its draw is E/U at an even
// iteration, Eo/Uo at an odd one, the same in both lanes -- and, at an
// even iteration, the next two draws (lane 1: e+1, lane 0: e+2).  The root
// is lane 0's half plus lane 1's, in that order in both lanes.
#define CWC_PAIR_STEP_BODY(st, EVEN)                                          \
    do {                                                                      \
        CWC_PAIR_TREE(h_);                                                    \
        const double s_ = CWC_PAIR_HALF;                                      \
        const double L0_ = cwc_pair_dpp<CWC_PAIR_LO>(s_);                     \
        const double R0_ = cwc_pair_dpp<CWC_PAIR_HI>(s_);                     \
        const double a0_ = L0_ + R0_;                                         \
        const double tn_ = t + ((EVEN) ? E : Eo) / a0_;                       \
        double x_ = ((EVEN) ? U : Uo) * a0_;                                  \
        const bool b0_ = (x_ >= L0_) && (R0_ != 0.0);                         \
        x_ = b0_ ? x_ - L0_ : x_;                                             \
        int jl_ = 0;                                                          \
        CWC_PAIR_DESCEND(x_, jl_);                                            \
        const int j0_ = cwc_pair_dpp_i<CWC_PAIR_LO>(jl_);                     \
        const int j1_ = cwc_pair_dpp_i<CWC_PAIR_HI>(jl_);                     \
        const i32 j_ = b0_ ? CWC_PB + j1_ : j0_;                              \
        CWC_PAIR_APPLY_MX(j_, mxl_);                                          \
        const unsigned mxo_ = (unsigned)cwc_pair_dpp_i<CWC_PAIR_SWAP>((int)mxl_); \
        const bool ovf_ = (mxl_ > mxo_ ? mxl_ : mxo_) > p.cap;                \
        double En_ = 0.0, Un_ = 0.0;                                          \
        if (EVEN) {                                                           \
            const u64 d1_ = e + 2ull - (u64)h_;                               \
            CWC_DRAW(d1_, En_, Un_);                                          \
        }                                                                     \
        const bool slow_ = (a0_ == 0.0) | (t_next < tn_) | ovf_ |             \
                           (e + 1 == (u64)p.max_events);                      \
        if (!slow_) {                                                         \
            t = tn_; e = e + 1;                                               \
            if (EVEN) CWC_PAIR_SPREAD(En_, Un_);                              \
            if (p.want_digest) dig = (dig ^ (u64)(u32)j_) * 0x100000001b3ull; \
        } else if (a0_ == 0.0) {                                              \
            CWC_PAIR_UNDO();                                                  \
            while (kn < p.K1 && kn < kstop) CWC_PEMIT();                   \
            (st) = kn < p.K1 ? CWC_ST_WINDOW : CWC_ST_ABSORBED;               \
        } else {                                                              \
            CWC_PAIR_UNDO();                                                  \
            while (t_next < tn_ && kn < kstop) CWC_PEMIT();                \
            if (t_next < tn_) {                                               \
                (st) = CWC_ST_WINDOW;                                         \
            } else if (kn >= p.K1) {                                          \
                (st) = CWC_ST_OK;                                             \
            } else if (ovf_) {                                                \
                (st) = CWC_ST_OVERFLOW;                                       \
            } else {                                                          \
                CWC_PAIR_REDO();                                              \
                t = tn_; e = e + 1;                                           \
                if (EVEN) CWC_PAIR_SPREAD(En_, Un_);                          \
                if (p.want_digest) dig = (dig ^ (u64)(u32)j_) * 0x100000001b3ull; \
                if (e == (u64)p.max_events) (st) = CWC_ST_EVENT_CAP;          \
            }                                                                 \
        }                                                                     \
    } while (0)

template <bool PERSIST, bool SHARED_K>
__device__ __forceinline__ void cwc_pair_main(const cwc_kparams &p)
{
    CWC_PAIR_LOCALS;
    const int h_ = (int)(__lane_id() & 1u);
    if (SHARED_K) { CWC_PAIR_LOAD_K(p.rates, h_); }
    u32 it = 0;                     // wavefront iteration (parity: whose draw)
    double Eo = 0.0, Uo = 0.0;      // draw of the next odd-iteration event

    // begin the trajectory of item `item` at the current iteration: at an
    // even one both lanes take draw 0 (E/U); at an odd one draw 0 goes to
    // Eo/Uo and draw 1, for the even iteration after, to E/U (that
    // iteration then draws 2 and 3)
#define CWC_PBEGIN(item)                                                      \
    do {                                                                      \
        i64 lg0_ = (item);                                                    \
        if (p.order) {                                                        \
            const u32 grp_ = (u32)(item) / (u32)p.R;                          \
            const u32 rep_ = (u32)(item) - grp_ * (u32)p.R;                   \
            lg0_ = (i64)p.order[grp_] * p.R + rep_;                           \
        }                                                                     \
        lg = lg0_;                                                            \
        inst = (i64)((u32)lg / (u32)p.R);                                     \
        g = p.g_base + lg;                                                    \
        if (!SHARED_K) {                                                      \
            const double *kr_ = p.rates + (i64)p.rate_stride * inst;          \
            CWC_PAIR_LOAD_K(kr_, h_);                                         \
        }                                                                     \
        { const i32 *ini_ = p.init + (i64)p.init_stride * inst;               \
          CWC_PAIR_LOAD_COUNTS(ini_, h_); }                                   \
        t = 0.0; t_next = 0.0; e = 0; kn = 0;                                 \
        dig = 0xcbf29ce484222325ull;                                          \
        if (it & 1u) {                                                        \
            /* odd iteration: lane 1 draws 0 (this event), lane 0 draws 1 */  \
            double Et_, Ut_;                                                  \
            const u64 d0_ = (u64)(1 - h_);                                    \
            CWC_DRAW(d0_, Et_, Ut_);                                          \
            CWC_PAIR_SPREAD(Et_, Ut_);                                        \
        } else {                                                              \
            CWC_DRAW(0ull, E, U);                                             \
        }                                                                     \
    } while (0)

    // sample kn of the current state (lane 0 of the pair records it)
#define CWC_PEMIT()                                                           \
    do {                                                                      \
        CWC_GROUP_STAGE_ALL(CWC_PAIR_STAGE);                                                 \
        if (h_ == 0) {                                                        \
            i32 *tr_ = CWC_TRAJ_AT(p, lg, kn);                                \
            cwc_emit_moments(p, acc, col, inst, kn, tr_);                     \
        }                                                                     \
        kn += 1;                                                              \
        t_next = (kn < p.K1) ? (double)kn * p.dt : INF;                       \
    } while (0)

    const i64 tid = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const i64 pid = tid >> 1;
    bool active = pid < p.G;
    bool live = active;
    i64 w_next = 0, w_end = 0;      // chunked claims: the wavefront's window
    if (active) CWC_PBEGIN(pid);

    // persistent form: pairs whose trajectory ended take the next items
#define CWC_PREFILL                                                           \
    if (PERSIST) {                                                            \
        const u64 want = __ballot(live && !active);                           \
        if (want) {                                                           \
            const i64 item = cwc_claim<2>(p, want, w_next, w_end);           \
            if (live && !active) {                                            \
                if (item < p.G) {                                             \
                    CWC_PBEGIN(item);                                         \
                    active = true;                                            \
                } else {                                                      \
                    live = false;                                             \
                }                                                             \
            }                                                                 \
        }                                                                     \
        if (!__any(live)) break;                                              \
    } else {                                                                  \
        if (!__any(active)) break;                                            \
    }

    for (;;) {
        CWC_PREFILL
        if (active) {
            int st = CWC_ST_RUNNING;
            CWC_PAIR_STEP_BODY(st, true);
            if (st != CWC_ST_RUNNING) {
                CWC_GROUP_FINISH(st, CWC_PAIR_STORE_COUNTS);
                active = false;
            }
        }
        it += 1u;
        CWC_PREFILL
        if (active) {
            int st = CWC_ST_RUNNING;
            CWC_PAIR_STEP_BODY(st, false);
            if (st != CWC_ST_RUNNING) {
                CWC_GROUP_FINISH(st, CWC_PAIR_STORE_COUNTS);
                active = false;
            }
        }
        it += 1u;
    }
    cwc_acc_flush_all(p, acc);
#undef CWC_PREFILL
#undef CWC_PEMIT
#undef CWC_PBEGIN
}

// Time-sliced pair form (serving): wavefront w works on job wave_job[w],
// trajectories wave_first[w] + lane / 2; each pair resumes from its
// checkpoint (or starts), runs at most `budget` draws, then finishes or is
// suspended.  The slice starts at an even iteration, so lane 0 takes the
// draw of the current event and lane 1 receives the next one from the
// first even iteration's pair of draws.  Resident form (RESIDENT): items
// claimed from the host's queue, each run to its end (as the lane form).
template <bool SHARED_K, bool RESIDENT>
__device__ __forceinline__ void cwc_pair_slice(const cwc_kparams *jobs, const int *wave_job,
                                               const long long *wave_first, long long budget,
                                               const cwc_rq &q)
{
    const int w = (int)((blockIdx.x * (u64)blockDim.x + threadIdx.x) >> 6);
    cwc_kparams pr{};
    pr.nslot = q.nslot;
    pr.k_stop = 0x7FFFFFFF;
    const cwc_kparams &p = RESIDENT ? pr : jobs[wave_job[w]];
    CWC_PAIR_LOCALS;
    const int h_ = (int)(__lane_id() & 1u);
    double Eo = 0.0, Uo = 0.0;      // draw of the next odd-iteration event
    auto item = [&](const cwc_kparams &p, i64 first, long long budget) -> u32 {
        kstop = p.k_stop;
        if (SHARED_K) { CWC_PAIR_LOAD_K(p.rates, h_); }
        const i64 my = first + (i64)((threadIdx.x & 63) >> 1);
        bool active = my < p.G && p.ck_state[my] != 2;
        if (active) {
            lg = my;
            inst = (i64)((u32)lg / (u32)p.R);
            g = p.g_base + lg;
            if (!SHARED_K) {
                const double *kr_ = p.rates + (i64)p.rate_stride * inst;
                CWC_PAIR_LOAD_K(kr_, h_);
            }
            if (p.ck_state[my] == 0) {
                { const i32 *ini_ = p.init + (i64)p.init_stride * inst; CWC_PAIR_LOAD_COUNTS(ini_, h_); }
                t = 0.0; t_next = 0.0; e = 0; kn = 0;
                dig = 0xcbf29ce484222325ull;
            } else {
                { const i32 *ck_ = p.ck_counts + lg * (i64)CWC_C; CWC_PAIR_LOAD_COUNTS(ck_, h_); }
                t = p.ck_t[lg];
                e = p.ck_e[lg];
                dig = p.ck_dig[lg];
                kn = p.ck_kn[lg];
                t_next = (kn < p.K1) ? (double)kn * p.dt : INF;
            }
            CWC_DRAW(e, E, U);
            CWC_SLICE_STOP();
        }
        bool fin = false;
        long long n = 0;
#define CWC_PEMIT()                                                           \
    do {                                                                      \
        CWC_GROUP_STAGE_ALL(CWC_PAIR_STAGE);                                                 \
        if (h_ == 0) {                                                        \
            i32 *tr_ = CWC_TRAJ_AT(p, lg, kn);                                \
            cwc_emit_moments(p, acc, col, inst, kn, tr_);                     \
        }                                                                     \
        kn += 1;                                                              \
        t_next = (kn < p.K1) ? (double)kn * p.dt : INF;                       \
    } while (0)
    // after a step: finish, or suspend once the slice's draws are used
#define CWC_PSLICE_AFTER(st)                                                  \
    do {                                                                      \
        if ((st) != CWC_ST_RUNNING && (st) != CWC_ST_WINDOW) {                \
            { i32 *fc_ = p.final_counts + lg * (i64)CWC_C;                    \
              CWC_PAIR_STORE_COUNTS(fc_, h_); }                               \
            if (h_ == 0) {                                                    \
                CWC_FINISH_REST(st);                                          \
                p.ck_state[lg] = 2;                                           \
                if (!RESIDENT) atomicAdd(p.done_count, 1ull);                 \
                fin = true;                                                   \
            }                                                                 \
            active = false;                                                   \
        } else if ((st) == CWC_ST_WINDOW || n == budget) {                    \
            { i32 *ck_ = p.ck_counts + lg * (i64)CWC_C;                       \
              CWC_PAIR_STORE_COUNTS(ck_, h_); }                               \
            if (h_ == 0) {                                                    \
                p.ck_t[lg] = t;                                               \
                p.ck_e[lg] = e;                                               \
                p.ck_dig[lg] = dig;                                           \
                p.ck_kn[lg] = kn;                                             \
                p.ck_state[lg] = 1;                                           \
            }                                                                 \
            active = false;                                                   \
        }                                                                     \
    } while (0)
        while (__any(active)) {
            if (active) {
                int st = CWC_ST_RUNNING;
                ++n;
                CWC_PAIR_STEP_BODY(st, true);
                CWC_PSLICE_AFTER(st);
            }
            if (!__any(active)) break;
            if (active) {
                int st = CWC_ST_RUNNING;
                ++n;
                CWC_PAIR_STEP_BODY(st, false);
                CWC_PSLICE_AFTER(st);
            }
        }
#undef CWC_PSLICE_AFTER
#undef CWC_PEMIT
        cwc_acc_flush_all(p, acc);
        return (u32)__popcll(__ballot(fin));
    };
    if (!RESIDENT) {
        item(p, wave_first[w], budget);
        return;
    }
    __shared__ cwc_kparams rq_kp[4];                  // per wavefront of the block
    cwc_kparams &jp = rq_kp[threadIdx.x >> 6];
    int slot;
    i64 first, job;
    while (cwc_rq_claim(q, slot, first, job)) {
        cwc_rq_params(&jp, jobs + slot);
        const u32 n = item(jp, first, 0x7FFFFFFFFFFFFFFFll);
        cwc_rq_finish(q, jp, slot, job, n);
    }
}

extern "C" __global__ void __launch_bounds__(256)
cwc_pair_plain_shared(cwc_kparams p) { cwc_pair_main<false, true>(p); }
extern "C" __global__ void __launch_bounds__(256)
cwc_pair_plain_table(cwc_kparams p) { cwc_pair_main<false, false>(p); }
extern "C" __global__ void __launch_bounds__(256)
cwc_pair_persistent_shared(cwc_kparams p) { cwc_pair_main<true, true>(p); }
extern "C" __global__ void __launch_bounds__(256)
cwc_pair_persistent_table(cwc_kparams p) { cwc_pair_main<true, false>(p); }
extern "C" __global__ void __launch_bounds__(256)
cwc_pair_slice_shared(const cwc_kparams *jobs, const int *wave_job, const long long *wave_first,
                      long long budget)
{ cwc_pair_slice<true, false>(jobs, wave_job, wave_first, budget, cwc_rq{}); }
extern "C" __global__ void __launch_bounds__(256)
cwc_pair_slice_table(const cwc_kparams *jobs, const int *wave_job, const long long *wave_first,
                     long long budget)
{ cwc_pair_slice<false, false>(jobs, wave_job, wave_first, budget, cwc_rq{}); }
extern "C" __global__ void __launch_bounds__(256)
cwc_pair_resident_shared(const cwc_kparams *jobs, cwc_rq q)
{ cwc_pair_slice<true, true>(jobs, nullptr, nullptr, 0, q); }
extern "C" __global__ void __launch_bounds__(256)
cwc_pair_resident_table(const cwc_kparams *jobs, cwc_rq q)
{ cwc_pair_slice<false, true>(jobs, nullptr, nullptr, 0, q); }
#endif  // CWC_PAIR

#ifdef CWC_QUAD
// ------------------------------------------------------------ quad layout
// Four lanes per trajectory (lane bits h = lane & 3): lane h holds quarter h
// of the propensity tree (leaves [h*B, (h+1)*B)) and the counts that quarter
// reads (the generated per-lane slots, as the pair layout's).
// Per event: each lane builds its quarter; every lane reads the four
// quarter sums (DPP broadcasts of lanes 0..3 of the quad) and forms the two
// halves and the root in the canonical order; all take the two top
// decisions, each descends its own quarter and the leaf index is read from
// the lane holding the chosen quarter; each lane applies the change to its
// slots, and the cap test takes the largest growth of the four lanes.  Draws: at
// iterations of phase 0 (it % 4 == 0) lane k draws e + 1 + ((k + 3) % 4)
// and the four draws are spread at once, so the events of phases 1, 2, 3
// and the next phase 0 find theirs in E1..E3 and E0.  Every quad of a
// wavefront follows the wavefront's phase.  Results are those of the lane
// layout bit for bit.  Like a pair, a quad's lanes are always active
// together.  (Lanes of a quad whose quarter holds no slot compute zeros.)
#define CWC_QL0 0x00
#define CWC_QL1 0x55
#define CWC_QL2 0xAA
#define CWC_QL3 0xFF
#define CWC_QSWAP1 0xB1
#define CWC_QSWAP2 0x4E

#define CWC_QUAD_SPREAD(EN, UN)                                               \
    do {                                                                      \
        E0 = cwc_pair_dpp<CWC_QL0>(EN); U0 = cwc_pair_dpp<CWC_QL0>(UN);       \
        E1 = cwc_pair_dpp<CWC_QL1>(EN); U1 = cwc_pair_dpp<CWC_QL1>(UN);       \
        E2 = cwc_pair_dpp<CWC_QL2>(EN); U2 = cwc_pair_dpp<CWC_QL2>(UN);       \
        E3 = cwc_pair_dpp<CWC_QL3>(EN); U3 = cwc_pair_dpp<CWC_QL3>(UN);       \
    } while (0)

// One step of a quad at phase PH (0..3, a constant): the event of this
// iteration with draw E<PH>/U<PH>; at phase 0 also the next four draws.
#define CWC_QUAD_STEP_BODY(st, PH)                                            \
    do {                                                                      \
        CWC_QUAD_TREE(h_);                                                    \
        const double s_ = CWC_QUAD_PART;                                      \
        const double p0_ = cwc_pair_dpp<CWC_QL0>(s_);                         \
        const double p1_ = cwc_pair_dpp<CWC_QL1>(s_);                         \
        const double p2_ = cwc_pair_dpp<CWC_QL2>(s_);                         \
        const double p3_ = cwc_pair_dpp<CWC_QL3>(s_);                         \
        const double n1_ = p0_ + p1_;                                         \
        const double n2_ = p2_ + p3_;                                         \
        const double a0_ = n1_ + n2_;                                         \
        const double Ec_ = (PH) == 0 ? E0 : (PH) == 1 ? E1 : (PH) == 2 ? E2 : E3; \
        const double Uc_ = (PH) == 0 ? U0 : (PH) == 1 ? U1 : (PH) == 2 ? U2 : U3; \
        const double tn_ = t + Ec_ / a0_;                                     \
        double x_ = Uc_ * a0_;                                                \
        const bool b0_ = (x_ >= n1_) && (n2_ != 0.0);                         \
        x_ = b0_ ? x_ - n1_ : x_;                                             \
        const double L1_ = b0_ ? p2_ : p0_;                                   \
        const double R1_ = b0_ ? p3_ : p1_;                                   \
        const bool b1_ = (x_ >= L1_) && (R1_ != 0.0);                         \
        x_ = b1_ ? x_ - L1_ : x_;                                             \
        int jl_ = 0;                                                          \
        CWC_QUAD_DESCEND(x_, jl_);                                            \
        const int j0_ = cwc_pair_dpp_i<CWC_QL0>(jl_);                         \
        const int j1_ = cwc_pair_dpp_i<CWC_QL1>(jl_);                         \
        const int j2_ = cwc_pair_dpp_i<CWC_QL2>(jl_);                         \
        const int j3_ = cwc_pair_dpp_i<CWC_QL3>(jl_);                         \
        const i32 jq_ = b0_ ? (b1_ ? j3_ : j2_) : (b1_ ? j1_ : j0_);          \
        const i32 j_ = ((b0_ ? 2 : 0) + (b1_ ? 1 : 0)) * CWC_QB + jq_;         \
        CWC_QUAD_APPLY_MX(j_, mxl_);                                          \
        const unsigned mx1_ = (unsigned)cwc_pair_dpp_i<CWC_QSWAP1>((int)mxl_); \
        const unsigned mx2_ = mxl_ > mx1_ ? mxl_ : mx1_;                      \
        const unsigned mx3_ = (unsigned)cwc_pair_dpp_i<CWC_QSWAP2>((int)mx2_); \
        const bool ovf_ = (mx2_ > mx3_ ? mx2_ : mx3_) > p.cap;                \
        double En_ = 0.0, Un_ = 0.0;                                          \
        if ((PH) == 0) {                                                      \
            const u64 d1_ = e + 1ull + (u64)((h_ + 3) & 3);                   \
            CWC_DRAW(d1_, En_, Un_);                                          \
        }                                                                     \
        const bool slow_ = (a0_ == 0.0) | (t_next < tn_) | ovf_ |             \
                           (e + 1 == (u64)p.max_events);                      \
        if (!slow_) {                                                         \
            t = tn_; e = e + 1;                                               \
            if ((PH) == 0) CWC_QUAD_SPREAD(En_, Un_);                         \
            if (p.want_digest) dig = (dig ^ (u64)(u32)j_) * 0x100000001b3ull; \
        } else if (a0_ == 0.0) {                                              \
            CWC_QUAD_UNDO();                                                  \
            while (kn < p.K1) CWC_QEMIT();                                    \
            (st) = CWC_ST_ABSORBED;                                           \
        } else {                                                              \
            CWC_QUAD_UNDO();                                                  \
            while (t_next < tn_) CWC_QEMIT();                                 \
            if (kn >= p.K1) {                                                 \
                (st) = CWC_ST_OK;                                             \
            } else if (ovf_) {                                                \
                (st) = CWC_ST_OVERFLOW;                                       \
            } else {                                                          \
                CWC_QUAD_REDO();                                              \
                t = tn_; e = e + 1;                                           \
                if ((PH) == 0) CWC_QUAD_SPREAD(En_, Un_);                     \
                if (p.want_digest) dig = (dig ^ (u64)(u32)j_) * 0x100000001b3ull; \
                if (e == (u64)p.max_events) (st) = CWC_ST_EVENT_CAP;          \
            }                                                                 \
        }                                                                     \
    } while (0)

template <bool PERSIST, bool SHARED_K>
__device__ __forceinline__ void cwc_quad_main(const cwc_kparams &p)
{
    CWC_GROUP_LOCALS;
    CWC_QUAD_STATE;
    CWC_QUAD_DECL;
    CWC_QUAD_SETUP;
    const int h_ = (int)(__lane_id() & 3u);
    if (SHARED_K) { CWC_QUAD_LOAD_K(p.rates, h_); }
    u32 it = 0;                     // wavefront iteration (phase it % 4)
    double E0 = 0.0, U0 = 0.0, E1 = 0.0, U1 = 0.0;   // draw of the next event
    double E2 = 0.0, U2 = 0.0, E3 = 0.0, U3 = 0.0;   // of each phase
    (void)E; (void)U;

    // begin the trajectory of item `item` at phase r = it % 4: the events
    // of phases r..3 and of the next phase 0 take draws 0..4-r, drawn by the
    // lanes of those phases (lane k >= r: draw k - r; lane 0: draw 4 - r)
#define CWC_QBEGIN(item)                                                      \
    do {                                                                      \
        i64 lg0_ = (item);                                                    \
        if (p.order) {                                                        \
            const u32 grp_ = (u32)(item) / (u32)p.R;                          \
            const u32 rep_ = (u32)(item) - grp_ * (u32)p.R;                   \
            lg0_ = (i64)p.order[grp_] * p.R + rep_;                           \
        }                                                                     \
        lg = lg0_;                                                            \
        inst = (i64)((u32)lg / (u32)p.R);                                     \
        g = p.g_base + lg;                                                    \
        if (!SHARED_K) {                                                      \
            const double *kr_ = p.rates + (i64)p.rate_stride * inst;          \
            CWC_QUAD_LOAD_K(kr_, h_);                                         \
        }                                                                     \
        { const i32 *ini_ = p.init + (i64)p.init_stride * inst;               \
          CWC_QUAD_LOAD_COUNTS(ini_, h_); }                                   \
        t = 0.0; t_next = 0.0; e = 0; kn = 0;                                 \
        dig = 0xcbf29ce484222325ull;                                          \
        {                                                                     \
            const int r_ = (int)(it & 3u);                                    \
            const int d_ = h_ >= r_ ? h_ - r_ : (h_ == 0 ? 4 - r_ : 0);       \
            double Et_, Ut_;                                                  \
            CWC_DRAW((u64)d_, Et_, Ut_);                                      \
            CWC_QUAD_SPREAD(Et_, Ut_);                                        \
        }                                                                     \
    } while (0)

    // sample kn of the current state (lane 0 of the quad records it)
#define CWC_QEMIT()                                                           \
    do {                                                                      \
        CWC_GROUP_STAGE_ALL(CWC_QUAD_STAGE);                                  \
        if (h_ == 0) {                                                        \
            i32 *tr_ = CWC_TRAJ_AT(p, lg, kn);                                \
            cwc_emit_moments(p, acc, col, inst, kn, tr_);                     \
        }                                                                     \
        kn += 1;                                                              \
        t_next = (kn < p.K1) ? (double)kn * p.dt : INF;                       \
    } while (0)

    const i64 tid = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const i64 qid = tid >> 2;
    bool active = qid < p.G;
    bool live = active;
    i64 w_next = 0, w_end = 0;      // chunked claims: the wavefront's window
    if (active) CWC_QBEGIN(qid);

    // persistent form: quads whose trajectory ended take the next items
#define CWC_QPREFILL                                                          \
    if (PERSIST) {                                                            \
        const u64 want = __ballot(live && !active);                           \
        if (want) {                                                           \
            const i64 item = cwc_claim<4>(p, want, w_next, w_end);           \
            if (live && !active) {                                            \
                if (item < p.G) {                                             \
                    CWC_QBEGIN(item);                                         \
                    active = true;                                            \
                } else {                                                      \
                    live = false;                                             \
                }                                                             \
            }                                                                 \
        }                                                                     \
        if (!__any(live)) break;                                              \
    } else {                                                                  \
        if (!__any(active)) break;                                            \
    }

#define CWC_QSTEP(PH)                                                         \
    CWC_QPREFILL                                                              \
    if (active) {                                                             \
        int st = CWC_ST_RUNNING;                                              \
        CWC_QUAD_STEP_BODY(st, PH);                                           \
        if (st != CWC_ST_RUNNING) {                                           \
            CWC_GROUP_FINISH(st, CWC_QUAD_STORE_COUNTS);                      \
            active = false;                                                   \
        }                                                                     \
    }                                                                         \
    it += 1u;

    for (;;) {
        CWC_QSTEP(0)
        CWC_QSTEP(1)
        CWC_QSTEP(2)
        CWC_QSTEP(3)
    }
    cwc_acc_flush_all(p, acc);
#undef CWC_QSTEP
#undef CWC_QPREFILL
#undef CWC_QEMIT
#undef CWC_QBEGIN
}

extern "C" __global__ void __launch_bounds__(256)
cwc_quad_plain_shared(cwc_kparams p) { cwc_quad_main<false, true>(p); }
extern "C" __global__ void __launch_bounds__(256)
cwc_quad_plain_table(cwc_kparams p) { cwc_quad_main<false, false>(p); }
extern "C" __global__ void __launch_bounds__(256)
cwc_quad_persistent_shared(cwc_kparams p) { cwc_quad_main<true, true>(p); }
extern "C" __global__ void __launch_bounds__(256)
cwc_quad_persistent_table(cwc_kparams p) { cwc_quad_main<true, false>(p); }
#endif  // CWC_QUAD
