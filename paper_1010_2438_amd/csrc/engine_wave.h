// Device engine, wavefront-per-replica layout, for models whose state does
// not fit one lane (many compartments: e.g. 32 cells in an outer
// compartment).  Lane q owns compartment q: its content (nc), wrap (nw), a
// copy of its parent's content (np) and the P_local leaves of its slot block
// with their subtree; lanes beyond the model's compartments hold zeros.
// Requires engine_common.h, engine_wavelib.h and the generated model section (CWC_NS,
// CWC_PL, CWC_PC, CWC_LP, tables cwc_kind / cwc_parent / cwc_cbase /
// cwc_wbase and the macros CWC_LEAVES, CWC_LOCAL_DESCEND, CWC_APPLY, ...).
//
// One event (paper Sec. 2.3 Match / Resolve / Update), all lanes together:
//   Match    - every lane evaluates its leaves k * prod C(n, m) (Sec. 2.2)
//              and its subtree; a butterfly over the wavefront adds the
//              compartment blocks level by level (xor-partner sums are the
//              canonical tree's node = left + right, by commutativity);
//   Resolve  - the draws come in batches of 64: lane i holds draw e0 + i
//              (Philox4x32-10 keyed by seed at counter (e0 + i, g)), with
//              -ssa_log(u_tau) and u_sel precomputed; tau and the selection
//              are wavefront-uniform: the descent reads the level sums and
//              then lane b's subtree with readlane under uniform branches;
//   Update   - a scalar switch over the chosen (kind, position) applies the
//              net change in the owner lanes and in the parent copies of
//              the children, after a wavefront-wide cap check.
// Samples: every lane reduces its own cells (exact 64-bit moments).

#define CWC_NCELL_LANE (CWC_HAS_WRAP ? 2 * CWC_NS : CWC_NS)

__device__ __forceinline__ void cwc_wave_emit(const cwc_kparams &p, const i32 *col, i64 row,
                                              i32 *tr, int cb, int wb)
{
#pragma unroll 1
    for (int s = 0; s < CWC_NCELL_LANE; ++s) {
        const int cell = s < CWC_NS ? cb + s : wb + (s - CWC_NS);
        if (s >= CWC_NS && wb < 0) break;
        const i32 v = col[s * 64];
        const u64 x = (u64)(u32)v;
        const u64 q = x * x;
        atomicAdd(p.s1 + row + cell, x);
        atomicAdd(p.s2_lo32 + row + cell, q & 0xFFFFFFFFull);
        if (q >> 32) atomicAdd(p.s2_hi32 + row + cell, q >> 32);
        if (tr) tr[(i64)cell * p.G] = v;   /* [sample][cell][trajectory] */
    }
}

#define CWC_FORM_PLAIN 0
#define CWC_FORM_PERSIST 1
#define CWC_FORM_SLICE 2
#define CWC_FORM_ITEM 3

// FORM: run to completion (plain: one trajectory per wavefront of the grid;
// persistent: wavefronts claim trajectories from the queue), time-sliced
// (serving: the wavefront works on trajectory item0 of job p for at most
// `budget` draws, resuming from and suspending to a checkpoint) or one
// item of a resident kernel (as time-sliced, to the trajectory's end,
// counted toward the job by the caller).
template <int FORM, bool SHARED_K>
__device__ __forceinline__ void cwc_wave_main(const cwc_kparams &p, i64 item0, long long budget)
{
    constexpr bool SLICED = FORM == CWC_FORM_SLICE || FORM == CWC_FORM_ITEM;
    const double INF = __longlong_as_double(0x7FF0000000000000ll);
    const int lane = (int)__lane_id();
    const int wib = (int)(threadIdx.x >> 6);
    __shared__ i32 stage[4 * CWC_NCELL_LANE * 64];       // [wave][cell][lane]
    i32 *const col = stage + wib * (CWC_NCELL_LANE * 64) + lane;
    const int kind = cwc_kind[lane];          // -1: no compartment
    const int mypar = cwc_parent[lane];
    const int cb = kind >= 0 ? cwc_cbase[lane] : -1;
    const int wb = kind >= 0 ? cwc_wbase[lane] : -1;
    const int pbase = (kind >= 0 && mypar >= 0) ? cwc_cbase[mypar] : -1;
    CWC_DECL_K;
    CWC_DECL_STATE;
    if (SHARED_K) {
        if (FORM == CWC_FORM_PERSIST) {
            CWC_LOAD_K_FREE(p.rates, kind);
        } else {
            CWC_LOAD_K(p.rates, kind);
        }
    }

    i64 item = item0;
    for (;;) {
        if (item >= p.G) break;
        // ---- begin (or resume) trajectory
        i64 lg = item;
        if (p.order) {
            const u32 grp = (u32)item / (u32)p.R;
            const u32 rep = (u32)item - grp * (u32)p.R;
            lg = (i64)p.order[grp] * p.R + rep;
        }
        const i64 inst = (i64)((u32)lg / (u32)p.R);
        const i64 g = p.g_base + lg;
        if (!SHARED_K) {
            const double *kr = p.rates + (i64)p.rate_stride * inst;
            if (FORM == CWC_FORM_PERSIST) {
                CWC_LOAD_K_FREE(kr, kind);
            } else {
                CWC_LOAD_K(kr, kind);
            }
        }
        double t = 0.0, t_next = 0.0;
        u64 e = 0, e0 = 0, dig = 0xcbf29ce484222325ull;
        i32 kn = 0;
        const int cks = SLICED ? (int)p.ck_state[lg] : 0;
        if (cks == 2) break;                          // already finished
        if (cks == 1) {
            const i32 *ck = p.ck_counts + lg * (i64)CWC_C;
            CWC_LOAD_COUNTS(ck, cb, wb, pbase);
            t = p.ck_t[lg];
            e = p.ck_e[lg];
            dig = p.ck_dig[lg];
            kn = p.ck_kn[lg];
            t_next = (kn < p.K1) ? (double)kn * p.dt : INF;
        } else {
            const i32 *ini = p.init + (i64)p.init_stride * inst;
            CWC_LOAD_COUNTS(ini, cb, wb, pbase);
        }
        // a time slice of p.k_slice sample points ends before this sample
        i32 kstop = p.k_stop;
        if (SLICED && p.k_slice > 0 &&
            (long long)kn + p.k_slice < (long long)p.k_stop)
            kstop = kn + p.k_slice;
        bool have_batch = false;
        double Eb = 0.0, Ub = 0.0;          // this lane's draw of the batch
        int st = CWC_ST_RUNNING;
        long long n = 0;                    // draws in this slice

#define CWC_WEMIT()                                                           \
    do {                                                                      \
        if (kind >= 0) {                                                      \
            const i64 rw_ = (i64)(inst) * (i64)p.KR + (i64)(kn - p.k_base);  \
            const i64 row_ = rw_ * (i64)CWC_C;                                \
            i32 *tr_ = p.traj ? p.traj + (i64)(kn - p.k_base) * (i64)CWC_C * p.G + lg : (i32 *)0; \
            if (p.n_rows && lane == 0) atomicAdd(p.n_rows + rw_, 1ull);       \
            CWC_STAGE(col, 64);                                               \
            cwc_wave_emit(p, col, row_, tr_, cb, wb);                         \
        }                                                                     \
        kn += 1;                                                              \
        t_next = (kn < p.K1) ? (double)kn * p.dt : INF;                       \
    } while (0)

        while (st == CWC_ST_RUNNING) {
            if (SLICED && n == budget) break;
            ++n;
            // ---- Match: leaves, subtree, butterfly over compartment blocks
            if (FORM == CWC_FORM_PERSIST) {
                CWC_LEAVES_FREE(kind);
            } else {
                CWC_LEAVES(kind);
            }
            const double v0 = a1;
            const double v1 = CWC_LP >= 1 ? cwc_bfly_sum(v0, 1) : v0;
            const double v2 = CWC_LP >= 2 ? cwc_bfly_sum(v1, 2) : v1;
            const double v3 = CWC_LP >= 3 ? cwc_bfly_sum(v2, 3) : v2;
            const double v4 = CWC_LP >= 4 ? cwc_bfly_sum(v3, 4) : v3;
            const double v5 = CWC_LP >= 5 ? cwc_bfly_sum(v4, 5) : v4;
            const double v6 = CWC_LP >= 6 ? cwc_bfly_sum(v5, 6) : v5;
            const double a0 = cwc_rl(v6, 0);
            // ---- draws, 64 at a time
            if (!have_batch || e - e0 >= 64ull) {
                e0 = e;
                have_batch = true;
                const u64 ed = e0 + (u64)lane;
                u32 x0, x1, x2, x3;
                cwc_philox((u32)ed, (u32)(ed >> 32), (u32)g, (u32)((u64)g >> 32),
                           (u32)p.seed, (u32)(p.seed >> 32), x0, x1, x2, x3);
                Eb = -cwc_ssa_log(cwc_u_open0(x0, x1));
                Ub = cwc_u_open1(x2, x3);
            }
            const int di = (int)(e - e0);
            if (a0 == 0.0) {
                while (kn < p.K1 && kn < kstop) CWC_WEMIT();
                st = kn < p.K1 ? CWC_ST_WINDOW : CWC_ST_ABSORBED;
                break;
            }
            const double tau = cwc_rl(Eb, di) / a0;
            const double tn = t + tau;
            while (t_next < tn && kn < kstop) CWC_WEMIT();
            if (t_next < tn) {
                st = CWC_ST_WINDOW;     // the window's last sample is done
                break;
            }
            if (kn >= p.K1) {
                st = CWC_ST_OK;
                break;
            }
            // ---- selection: uniform descent over the compartment levels
            double x = cwc_rl(Ub, di) * a0;
            int base = 0;
            // level l splits the current block of 2^l lanes into halves whose
            // sums sit in the level-(l-1) butterfly values of their first lanes
            // (x >= L is bit base and R != 0 bit base + half of ballots of
            // those comparisons in every lane -- x is the same in all lanes;
            // L is read from lane base only when the descent goes right)
#define CWC_XLEVEL(l, v)                                                      \
            if (CWC_LP >= (l)) {                                              \
                const int half_ = 1 << ((l) - 1);                             \
                const u64 ge_ = __ballot(x >= (v));                           \
                const u64 nz_ = __ballot((v) != 0.0);                         \
                if (((ge_ >> base) & (nz_ >> (base + half_))) & 1ull) {       \
                    x = x - cwc_rl((v), base);                                \
                    base += half_;                                            \
                }                                                             \
            }
            CWC_XLEVEL(6, v5)
            CWC_XLEVEL(5, v4)
            CWC_XLEVEL(4, v3)
            CWC_XLEVEL(3, v2)
            CWC_XLEVEL(2, v1)
            CWC_XLEVEL(1, v0)
#undef CWC_XLEVEL
            const int b = __builtin_amdgcn_readfirstlane(base);
            int jl = 0;
            CWC_LOCAL_DESCEND(x, b, jl);
            jl = __builtin_amdgcn_readfirstlane(jl);
            const int kb = cwc_kind[b];
            const int pb = cwc_parent[b];
            bool ovf = false;
            CWC_APPLY(kb, jl, b, pb, lane, mypar, p.cap, ovf);
            if (ovf) {
                st = CWC_ST_OVERFLOW;
                break;
            }
            t = tn;
            e += 1;
            const u32 j = (u32)(b * CWC_PL + jl);
            if (p.want_digest) dig = (dig ^ (u64)j) * 0x100000001b3ull;
            if (e == (u64)p.max_events) {
                st = CWC_ST_EVENT_CAP;
                break;
            }
        }
#undef CWC_WEMIT
        if (st == CWC_ST_RUNNING || st == CWC_ST_WINDOW) {
            // ---- suspend (time-sliced form): back to the checkpoint
            i32 *ck = p.ck_counts + lg * (i64)CWC_C;
            if (kind >= 0) { CWC_STORE_COUNTS(ck, cb, wb); }
            if (lane == 0) {
                p.ck_t[lg] = t;
                p.ck_e[lg] = e;
                p.ck_dig[lg] = dig;
                p.ck_kn[lg] = kn;
                p.ck_state[lg] = 1;
            }
            break;
        }
        // ---- finish trajectory
        if (kind >= 0) {
            i32 *fc = p.final_counts + lg * (i64)CWC_C;
            CWC_STORE_COUNTS(fc, cb, wb);
        }
        if (lane == 0) {
            p.events[lg] = (i64)e;
            p.t_final[lg] = t;
            p.digest[lg] = p.want_digest ? dig : 0ull;
            p.status[lg] = (unsigned char)st;
            p.n_recorded[lg] = kn;
            if (p.rec_hist) atomicAdd(p.rec_hist + inst * (i64)(p.K1 + 1) + kn, 1ull);
            if (SLICED) p.ck_state[lg] = 2;
            if (FORM == CWC_FORM_SLICE) atomicAdd(p.done_count, 1ull);
        }
        if (FORM != CWC_FORM_PERSIST) break;
        u64 nxt = 0;
        if (lane == 0) nxt = atomicAdd(p.cursor, 1ull);
        item = (i64)__shfl(nxt, 0);
    }
}

// Resident form: wavefronts claim items (job, trajectory) from the host's
// queue and run each to its end, until the queue is closed or stays empty.
template <bool SHARED_K>
__device__ __forceinline__ void cwc_wave_resident(const cwc_kparams *jobs, const cwc_rq &q)
{
    __shared__ cwc_kparams rq_kp[4];                  // per wavefront of the block
    cwc_kparams &jp = rq_kp[threadIdx.x >> 6];
    int slot;
    i64 first, job;
    while (cwc_rq_claim(q, slot, first, job)) {
        cwc_rq_params(&jp, jobs + slot);
        cwc_wave_main<CWC_FORM_ITEM, SHARED_K>(jp, first, 0x7FFFFFFFFFFFFFFFll);
        cwc_rq_finish(q, jp, slot, job, first < jp.G ? 1u : 0u);
    }
}

__device__ __forceinline__ i64 cwc_global_wave()
{
    return ((i64)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
}

extern "C" __global__ void __launch_bounds__(256)
cwc_wave_plain_shared(cwc_kparams p)
{ cwc_wave_main<CWC_FORM_PLAIN, true>(p, cwc_global_wave(), 0); }
extern "C" __global__ void __launch_bounds__(256)
cwc_wave_plain_table(cwc_kparams p)
{ cwc_wave_main<CWC_FORM_PLAIN, false>(p, cwc_global_wave(), 0); }
extern "C" __global__ void __launch_bounds__(256)
cwc_wave_persistent_shared(cwc_kparams p)
{ cwc_wave_main<CWC_FORM_PERSIST, true>(p, cwc_global_wave(), 0); }
extern "C" __global__ void __launch_bounds__(256)
cwc_wave_persistent_table(cwc_kparams p)
{ cwc_wave_main<CWC_FORM_PERSIST, false>(p, cwc_global_wave(), 0); }
extern "C" __global__ void __launch_bounds__(256)
cwc_wave_slice_shared(const cwc_kparams *jobs, const int *wave_job, const long long *wave_first,
                      long long budget)
{
    const i64 gw = cwc_global_wave();
    cwc_wave_main<CWC_FORM_SLICE, true>(jobs[wave_job[gw]], wave_first[gw], budget);
}
extern "C" __global__ void __launch_bounds__(256)
cwc_wave_slice_table(const cwc_kparams *jobs, const int *wave_job, const long long *wave_first,
                     long long budget)
{
    const i64 gw = cwc_global_wave();
    cwc_wave_main<CWC_FORM_SLICE, false>(jobs[wave_job[gw]], wave_first[gw], budget);
}
extern "C" __global__ void __launch_bounds__(256)
cwc_wave_resident_shared(const cwc_kparams *jobs, cwc_rq q) { cwc_wave_resident<true>(jobs, q); }
extern "C" __global__ void __launch_bounds__(256)
cwc_wave_resident_table(const cwc_kparams *jobs, cwc_rq q) { cwc_wave_resident<false>(jobs, q); }
