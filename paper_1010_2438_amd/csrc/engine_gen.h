// Device engine for general CWC models (paper Sec. 2.1): compartments are
// created, dissolved and deleted while a trajectory runs, and a rule's
// pattern may reach a child and a grandchild of its context.  One
// wavefront per trajectory; lane q holds compartment slot q of the term: its
// label (-1 = free slot), its parent's slot, its wrap and content atom
// counts.  Slot 0 is the top level.  A new compartment takes the lowest free
// slot.
//
// Requires engine_common.h, engine_wavelib.h and the generated model header
// (gmodel.cpp): G_NS species, G_NL labels, G_NR rules, G_MAXC slots, G_NP
// = next power of two of G_MAXC (G_LP = log2), G_PL leaves per slot (G_LL
// = log2), G_NOBS observables, G_NINIT initial compartments, and the
// constexpr tables g_rule_at[label][position] (the rule anchored at a
// label's position, -1 none), g_depth, g_lab[rule][level], g_lhs / g_delta
// [rule][region][species] (regions: context content, child wrap, child
// content, grandchild wrap, grandchild content), g_action, g_level,
// g_new_label / g_new_wrap / g_new_content, g_release, g_has_wrap, and the
// __constant__ initial term g_init_*.
//
// One event (paper Sec. 2.3; Fig. "simd": Match, Resolve, Update):
//   Match    - every lane gathers its parent's and grandparent's label and
//              counts (lane shuffles), evaluates the G_PL leaves of its slot
//              (for each position, the rule anchored there for the lane's
//              label, if the compartments above carry the pattern's labels:
//              k * prod binomial(n, m)) and its block's subtree; a butterfly
//              over the lanes forms the slot levels of the tree;
//   Resolve  - draws batched 64 per wavefront (lane i: draw e0 + i); tau and
//              the descent are wavefront-uniform;
//   Update   - the chosen rule's atom changes in the lanes of its match,
//              then its structural action; an event whose result exceeds
//              the count cap or needs a slot the pool does not have is not
//              applied (OVERFLOW).
// Samples: per label, the content and wrap atom totals of its live
// compartments and their number (wavefront sums), reduced on line into
// exact moments.

#define G_W (3 + 2 * G_NS)          // final-term row: alive, label, parent, wrap, content

__device__ __forceinline__ u64 gen_binom(int n, int m)
{
    if (m == 0) return 1ull;
    if (n < m) return 0ull;
    if (m == 1) return (u64)(u32)n;
    return (u64)(u32)n * (u64)(u32)(n - 1) / 2ull;        // m == 2
}

// wavefront sum of a non-negative int count (64-bit)
__device__ __forceinline__ long long gen_wave_sum(int v)
{
    long long s = (long long)v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int lo = __shfl_xor((int)s, off);
        const int hi = __shfl_xor((int)(s >> 32), off);
        s += ((long long)hi << 32) | (long long)(unsigned)lo;
    }
    return s;
}

struct GenLane {
    int lab, par;
    int c[G_NS], w[G_NS];
};

// The counts of the compartments above a lane, gathered for the patterns.
struct GenAbove {
    int plab, glab;                 // -2: no such compartment
    int pc[G_NS], pw[G_NS], gc[G_NS];
};

__device__ __forceinline__ void gen_gather(const GenLane &s, GenAbove &u, int lane)
{
    const int pl = s.par >= 0 ? s.par : lane;
    const int pp = __shfl(s.par, pl);
    const int gl = (s.par >= 0 && pp >= 0) ? pp : lane;
    const int plab = __shfl(s.lab, pl);
    const int glab = __shfl(s.lab, gl);
    u.plab = s.par >= 0 ? plab : -2;
    u.glab = (s.par >= 0 && pp >= 0) ? glab : -2;
#pragma unroll
    for (int a = 0; a < G_NS; ++a) {
        u.pc[a] = __shfl(s.c[a], pl);
        u.pw[a] = __shfl(s.w[a], pl);
        u.gc[a] = __shfl(s.c[a], gl);
    }
}

// Rate of rule R anchored at this lane (0 if the pattern's labels do not
// match the compartments above): k * prod over regions and atoms of
// binomial(n, m), the integer product exact, one rounding.
template <int R>
__device__ __forceinline__ double gen_rate(const GenLane &s, const GenAbove &u, double k)
{
    constexpr int d = g_depth[R];
    bool ok = s.lab == g_lab[R][d];
    if constexpr (d >= 1) ok = ok && u.plab == g_lab[R][d - 1];
    if constexpr (d >= 2) ok = ok && u.glab == g_lab[R][0];
    u64 h = 1ull;
#pragma unroll
    for (int a = 0; a < G_NS; ++a) {
        // region counts of the match, seen from its anchor (this lane)
        const int r0 = d == 0 ? s.c[a] : (d == 1 ? u.pc[a] : u.gc[a]);
        const int r1 = d == 1 ? s.w[a] : u.pw[a];
        const int r2 = d == 1 ? s.c[a] : u.pc[a];
        if (g_lhs[R][0][a]) h *= gen_binom(r0, g_lhs[R][0][a]);
        if (d >= 1 && g_lhs[R][1][a]) h *= gen_binom(r1, g_lhs[R][1][a]);
        if (d >= 1 && g_lhs[R][2][a]) h *= gen_binom(r2, g_lhs[R][2][a]);
        if (d >= 2 && g_lhs[R][3][a]) h *= gen_binom(s.w[a], g_lhs[R][3][a]);
        if (d >= 2 && g_lhs[R][4][a]) h *= gen_binom(s.c[a], g_lhs[R][4][a]);
    }
    return ok ? k * (double)h : 0.0;
}

// Leaf of position P: the rule anchored at P for the lane's label, over the
// labels (at most one matches; a free slot matches none).
template <int P, int L>
__device__ __forceinline__ double gen_leaf_lab(const GenLane &s, const GenAbove &u,
                                               const double *k)
{
    if constexpr (L >= G_NL) {
        return 0.0;
    } else {
        constexpr int r = g_rule_at[L][P];
        const double rest = gen_leaf_lab<P, L + 1>(s, u, k);
        if constexpr (r < 0) {
            return rest;
        } else {
            return s.lab == L ? gen_rate<r>(s, u, k[r]) : rest;
        }
    }
}

template <int P>
__device__ __forceinline__ void gen_leaves(const GenLane &s, const GenAbove &u, const double *k,
                                           double *a)
{
    if constexpr (P < G_PL) {
        a[G_PL + P] = gen_leaf_lab<P, 0>(s, u, k);
        gen_leaves<P + 1>(s, u, k, a);
    }
}

// descent inside slot b's block from node I: x is the same in every lane;
// "x >= L" and "R != 0" in lane b are bits b of ballots; L is read from
// lane b when the descent goes right
template <int I>
__device__ __forceinline__ int gen_local_descend(double &x, int b, const double *a)
{
    if constexpr (I >= G_PL) {
        return I - G_PL;
    } else {
        const u64 ge = __ballot(x >= a[2 * I]);
        const u64 nz = __ballot(a[2 * I + 1] != 0.0);
        if (((ge & nz) >> b) & 1ull) {
            x = x - cwc_rl(a[2 * I], b);
            return gen_local_descend<2 * I + 1>(x, b, a);
        }
        return gen_local_descend<2 * I>(x, b, a);
    }
}

// Update by rule R at the match whose anchor is lane b: atom changes, then
// the structural action.  Returns true (state kept) if the result would
// exceed the cap or needs a free slot the pool does not have.
template <int R>
__device__ __forceinline__ bool gen_apply(GenLane &s, int lane, int b, unsigned cap)
{
    constexpr int d = g_depth[R];
    int L[3] = {b, b, b};
    if constexpr (d >= 1) L[d - 1] = __builtin_amdgcn_readlane(s.par, L[d]);
    if constexpr (d >= 2) L[0] = __builtin_amdgcn_readlane(s.par, L[1]);
    GenLane n = s;
#pragma unroll
    for (int a = 0; a < G_NS; ++a) {
        if (lane == L[0]) n.c[a] += g_delta[R][0][a];
        if (d >= 1 && lane == L[1]) {
            n.w[a] += g_delta[R][1][a];
            n.c[a] += g_delta[R][2][a];
        }
        if (d >= 2 && lane == L[2]) {
            n.w[a] += g_delta[R][3][a];
            n.c[a] += g_delta[R][4][a];
        }
    }
    constexpr int act = g_action[R];
    constexpr int lv = g_level[R];
    if constexpr (act == GEN_CREATE) {
        const u64 free_ = __ballot(s.lab < 0 && lane >= 1 && lane < G_MAXC);
        if (!free_) return true;                      // no free slot
        const int z = __ffsll((long long)free_) - 1;  // the lowest
        if (lane == z) {
            n.lab = g_new_label[R];
            n.par = L[lv];
#pragma unroll
            for (int a = 0; a < G_NS; ++a) {
                n.w[a] = g_new_wrap[R][a];
                n.c[a] = g_new_content[R][a];
            }
        }
    } else if constexpr (act == GEN_DISSOLVE) {
        const int z = L[lv], pz = L[lv - 1];
#pragma unroll
        for (int a = 0; a < G_NS; ++a) {
            int add = __builtin_amdgcn_readlane(n.c[a], z);
            if constexpr (g_release[R] != 0) add += __builtin_amdgcn_readlane(n.w[a], z);
            if (lane == pz) n.c[a] += add;
        }
        if (n.par == z) n.par = pz;                   // its compartments move up
        if (lane == z) {
            n.lab = -1;
            n.par = -1;
#pragma unroll
            for (int a = 0; a < G_NS; ++a) n.c[a] = n.w[a] = 0;
        }
    } else if constexpr (act == GEN_DELETE) {
        const int z = L[lv];
        bool gone = lane == z;
        // close under "the parent is gone" (at most one level per pass)
        for (int it = 0; it < 64; ++it) {
            const u64 before = __ballot(gone);
            const int src = n.par >= 0 ? n.par : lane;
            const bool pg = __shfl((int)gone, src) != 0;
            gone = gone || (n.lab >= 0 && n.par >= 0 && pg);
            if (__ballot(gone) == before) break;
        }
        if (gone) {
            n.lab = -1;
            n.par = -1;
#pragma unroll
            for (int a = 0; a < G_NS; ++a) n.c[a] = n.w[a] = 0;
        }
    }
    bool bad = false;
    if (n.lab >= 0) {
#pragma unroll
        for (int a = 0; a < G_NS; ++a)
            bad = bad || (unsigned)n.c[a] > cap || (unsigned)n.w[a] > cap;
    }
    if (__any(bad)) return true;
    s = n;
    return false;
}

template <int R>
__device__ __forceinline__ bool gen_apply_rule(int r, GenLane &s, int lane, int b, unsigned cap)
{
    if constexpr (R >= G_NR) {
        return false;
    } else {
        if (r == R) return gen_apply<R>(s, lane, b, cap);
        return gen_apply_rule<R + 1>(r, s, lane, b, cap);
    }
}

// Observables of the term, the same in every lane: per label the content
// atom totals, the wrap atom totals (labels with a wrap), the number of
// live compartments; each total is taken as an int32 (as stored).
__device__ __forceinline__ void gen_observe(const GenLane &s, int *obs)
{
    int o = 0;
#pragma unroll
    for (int l = 0; l < G_NL; ++l) {
        const bool mine = s.lab == l;
#pragma unroll
        for (int a = 0; a < G_NS; ++a) obs[o++] = (int)gen_wave_sum(mine ? s.c[a] : 0);
        if (g_has_wrap[l]) {
#pragma unroll
            for (int a = 0; a < G_NS; ++a) obs[o++] = (int)gen_wave_sum(mine ? s.w[a] : 0);
        }
        obs[o++] = (int)gen_wave_sum(mine ? 1 : 0);
    }
}

#define G_FORM_PLAIN 0
#define G_FORM_PERSIST 1
#define G_FORM_SLICE 2
#define G_FORM_ITEM 3

// FORM: run to completion (plain: one trajectory per wavefront of the grid;
// persistent: wavefronts claim trajectories from the queue), time-sliced
// (streamed runs and serving: the wavefront works on trajectory item0 of
// job p for at most `budget` draws and before the slice's stop sample,
// resuming from and suspending to a checkpoint: the term in final_term,
// the time, event count, digest and next sample in ck_*) or one item of a
// resident kernel (as time-sliced, to the trajectory's end, counted toward
// the job by the caller).
template <int FORM, bool SHARED_K>
__device__ __forceinline__ void cwc_gen_main(const cwc_kparams &p, i64 item0, long long budget)
{
    constexpr bool SLICED = FORM == G_FORM_SLICE || FORM == G_FORM_ITEM;
    const double INF = __longlong_as_double(0x7FF0000000000000ll);
    const int lane = (int)__lane_id();
    double k[G_NR > 0 ? G_NR : 1];
    if (SHARED_K) {
#pragma unroll
        for (int r = 0; r < G_NR; ++r) k[r] = p.rates[r];
    }
    i64 item = item0;
    for (;;) {
        if (item >= p.G) break;
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
#pragma unroll
            for (int r = 0; r < G_NR; ++r) k[r] = kr[r];
        }
        const int cks = SLICED ? (int)p.ck_state[lg] : 0;
        if (cks == 2) break;                          // already finished
        GenLane s;
        double t = 0.0, t_next = 0.0;
        u64 e = 0, e0 = 0, dig = 0xcbf29ce484222325ull;
        i32 kn = 0;
        if (cks == 1) {
            // resume: the term and the scalars saved at the last suspension
            const bool in_ = lane < G_MAXC;
            const int *row = p.final_term + (lg * G_MAXC + (in_ ? lane : 0)) * (i64)G_W;
            s.lab = in_ ? row[1] : -1;
            s.par = in_ ? row[2] : -1;
#pragma unroll
            for (int a = 0; a < G_NS; ++a) {
                s.w[a] = in_ ? row[3 + a] : 0;
                s.c[a] = in_ ? row[3 + G_NS + a] : 0;
            }
            t = p.ck_t[lg];
            e = p.ck_e[lg];
            dig = p.ck_dig[lg];
            kn = p.ck_kn[lg];
            t_next = (kn < p.K1) ? (double)kn * p.dt : INF;
        } else {
            // the initial term
            const bool init_ = lane < G_NINIT;
            const int il = init_ ? lane : 0;      // every table read in bounds
            s.lab = init_ ? g_init_label[il] : -1;
            s.par = init_ ? g_init_parent[il] : -1;
#pragma unroll
            for (int a = 0; a < G_NS; ++a) {
                s.c[a] = init_ ? g_init_content[il * G_NS + a] : 0;
                s.w[a] = init_ ? g_init_wrap[il * G_NS + a] : 0;
            }
        }
        // the slice stops before this sample (streamed windows, sample
        // slices); the run-to-completion forms never stop early
        i32 kstop = 0x7FFFFFFF;
        if (SLICED) {
            kstop = p.k_stop;
            if (p.k_slice > 0 && (long long)kn + p.k_slice < (long long)p.k_stop)
                kstop = kn + p.k_slice;
        }
        bool have_batch = false;
        double Eb = 0.0, Ub = 0.0;
        int st = CWC_ST_RUNNING;
        long long n = 0;                    // draws in this slice
        int obs[G_NOBS];

#define GEN_EMIT()                                                            \
    do {                                                                      \
        gen_observe(s, obs);                                                  \
        if (lane == 0) {                                                      \
            const i64 row_ = ((i64)inst * p.KR + (kn - p.k_base)) * (i64)G_NOBS; \
            _Pragma("unroll")                                                 \
            for (int o_ = 0; o_ < G_NOBS; ++o_) {                             \
                const u64 x_ = (u64)(u32)obs[o_];                             \
                const u64 q_ = x_ * x_;                                       \
                atomicAdd(p.s1 + row_ + o_, x_);                              \
                atomicAdd(p.s2_lo32 + row_ + o_, q_ & 0xFFFFFFFFull);         \
                if (q_ >> 32) atomicAdd(p.s2_hi32 + row_ + o_, q_ >> 32);     \
                if (p.traj)                                                   \
                    p.traj[((i64)(kn - p.k_base) * G_NOBS + o_) * p.G + lg] = obs[o_]; \
            }                                                                 \
            if (p.n_rows) atomicAdd(p.n_rows + (i64)inst * p.KR + (kn - p.k_base), 1ull); \
        }                                                                     \
        kn += 1;                                                              \
        t_next = (kn < p.K1) ? (double)kn * p.dt : INF;                       \
    } while (0)

        while (st == CWC_ST_RUNNING) {
            if (SLICED && n == budget) break;
            ++n;
            // ---- Match
            GenAbove u;
            gen_gather(s, u, lane);
            double a[2 * G_PL];
            gen_leaves<0>(s, u, k, a);
#pragma unroll
            for (int i = G_PL - 1; i >= 1; --i) a[i] = a[2 * i] + a[2 * i + 1];
            double v[G_LP + 1];
            v[0] = a[1];
#pragma unroll
            for (int l = 1; l <= G_LP; ++l) v[l] = cwc_bfly_sum(v[l - 1], l);
            const double a0 = cwc_rl(v[G_LP], 0);
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
            // (the stop sample exists in the sliced forms only: the
            // run-to-completion forms keep the loops without it)
            if (a0 == 0.0) {
                while (kn < p.K1 && (!SLICED || kn < kstop)) GEN_EMIT();
                st = kn < p.K1 ? CWC_ST_WINDOW : CWC_ST_ABSORBED;
                break;
            }
            const double tn = t + cwc_rl(Eb, di) / a0;
            while (t_next < tn && (!SLICED || kn < kstop)) GEN_EMIT();
            if (SLICED && t_next < tn) {
                st = CWC_ST_WINDOW;     // the slice's last sample is done
                break;
            }
            if (kn >= p.K1) {
                st = CWC_ST_OK;
                break;
            }
            // ---- Resolve: slot levels, then the slot's block
            double x = cwc_rl(Ub, di) * a0;
            int base = 0;
#pragma unroll
            for (int l = G_LP; l >= 1; --l) {
                const int half = 1 << (l - 1);
                const u64 ge = __ballot(x >= v[l - 1]);
                const u64 nz = __ballot(v[l - 1] != 0.0);
                if (((ge >> base) & (nz >> (base + half))) & 1ull) {
                    x = x - cwc_rl(v[l - 1], base);
                    base += half;
                }
            }
            const int b = __builtin_amdgcn_readfirstlane(base);
            const int jl = __builtin_amdgcn_readfirstlane(gen_local_descend<1>(x, b, a));
            const int lab_b = __builtin_amdgcn_readlane(s.lab, b);
            int r = -1;
#pragma unroll
            for (int l = 0; l < G_NL; ++l)
#pragma unroll
                for (int q = 0; q < G_PL; ++q)
                    if (l == lab_b && q == jl) r = g_rule_at[l][q];
            // ---- Update
            if (gen_apply_rule<0>(r, s, lane, b, p.cap)) {
                st = CWC_ST_OVERFLOW;
                break;
            }
            t = tn;
            e += 1;
            const u32 j = (u32)(b * G_PL + jl);
            if (p.want_digest) dig = (dig ^ (u64)j) * 0x100000001b3ull;
            if (e == (u64)p.max_events) {
                st = CWC_ST_EVENT_CAP;
                break;
            }
        }
#undef GEN_EMIT
        if (SLICED && (st == CWC_ST_RUNNING || st == CWC_ST_WINDOW)) {
            // ---- suspend: the term and the scalars back to the checkpoint
            if (lane < G_MAXC) {
                int *row = p.final_term + (lg * G_MAXC + lane) * (i64)G_W;
                row[0] = s.lab >= 0 ? 1 : 0;
                row[1] = s.lab;
                row[2] = s.par;
#pragma unroll
                for (int a2 = 0; a2 < G_NS; ++a2) {
                    row[3 + a2] = s.w[a2];
                    row[3 + G_NS + a2] = s.c[a2];
                }
            }
            if (lane == 0) {
                p.ck_t[lg] = t;
                p.ck_e[lg] = e;
                p.ck_dig[lg] = dig;
                p.ck_kn[lg] = kn;
                p.ck_state[lg] = 1;
            }
            break;
        }
        // ---- finish: observables, per-trajectory results, final term
        gen_observe(s, obs);
        if (lane == 0) {
            int *fc = p.final_counts + lg * (i64)G_NOBS;
#pragma unroll
            for (int o = 0; o < G_NOBS; ++o) fc[o] = obs[o];
            p.events[lg] = (i64)e;
            p.t_final[lg] = t;
            p.digest[lg] = p.want_digest ? dig : 0ull;
            p.status[lg] = (unsigned char)st;
            p.n_recorded[lg] = kn;
            if (p.rec_hist) atomicAdd(p.rec_hist + inst * (i64)(p.K1 + 1) + kn, 1ull);
            if (SLICED) p.ck_state[lg] = 2;
            if (FORM == G_FORM_SLICE) atomicAdd(p.done_count, 1ull);
        }
        if (p.final_term && lane < G_MAXC) {
            int *row = p.final_term + (lg * G_MAXC + lane) * (i64)G_W;
            row[0] = s.lab >= 0 ? 1 : 0;
            row[1] = s.lab;
            row[2] = s.par;
#pragma unroll
            for (int a2 = 0; a2 < G_NS; ++a2) {
                row[3 + a2] = s.w[a2];
                row[3 + G_NS + a2] = s.c[a2];
            }
        }
        if (FORM != G_FORM_PERSIST) break;
        u64 nxt = 0;
        if (lane == 0) nxt = atomicAdd(p.cursor, 1ull);
        item = (i64)__shfl((long long)nxt, 0);
    }
}

// Resident form: wavefronts claim items (job, trajectory) from the host's
// queue and run each to its end, until the queue is closed or stays empty.
template <bool SHARED_K>
__device__ __forceinline__ void cwc_gen_resident(const cwc_kparams *jobs, const cwc_rq &q)
{
    __shared__ cwc_kparams rq_kp[4];                  // per wavefront of the block
    cwc_kparams &jp = rq_kp[threadIdx.x >> 6];
    int slot;
    i64 first, job;
    while (cwc_rq_claim(q, slot, first, job)) {
        cwc_rq_params(&jp, jobs + slot);
        cwc_gen_main<G_FORM_ITEM, SHARED_K>(jp, first, 0x7FFFFFFFFFFFFFFFll);
        cwc_rq_finish(q, jp, slot, job, first < jp.G ? 1u : 0u);
    }
}

__device__ __forceinline__ i64 gen_global_wave()
{
    return __builtin_amdgcn_readfirstlane((int)(((i64)blockIdx.x * blockDim.x + threadIdx.x) >> 6));
}

extern "C" __global__ void __launch_bounds__(256)
cwc_gen_plain_shared(cwc_kparams p) { cwc_gen_main<G_FORM_PLAIN, true>(p, gen_global_wave(), 0); }
extern "C" __global__ void __launch_bounds__(256)
cwc_gen_plain_table(cwc_kparams p) { cwc_gen_main<G_FORM_PLAIN, false>(p, gen_global_wave(), 0); }
extern "C" __global__ void __launch_bounds__(256)
cwc_gen_persistent_shared(cwc_kparams p)
{ cwc_gen_main<G_FORM_PERSIST, true>(p, gen_global_wave(), 0); }
extern "C" __global__ void __launch_bounds__(256)
cwc_gen_persistent_table(cwc_kparams p)
{ cwc_gen_main<G_FORM_PERSIST, false>(p, gen_global_wave(), 0); }
extern "C" __global__ void __launch_bounds__(256)
cwc_gen_slice_shared(const cwc_kparams *jobs, const int *wave_job, const long long *wave_first,
                     long long budget)
{
    const i64 gw = gen_global_wave();
    cwc_gen_main<G_FORM_SLICE, true>(jobs[wave_job[gw]], wave_first[gw], budget);
}
extern "C" __global__ void __launch_bounds__(256)
cwc_gen_slice_table(const cwc_kparams *jobs, const int *wave_job, const long long *wave_first,
                    long long budget)
{
    const i64 gw = gen_global_wave();
    cwc_gen_main<G_FORM_SLICE, false>(jobs[wave_job[gw]], wave_first[gw], budget);
}
extern "C" __global__ void __launch_bounds__(256)
cwc_gen_resident_shared(const cwc_kparams *jobs, cwc_rq q) { cwc_gen_resident<true>(jobs, q); }
extern "C" __global__ void __launch_bounds__(256)
cwc_gen_resident_table(const cwc_kparams *jobs, cwc_rq q) { cwc_gen_resident<false>(jobs, q); }
