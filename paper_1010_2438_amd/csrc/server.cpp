// Serving: continuous batching of simulation jobs on one device.
//
// The paper's schema ii (Sec. 5.2) makes each simulation instance an object
// that can be stopped and restarted so that an on-line scheduler can
// time-slice instances across workers.  Here the scheduler is a host thread
// and the "workers" are four device streams, each running one slice launch
// at a time:
//   admit:    queued jobs (FIFO) while a job slot and pool memory are free;
//   launch:   a stream without work takes the ready jobs of one model group
//             (model, layout, rate-table use), up to about half a device of
//             wavefronts, and advances each of their unfinished trajectories
//             by at most slice_events draws, suspending the rest to a device
//             checkpoint;
//   complete: when a stream's slice has finished, its jobs' finished-
//             trajectory counters are read; jobs whose trajectories have all
//             finished get their statistics finalised and leave their slot,
//             the others are ready for another slice.
// Streams run independently, so a model whose slices are slow does not hold
// up the others, and the device keeps up to four slices in flight.  A
// trajectory's events do not depend on how it was sliced or which jobs
// shared a launch (counter-based random stream), so every job is
// bit-identical to the same run submitted alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/cwcssa.h"
#include "runtime.h"
#include "stats.h"

using namespace cwc;

namespace {

constexpr int kStreams = 4;
// resident mode: streams for resident kernels, created on first use (each,
// like every stream of the server, with a hardware queue of its own, since
// a resident kernel holds its queue until it leaves)
constexpr int kRStreams = 8;
// launches of at most this many trajectories use two lanes per trajectory
constexpr long long kPairSliceMax = 32768;

// First-fit sub-allocator over the server's device pool.
struct Pool {
    char *base = nullptr;
    size_t bytes = 0, used = 0, peak = 0;
    std::map<size_t, size_t> free_blocks;   // offset -> size
    std::map<size_t, size_t> live;          // offset -> size

    void init(void *p, size_t n)
    {
        base = (char *)p;
        bytes = n & ~size_t(255);
        free_blocks.clear();
        free_blocks[0] = bytes;
    }
    void *alloc(size_t n)
    {
        n = std::max<size_t>(256, (n + 255) & ~size_t(255));
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second < n) continue;
            size_t off = it->first, sz = it->second;
            free_blocks.erase(it);
            if (sz > n) free_blocks[off + n] = sz - n;
            live[off] = n;
            used += n;
            return base + off;
        }
        return nullptr;
    }
    void release(void *p)
    {
        size_t off = (char *)p - base;
        auto it = live.find(off);
        if (it == live.end()) return;
        size_t n = it->second;
        live.erase(it);
        used -= n;
        auto nx = free_blocks.lower_bound(off);
        if (nx != free_blocks.end() && off + n == nx->first) {
            n += nx->second;
            nx = free_blocks.erase(nx);
        }
        if (nx != free_blocks.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += n;
                return;
            }
        }
        free_blocks[off] = n;
    }
};

size_t rounded(size_t n) { return std::max<size_t>(256, (n + 255) & ~size_t(255)); }

struct Job {
    uint64_t id = 0;
    cwc_model *m = nullptr;
    int layout = 0;
    bool shared_k = true;
    long long I = 0, R = 0, G = 0;
    int K1 = 0, C = 0, NR = 1;
    long long term_ints = 0;          // general models: the terms [G][slots][row]
    int group = -1;                   // resident mode: the job's queue
    cwc_run_desc d{};
    std::vector<double> rates;
    std::vector<int> init;
    cwc_kparams kp{};
    long long *nk = nullptr;
    double *mean = nullptr, *var = nullptr;
    std::vector<void *> bufs;
    size_t bytes = 0;
    int state = CWC_JOB_QUEUED;
    int slot = -1;
    int n_ticks = 0;
    // history for the predictive policy: slices taken, their wall time, and
    // sample points done (exact with time slices: every unfinished
    // trajectory advances by the slice's sample points)
    int k_slice = 0;
    int samples_done = 0;
    double slice_wall = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    long long events = 0;
};

// Device bytes a job holds while admitted (same list as admit()).
size_t job_bytes(const Job &j)
{
    const size_t G = j.G, C = j.C, mom = (size_t)j.I * j.K1 * j.C, I = j.I, K1 = j.K1;
    size_t b = 0;
    b += rounded(j.rates.size() * 8) + rounded(j.init.size() * 4);
    b += rounded(G * C * 4) * 2;                                         // final, checkpoint counts
    b += rounded(G * 8) * 6;                                             // events t digest ck_t ck_e ck_dig
    b += rounded(G) * 2 + rounded(G * 4) * 2;                            // status ck_state, n_rec ck_kn
    b += rounded(mom * 8) * 5;                                           // s1 s2hi s2lo mean var
    b += rounded(I * (K1 + 1) * 8) + rounded(I * K1 * 8);                // hist, n
    if (j.term_ints) b += rounded((size_t)j.term_ints * 4);              // terms (checkpoint)
    return b;
}

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Resident mode: the item queue of one model group (model, layout,
// rate-table use).  Items are published into a ring in coherent host
// memory and claimed by the group's resident kernels through a device
// counter.
constexpr long long kRingItems = 1ll << 18;
struct RGroup {
    cwc_model *m = nullptr;
    int layout = 0;
    bool shared_k = true;
    bool pair = false;
    hipFunction_t fn = nullptr;
    long long per_wave = 64;               // trajectories per item
    int wpb = 4;                           // wavefronts per block
    unsigned lds = 0;
    long long *h_items = nullptr;          // [kRingItems][CWC_RQ_ITEM], coherent host memory
    long long *h_tail = nullptr;           // [1] items published, coherent host memory
    long long *dv_items = nullptr;         // the kernels' addresses of the two
    long long *dv_tail = nullptr;
    unsigned long long *d_head = nullptr;  // [1] items claimed (device)
    long long published = 0;
    long long claimed = 0;                 // last value read back
    double t_unclaimed = -1.0;             // since when items have waited unclaimed
};

}  // namespace

struct cwc_server {
    cwc_ctx *ctx = nullptr;
    void *pool_mem = nullptr;
    Pool pool;
    int max_active = 0;
    long long slice = 0;
    int slice_samples = 0;                   // guarded by mu (read at admission)
    int policy = CWC_SCHED_FIFO;             // guarded by mu
    std::chrono::steady_clock::time_point t0;
    std::thread th;
    std::mutex mu;                       // guards everything below
    std::condition_variable cv, idle_cv;
    bool stop = false;
    std::string error;
    uint64_t next_id = 1;
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    std::vector<uint64_t> unreported;
    std::vector<Job *> active;
    std::vector<int> free_slots;
    cwc_server_stats stats{};
    // device side (scheduler thread only)
    cwc_kparams *d_jobs = nullptr;           // [max_active]
    unsigned long long *d_done = nullptr;    // [max_active]
    hipStream_t streams[kStreams] = {};
    hipStream_t aux = nullptr;
    hipStream_t fetch = nullptr;             // result copies of client calls
    std::mutex fetch_mu;                     // one client copy at a time on it
    int *d_wave_job[kStreams] = {};
    long long *d_wave_first[kStreams] = {};
    size_t wave_cap[kStreams] = {};
    std::vector<int> h_wave_job[kStreams];         // tables of the slice in flight
    std::vector<long long> h_wave_first[kStreams];
    hipEvent_t ev_slice[kStreams] = {};           // end of each stream's slice
    double t_slice[kStreams] = {};                 // launch time of each stream's slice
    // resident mode (scheduler thread only, after creation): one item queue
    // per model group; flags shared with the kernels in coherent host memory
    std::vector<std::unique_ptr<RGroup>> groups;
    hipStream_t rstreams[kRStreams] = {};          // resident kernels' streams
    hipEvent_t ev_res[kRStreams] = {};             // end of each stream's kernel
    int rkern[kRStreams] = {-1, -1, -1, -1, -1, -1, -1, -1};  // group of each stream's kernel
    int *h_stop = nullptr;                         // [1] close every queue
    long long *h_done = nullptr;                   // [max_active] completed job ids by slot
    int *dv_stop = nullptr;                        // the kernels' addresses of the two
    long long *dv_done = nullptr;
    long long idle_ticks = 0;                      // wall-clock ticks of 2 ms
    std::vector<long long> h_head;                 // read-back buffer for claim counters
};

namespace {

void fail_locked(cwc_server *s, const std::string &msg)
{
    if (s->error.empty()) s->error = msg;
}

#define SCHK(call)                                                                  \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            std::lock_guard<std::mutex> lk_(s->mu);                                 \
            fail_locked(s, std::string(#call) + ": " + hipGetErrorString(e_));      \
            return false;                                                           \
        }                                                                           \
    } while (0)

template <class T>
bool take(cwc_server *s, Job *j, T **p, size_t count)
{
    void *q = s->pool.alloc(std::max<size_t>(1, count) * sizeof(T));
    if (!q) return false;
    j->bufs.push_back(q);
    *p = (T *)q;
    return true;
}

void drop(cwc_server *s, Job *j)
{
    for (void *p : j->bufs) s->pool.release(p);
    j->bufs.clear();
}

// Reserves an admitted job's device buffers in the pool (mutex held).
// Returns false (nothing held) if the pool is too full right now.
bool reserve(cwc_server *s, Job *j)
{
    if (s->pool.bytes - s->pool.used < job_bytes(*j)) return false;
    cwc_kparams &kp = j->kp;
    std::memset(&kp, 0, sizeof kp);
    const long long G = j->G, mom = j->I * (long long)j->K1 * j->C;
    double *d_rates = nullptr;
    int *d_init = nullptr;
    bool ok = take(s, j, &d_rates, j->rates.size()) && take(s, j, &d_init, j->init.size()) &&
              take(s, j, &kp.final_counts, G * j->C) && take(s, j, &kp.ck_counts, G * j->C) &&
              take(s, j, &kp.events, G) && take(s, j, &kp.t_final, G) &&
              take(s, j, &kp.digest, G) && take(s, j, &kp.ck_t, G) && take(s, j, &kp.ck_e, G) &&
              take(s, j, &kp.ck_dig, G) && take(s, j, &kp.status, G) &&
              take(s, j, &kp.ck_state, G) && take(s, j, &kp.n_recorded, G) &&
              take(s, j, &kp.ck_kn, G) && take(s, j, &kp.s1, mom) &&
              take(s, j, &kp.s2_hi32, mom) && take(s, j, &kp.s2_lo32, mom) &&
              take(s, j, &j->mean, mom) && take(s, j, &j->var, mom) &&
              take(s, j, &kp.rec_hist, j->I * (long long)(j->K1 + 1)) &&
              take(s, j, &j->nk, j->I * (long long)j->K1) &&
              (!j->term_ints || take(s, j, &kp.final_term, j->term_ints));
    if (!ok) {
        drop(s, j);
        return false;
    }
    kp.rates = d_rates;
    kp.init = d_init;
    j->bytes = 0;
    for (void *p : j->bufs) j->bytes += s->pool.live[(char *)p - s->pool.base];
    s->pool.peak = std::max(s->pool.peak, s->pool.used);   // committed reservations only
    return true;
}

// Uploads tables, zeroes accumulators and checkpoint states and publishes
// the job's parameters in its slot (scheduler thread, mutex not held).
bool init_job(cwc_server *s, Job *j, int slot)
{
    cwc_kparams &kp = j->kp;
    const long long G = j->G, mom = j->I * (long long)j->K1 * j->C;
    kp.seed = j->d.seed;
    kp.G = G;
    kp.R = j->R;
    kp.g_base = 0;
    kp.max_events = j->d.max_events;
    kp.dt = j->d.dt;
    kp.K1 = j->K1;
    kp.KR = kp.K1;          // one accumulator row per sample
    kp.k_base = 0;
    kp.k_stop = 0x7FFFFFFF; // no window: trajectories run to the horizon
    kp.k_slice = j->k_slice;            // 0: slices bounded by draws only
    kp.n_rows = nullptr;
    kp.cap = (unsigned)j->d.count_cap;
    kp.rate_stride = j->shared_k ? 0 : j->NR;
    kp.init_stride = j->d.init_table ? j->C : 0;
    kp.want_traj = 0;
    kp.want_digest = j->d.want_digest ? 1 : 0;
    kp.done_count = s->d_done + slot;
    kp.nslot = kDefaultSampleSlots;
    kp.chunk = 1;
    hipStream_t a = s->aux;
    SCHK(hipMemcpyAsync((void *)kp.rates, j->rates.data(), j->rates.size() * 8,
                        hipMemcpyHostToDevice, a));
    SCHK(hipMemcpyAsync((void *)kp.init, j->init.data(), j->init.size() * 4,
                        hipMemcpyHostToDevice, a));
    SCHK(launch_fill_u64(kp.s1, 0, mom, a));
    SCHK(launch_fill_u64(kp.s2_hi32, 0, mom, a));
    SCHK(launch_fill_u64(kp.s2_lo32, 0, mom, a));
    SCHK(launch_fill_u64(kp.rec_hist, 0, j->I * (long long)(j->K1 + 1), a));
    SCHK(launch_fill_u64((unsigned long long *)kp.ck_state, 0, (G + 7) / 8, a));
    SCHK(launch_fill_u64(kp.done_count, 0, 1, a));
    SCHK(hipMemcpyAsync(s->d_jobs + slot, &kp, sizeof kp, hipMemcpyHostToDevice, a));
    SCHK(hipStreamSynchronize(a));
    j->slot = slot;
    return true;
}

// Launches one slice over `jobs` (all of one model group) on stream `si`
// (scheduler thread, mutex not held); the stream's table buffers are free
// because the stream has no work in flight.
bool launch_slice(cwc_server *s, int si, const std::vector<Job *> &jobs)
{
    std::vector<int> &wave_job = s->h_wave_job[si];
    std::vector<long long> &wave_first = s->h_wave_first[si];
    wave_job.clear();
    wave_first.clear();
    const Job *j0 = jobs.front();
    // a lane-layout launch that leaves most lanes idle runs two lanes per
    // trajectory (shorter per-trajectory latency), when the model has them
    long long traj = 0;
    for (Job *j : jobs) traj += j->G;
    const bool pair = j0->layout == 0 && j0->m->pair_fn[4] && traj <= kPairSliceMax;
    const long long per_wave = pair ? 32 : 64;
    for (Job *j : jobs) {
        if (j->layout == 0) {
            for (long long f = 0; f < j->G; f += per_wave) {
                wave_job.push_back(j->slot);
                wave_first.push_back(f);
            }
        } else {
            for (long long f = 0; f < j->G; ++f) {
                wave_job.push_back(j->slot);
                wave_first.push_back(f);
            }
        }
        j->n_ticks += 1;
    }
    // up to four wavefronts per block (fewer where the lane layout's LDS
    // would not fit); pad with entries that start past the end
    int wpb = 4;
    while (j0->layout == 0 && wpb > 1 &&
           cwc_lane_lds_bytes(j0->m->flat.n_cells, wpb, kDefaultSampleSlots) > s->ctx->max_lds)
        wpb /= 2;
    while (wave_job.size() % wpb) {
        wave_job.push_back(wave_job.back());
        wave_first.push_back(1ll << 40);
    }
    hipStream_t st = s->streams[si];
    const size_t n = wave_job.size();
    if (n > s->wave_cap[si]) {
        if (s->d_wave_job[si]) {
            SCHK(hipFree(s->d_wave_job[si]));
            SCHK(hipFree(s->d_wave_first[si]));
        }
        size_t cap = std::max<size_t>(n, 2 * s->wave_cap[si]);
        SCHK(hipMalloc(&s->d_wave_job[si], cap * sizeof(int)));
        SCHK(hipMalloc(&s->d_wave_first[si], cap * sizeof(long long)));
        s->wave_cap[si] = cap;
    }
    // the host vectors stay untouched until this stream's slice completes
    SCHK(hipMemcpyAsync(s->d_wave_job[si], wave_job.data(), n * sizeof(int),
                        hipMemcpyHostToDevice, st));
    SCHK(hipMemcpyAsync(s->d_wave_first[si], wave_first.data(), n * sizeof(long long),
                        hipMemcpyHostToDevice, st));
    hipFunction_t fn = pair ? j0->m->pair_fn[j0->shared_k ? 4 : 5]
                            : j0->m->fn[j0->layout][j0->shared_k ? 4 : 5];
    long long budget = s->slice;
    void *args[] = {&s->d_jobs, &s->d_wave_job[si], &s->d_wave_first[si], &budget};
    const unsigned lds =
        j0->layout == 0 ? (unsigned)cwc_lane_lds_bytes(j0->m->flat.n_cells, wpb, kDefaultSampleSlots)
                        : 0u;
    SCHK(hipModuleLaunchKernel(fn, (unsigned)(n / wpb), 1, 1, 64 * wpb, 1, 1, lds, st, args,
                               nullptr));
    SCHK(hipEventRecord(s->ev_slice[si], st));
    return true;
}

bool finish_job(cwc_server *s, Job *j)
{
    hipStream_t a = s->aux;
    SCHK(launch_hist_to_n(j->kp.rec_hist, j->nk, j->I, j->K1, a));
    SCHK(launch_finalize(j->nk, j->kp.s1, j->kp.s2_hi32, j->kp.s2_lo32, j->I * (long long)j->K1,
                         j->C, j->mean, j->var, a));
    std::vector<long long> ev(j->G);
    SCHK(hipMemcpyAsync(ev.data(), j->kp.events, j->G * 8, hipMemcpyDeviceToHost, a));
    SCHK(hipStreamSynchronize(a));
    long long tot = 0;
    for (long long v : ev) tot += v;
    j->events = tot;
    return true;
}

// Wavefronts one slice launch may cover: about half the device at two
// wavefronts per SIMD, so one model's jobs can occupy several streams.
long long slice_wave_cap(const cwc_server *s) { return (long long)s->ctx->n_cu * 4; }

// ---- resident mode

// The queue of the job's model group, created on first use (scheduler
// thread).  Lane-layout models run two lanes per trajectory where they have
// two leaves (the shorter chain per event), else one.
int group_of(cwc_server *s, Job *j)
{
    for (size_t i = 0; i < s->groups.size(); ++i) {
        const RGroup &g = *s->groups[i];
        if (g.m == j->m && g.layout == j->layout && g.shared_k == j->shared_k) return (int)i;
    }
    auto g = std::make_unique<RGroup>();
    g->m = j->m;
    g->layout = j->layout;
    g->shared_k = j->shared_k;
    g->pair = j->layout == 0 && j->m->pair_fn[6] != nullptr;
    const int k = j->shared_k ? 6 : 7;
    g->fn = g->pair ? j->m->pair_fn[k] : j->m->fn[j->layout][k];
    g->per_wave = j->layout == 0 ? (g->pair ? 32 : 64) : 1;
    g->wpb = 4;
    while (j->layout == 0 && g->wpb > 1 &&
           cwc_lane_lds_bytes(j->m->flat.n_cells, g->wpb, kDefaultSampleSlots) > s->ctx->max_lds)
        g->wpb /= 2;
    g->lds = j->layout == 0
                 ? (unsigned)cwc_lane_lds_bytes(j->m->flat.n_cells, g->wpb, kDefaultSampleSlots)
                 : 0u;
    if (hipHostMalloc((void **)&g->h_items, kRingItems * CWC_RQ_ITEM * sizeof(long long),
                      hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&g->h_tail, sizeof(long long), hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&g->dv_items, g->h_items, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&g->dv_tail, g->h_tail, 0) != hipSuccess ||
        hipMalloc((void **)&g->d_head, sizeof(unsigned long long)) != hipSuccess ||
        hipMemsetAsync(g->d_head, 0, sizeof(unsigned long long), s->aux) != hipSuccess ||
        hipStreamSynchronize(s->aux) != hipSuccess) {
        if (g->h_items) (void)hipHostFree(g->h_items);
        if (g->h_tail) (void)hipHostFree(g->h_tail);
        if (g->d_head) (void)hipFree(g->d_head);
        return -1;
    }
    __atomic_store_n(g->h_tail, 0ll, __ATOMIC_RELEASE);
    s->groups.push_back(std::move(g));
    return (int)s->groups.size() - 1;
}

// Items of one admitted job: its trajectories in wavefront-sized runs,
// written into the ring before the tail that publishes them (release: a
// kernel that reads the tail sees the items and the job's tables).
void publish_items(cwc_server *s, Job *j)
{
    RGroup &g = *s->groups[j->group];
    long long t = g.published;
    for (long long f = 0; f < j->G; f += g.per_wave, ++t) {
        long long *it = g.h_items + CWC_RQ_ITEM * (t & (kRingItems - 1));
        it[0] = j->slot;
        it[1] = f;
        it[2] = (long long)j->id;
        it[3] = 0;
    }
    g.published = t;
    __atomic_store_n(g.h_tail, t, __ATOMIC_RELEASE);
}

// Launches a resident kernel of group gi with `waves` wavefronts on stream
// si (which has nothing in flight).
bool launch_resident(cwc_server *s, int si, int gi, long long waves)
{
    RGroup &g = *s->groups[gi];
    const long long blocks = (waves + g.wpb - 1) / g.wpb;
    cwc_rq q{};
    q.head = g.d_head;
    q.tail = g.dv_tail;
    q.items = g.dv_items;
    q.stop = s->dv_stop;
    q.done = s->dv_done;
    q.mask = kRingItems - 1;
    q.idle_ticks = s->idle_ticks;
    q.nslot = kDefaultSampleSlots;
    void *args[] = {&s->d_jobs, &q};
    if (!s->rstreams[si]) {
        if (!own_queue_stream(s->ctx, &s->rstreams[si])) {
            std::lock_guard<std::mutex> lk(s->mu);
            fail_locked(s, "resident stream creation failed");
            return false;
        }
        SCHK(hipEventCreateWithFlags(&s->ev_res[si], hipEventDisableTiming));
    }
    SCHK(hipModuleLaunchKernel(g.fn, (unsigned)blocks, 1, 1, 64 * g.wpb, 1, 1, g.lds,
                               s->rstreams[si], args, nullptr));
    SCHK(hipEventRecord(s->ev_res[si], s->rstreams[si]));
    s->rkern[si] = gi;
    return true;
}

void scheduler(cwc_server *s)
{
    if (hipSetDevice(s->ctx->device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(s->mu);
        fail_locked(s, "hipSetDevice failed in the scheduler");
        return;
    }
    std::vector<unsigned long long> done(s->max_active);
    std::vector<Job *> admitted;
    std::vector<Job *> inflight[kStreams];       // jobs of each stream's slice
    std::vector<Job *> ready;                    // admitted, not in a slice
    std::vector<Job *> unpublished;              // resident: admitted, items not yet published
    std::vector<Job *> published;                // resident: items published, not finished
    bool ok = true;
    bool stopping = false;
    double t_last = now_s(s->t0);
    for (;;) {
        bool kernels = false;                    // slices or resident kernels in flight
        for (int i = 0; i < kStreams; ++i) kernels = kernels || !inflight[i].empty();
        for (int i = 0; i < kRStreams; ++i) kernels = kernels || s->rkern[i] >= 0;
        const bool busy = kernels || !published.empty() || !unpublished.empty();
        int policy = CWC_SCHED_FIFO;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            const double t = now_s(s->t0);
            if (busy) s->stats.busy_s += t - t_last;
            t_last = t;
            if (!busy)
                s->cv.wait(lk, [&] { return s->stop || !s->queue.empty() || !ready.empty(); });
            t_last = now_s(s->t0);
            stopping = s->stop;
            policy = s->policy;
            if (stopping && !kernels) return;
            if (stopping) {
                // drain what is in flight, start nothing new; resident
                // kernels leave once their current items end
                __atomic_store_n(s->h_stop, 1, __ATOMIC_RELEASE);
            } else if (!s->error.empty() || !ok) {
                if (!kernels) {
                    s->idle_cv.notify_all();
                    s->cv.wait(lk, [&] { return s->stop; });
                    return;
                }
                __atomic_store_n(s->h_stop, 1, __ATOMIC_RELEASE);
            } else {
                // admission: FIFO, while a slot and pool memory are free
                while (!s->queue.empty() && !s->free_slots.empty()) {
                    Job *j = s->jobs[s->queue.front()].get();
                    if (!reserve(s, j)) break;
                    j->slot = s->free_slots.back();
                    j->k_slice = policy == CWC_SCHED_RESIDENT ? 0 : s->slice_samples;
                    s->free_slots.pop_back();
                    s->queue.pop_front();
                    admitted.push_back(j);
                }
            }
        }
        const bool resident = policy == CWC_SCHED_RESIDENT;
        for (Job *j : admitted)
            if (ok) ok = init_job(s, j, j->slot);
        if (!admitted.empty()) {
            std::lock_guard<std::mutex> lk(s->mu);
            for (Job *j : admitted) {
                j->state = CWC_JOB_ACTIVE;
                j->t_admit = now_s(s->t0);
                s->active.push_back(j);
                (resident ? unpublished : ready).push_back(j);
            }
            admitted.clear();
        }
        std::vector<Job *> finished;
        bool progressed = false;
        if (resident && ok && !stopping) {
            // publish admitted jobs' items in admission order while the
            // ring has room beyond the items not yet claimed
            size_t n_pub = 0;
            for (Job *j : unpublished) {
                if (j->group < 0) j->group = group_of(s, j);
                if (j->group < 0) {
                    std::lock_guard<std::mutex> lk(s->mu);
                    fail_locked(s, "resident queue setup failed");
                    ok = false;
                    break;
                }
                RGroup &g = *s->groups[j->group];
                const long long need = (j->G + g.per_wave - 1) / g.per_wave;
                if (g.published + need - g.claimed > kRingItems) break;
                publish_items(s, j);
                published.push_back(j);
                ++n_pub;
                progressed = true;
            }
            unpublished.erase(unpublished.begin(), unpublished.begin() + n_pub);
            // completions: the kernel that finished a job's last item wrote
            // its id into the job's slot
            for (size_t i = 0; ok && i < published.size();) {
                Job *j = published[i];
                if (__atomic_load_n(s->h_done + j->slot, __ATOMIC_ACQUIRE) == (long long)j->id) {
                    if (!finish_job(s, j)) {
                        ok = false;
                        break;
                    }
                    finished.push_back(j);
                    published.erase(published.begin() + i);
                    progressed = true;
                } else {
                    ++i;
                }
            }
        }
        // resident kernels that have ended
        for (int i = 0; i < kRStreams; ++i) {
            if (s->rkern[i] < 0) continue;
            const hipError_t q = hipEventQuery(s->ev_res[i]);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                std::lock_guard<std::mutex> lk(s->mu);
                fail_locked(s, "a resident kernel failed");
                ok = false;
            }
            s->rkern[i] = -1;
            progressed = true;
        }
        for (int i = 0; i < kStreams; ++i) {
            if (inflight[i].empty()) continue;
            const hipError_t q = hipEventQuery(s->ev_slice[i]);
            if (q == hipErrorNotReady) continue;
            if (!ok) {
                // after a failure the slices in flight are only drained, so
                // the scheduler can stop
                inflight[i].clear();
                progressed = true;
                continue;
            }
            if (q != hipSuccess ||
                hipMemcpyAsync(done.data(), s->d_done, s->max_active * 8, hipMemcpyDeviceToHost,
                               s->aux) != hipSuccess ||
                hipStreamSynchronize(s->aux) != hipSuccess) {
                std::lock_guard<std::mutex> lk(s->mu);
                fail_locked(s, "a slice launch failed");
                ok = false;
                break;
            }
            progressed = true;
            const double dt_slice = now_s(s->t0) - s->t_slice[i];
            for (Job *j : inflight[i]) {
                j->slice_wall += dt_slice;
                if (j->k_slice > 0) j->samples_done = std::min(j->K1, j->samples_done + j->k_slice);
                if ((long long)done[j->slot] == j->G) {
                    if (!finish_job(s, j)) {
                        ok = false;
                        break;
                    }
                    finished.push_back(j);
                } else {
                    ready.push_back(j);
                }
            }
            inflight[i].clear();
        }
        if (!finished.empty()) {
            std::lock_guard<std::mutex> lk(s->mu);
            for (Job *j : finished) {
                j->state = CWC_JOB_DONE;
                j->t_done = now_s(s->t0);
                s->free_slots.push_back(j->slot);
                s->active.erase(std::find(s->active.begin(), s->active.end(), j));
                s->unreported.push_back(j->id);
                s->stats.jobs_done += 1;
                s->stats.events += j->events;
            }
        }
        if (resident && ok && !stopping) {
            // resident kernels: a group whose items wait unclaimed gets a
            // kernel on a free stream, at once if it has none running, else
            // once its items have waited 0.2 ms (its kernels' wavefronts are
            // all busy or gone); the claim counters are read back for this
            const double now = now_s(s->t0);
            for (size_t gi = 0; ok && gi < s->groups.size(); ++gi) {
                RGroup &g = *s->groups[gi];
                if (g.published == g.claimed) continue;
                if (hipMemcpyAsync(&s->h_head[0], g.d_head, 8, hipMemcpyDeviceToHost, s->aux) !=
                        hipSuccess ||
                    hipStreamSynchronize(s->aux) != hipSuccess) {
                    std::lock_guard<std::mutex> lk(s->mu);
                    fail_locked(s, "claim counter read-back failed");
                    ok = false;
                    break;
                }
                g.claimed = std::max(g.claimed, std::min(s->h_head[0], g.published));
                const long long waiting = g.published - g.claimed;
                if (waiting == 0) {
                    g.t_unclaimed = -1.0;
                    continue;
                }
                if (g.t_unclaimed < 0) g.t_unclaimed = now;
                int running = 0, free_si = -1;
                for (int i = 0; i < kRStreams; ++i) {
                    running += s->rkern[i] == (int)gi;
                    if (free_si < 0 && s->rkern[i] < 0) free_si = i;
                }
                if (free_si < 0 || (running > 0 && now - g.t_unclaimed < 2e-4)) continue;
                const long long waves = std::min(waiting, slice_wave_cap(s));
                if (!launch_resident(s, free_si, (int)gi, waves)) {
                    ok = false;
                    break;
                }
                g.t_unclaimed = now;
                progressed = true;
                std::lock_guard<std::mutex> lk(s->mu);
                s->stats.ticks += 1;
            }
        }
        // launches: an idle stream takes the group of the first ready job:
        // the oldest (FIFO), or under the predictive policy (paper Sec. 5.2
        // schema ii: heuristics from the instances' history) jobs without a
        // slice yet first, in arrival order (one slice gives a short job its
        // result, a long one its history), then the job with the longest
        // predicted remaining time: its remaining slices times its mean slice
        // wall time so far
        if (policy == CWC_SCHED_PREDICTED && ready.size() > 1) {
            auto predicted = [](const Job *j) {
                if (j->n_ticks == 0 || j->k_slice <= 0) return -1.0;
                const double left = (double)(j->K1 - j->samples_done) / (double)j->k_slice;
                return std::max(0.0, left) * j->slice_wall / (double)j->n_ticks;
            };
            std::stable_sort(ready.begin(), ready.end(), [&](const Job *a, const Job *b) {
                const bool na = a->n_ticks == 0, nb = b->n_ticks == 0;
                if (na != nb) return na;
                if (na) return a->id < b->id;
                return predicted(a) > predicted(b);
            });
        }
        for (int i = 0; ok && !stopping && i < kStreams && !ready.empty(); ++i) {
            if (!inflight[i].empty()) continue;
            const Job *lead = ready.front();
            std::vector<Job *> take_jobs, rest;
            long long waves = 0;
            for (Job *j : ready) {
                const bool same = j->m == lead->m && j->layout == lead->layout &&
                                  j->shared_k == lead->shared_k;
                const long long w = j->layout == 0 ? (j->G + 63) / 64 : j->G;
                if (same && (take_jobs.empty() || waves + w <= slice_wave_cap(s))) {
                    take_jobs.push_back(j);
                    waves += w;
                } else {
                    rest.push_back(j);
                }
            }
            ready.swap(rest);
            s->t_slice[i] = now_s(s->t0);
            if (!launch_slice(s, i, take_jobs)) {
                ok = false;
                break;
            }
            inflight[i] = take_jobs;
            progressed = true;
            std::lock_guard<std::mutex> lk(s->mu);
            s->stats.ticks += 1;
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (!ok) fail_locked(s, "scheduler stopped after a device error");
            bool any = false;
            for (int i = 0; i < kStreams; ++i) any = any || !inflight[i].empty();
            if (s->queue.empty() && s->active.empty() && !any) s->idle_cv.notify_all();
            if (!ok) s->idle_cv.notify_all();
        }
        if (!progressed) {
            // work in flight and none finished: poll again shortly; nothing
            // in flight and nothing admissible (the pool is held by finished,
            // unreleased jobs): sleep until a submission or release
            bool any = !published.empty() || !unpublished.empty();
            for (int i = 0; i < kStreams; ++i) any = any || !inflight[i].empty();
            for (int i = 0; i < kRStreams; ++i) any = any || s->rkern[i] >= 0;
            std::unique_lock<std::mutex> lk(s->mu);
            if (any)
                s->cv.wait_for(lk, std::chrono::microseconds(200));
            else
                s->cv.wait_for(lk, std::chrono::milliseconds(20));
        }
    }
}

Job *find_done(cwc_server *s, uint64_t id, cwc_status *st)
{
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) {
        *st = set_err(CWC_E_INVALID, "unknown job %llu", (unsigned long long)id);
        return nullptr;
    }
    if (it->second->state != CWC_JOB_DONE) {
        *st = set_err(CWC_E_NOTREADY, "job %llu not finished", (unsigned long long)id);
        return nullptr;
    }
    return it->second.get();
}

cwc_status copy_out(void *dst, const void *src, size_t bytes, int dev, hipStream_t st)
{
    if (!dst || !bytes) return CWC_OK;
    if (hipMemcpyAsync(dst, src, bytes, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                       st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return set_err(CWC_E_DEVICE, "result copy failed");
    return CWC_OK;
}

}  // namespace

extern "C" {

cwc_status cwc_server_create(cwc_ctx *ctx, size_t hbm_budget, int32_t max_active,
                             int64_t slice_events, cwc_server **out)
{
    if (!ctx || !out) return set_err(CWC_E_INVALID, "null argument");
    *out = nullptr;
    if (max_active < 1 || max_active > 1024) return set_err(CWC_E_INVALID, "max_active must be in [1, 1024]");
    if (slice_events < 1) return set_err(CWC_E_INVALID, "slice_events must be >= 1");
    if (hbm_budget < (1u << 20)) return set_err(CWC_E_NOMEM, "hbm_budget below 1 MiB");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(CWC_E_DEVICE, "hipSetDevice failed");
    auto s = std::make_unique<cwc_server>();
    s->ctx = ctx;
    s->max_active = max_active;
    s->slice = slice_events;
    cwc_status st = CWC_OK;
    s->pool_mem = ctx->alloc(hbm_budget, &st);
    if (!s->pool_mem) return st;
    s->pool.init(s->pool_mem, hbm_budget);
    bool ok = hipMalloc(&s->d_jobs, sizeof(cwc_kparams) * max_active) == hipSuccess &&
              hipMalloc(&s->d_done, 8 * max_active) == hipSuccess &&
              own_queue_stream(ctx, &s->aux) && own_queue_stream(ctx, &s->fetch);
    for (int i = 0; ok && i < kStreams; ++i)
        ok = own_queue_stream(ctx, &s->streams[i]) &&
             hipEventCreateWithFlags(&s->ev_slice[i], hipEventDisableTiming) == hipSuccess;
    // resident mode's flags in coherent host memory; a resident wavefront
    // gives up waiting for items after 2 ms of the device's wall clock
    int khz = 0;
    ok = ok &&
         hipHostMalloc((void **)&s->h_stop, sizeof(int), hipHostMallocCoherent) == hipSuccess &&
         hipHostMalloc((void **)&s->h_done, sizeof(long long) * max_active,
                       hipHostMallocCoherent) == hipSuccess &&
         hipHostGetDevicePointer((void **)&s->dv_stop, s->h_stop, 0) == hipSuccess &&
         hipHostGetDevicePointer((void **)&s->dv_done, s->h_done, 0) == hipSuccess &&
         hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) == hipSuccess &&
         khz > 0;
    if (!ok) {
        for (int i = 0; i < kStreams; ++i) {
            if (s->streams[i]) (void)hipStreamDestroy(s->streams[i]);
            if (s->ev_slice[i]) (void)hipEventDestroy(s->ev_slice[i]);
        }
        if (s->aux) (void)hipStreamDestroy(s->aux);
        if (s->fetch) (void)hipStreamDestroy(s->fetch);
        if (s->d_jobs) (void)hipFree(s->d_jobs);
        if (s->d_done) (void)hipFree(s->d_done);
        if (s->h_stop) (void)hipHostFree(s->h_stop);
        if (s->h_done) (void)hipHostFree(s->h_done);
        ctx->release(s->pool_mem);
        return set_err(CWC_E_DEVICE, "server device setup failed");
    }
    *s->h_stop = 0;
    for (int i = 0; i < max_active; ++i) s->h_done[i] = 0;
    s->idle_ticks = 2ll * khz;
    s->h_head.assign(1, 0);
    for (int i = max_active - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->stats.pool_bytes = (int64_t)s->pool.bytes;
    s->t0 = std::chrono::steady_clock::now();
    ctx_retain(ctx);                    // dropped by cwc_server_destroy
    cwc_server *raw = s.release();
    raw->th = std::thread(scheduler, raw);
    *out = raw;
    return CWC_OK;
}

cwc_status cwc_server_set_policy(cwc_server *s, int32_t slice_samples, int32_t policy)
{
    if (!s) return set_err(CWC_E_INVALID, "null server");
    if (slice_samples < 0) return set_err(CWC_E_INVALID, "slice_samples must be >= 0");
    if (policy != CWC_SCHED_FIFO && policy != CWC_SCHED_PREDICTED && policy != CWC_SCHED_RESIDENT)
        return set_err(CWC_E_INVALID, "unknown scheduling policy %d", policy);
    std::lock_guard<std::mutex> lk(s->mu);
    if ((policy == CWC_SCHED_RESIDENT) != (s->policy == CWC_SCHED_RESIDENT) &&
        (!s->queue.empty() || !s->active.empty()))
        return set_err(CWC_E_INVALID, "switching to or from the resident policy needs a server "
                                      "with no queued or active job");
    s->slice_samples = slice_samples;
    s->policy = policy;
    return CWC_OK;
}

cwc_status cwc_server_submit(cwc_server *s, const cwc_model *m, const cwc_run_desc *d,
                             uint64_t *job_id)
{
    if (!s || !m || !d || !job_id) return set_err(CWC_E_INVALID, "null argument");
    if (m->ctx != s->ctx) return set_err(CWC_E_INVALID, "model belongs to another context");
    auto j = std::make_unique<Job>();
    cwc_status st = validate_run(m, d, &j->rates, &j->init);
    if (st != CWC_OK) return st;
    // general models run one wavefront per trajectory (layout 2), their
    // terms checkpointed in the job's term buffer between slices
    st = ensure_layout(const_cast<cwc_model *>(m), m->flat.layout);
    if (st != CWC_OK) return st;
    j->m = const_cast<cwc_model *>(m);
    j->layout = m->flat.layout;
    if (m->gen)
        j->term_ints = d->n_instances * d->replicas_per_instance * (long long)m->gen->max_comp *
                       (3 + 2 * m->gen->n_species);
    j->d = *d;
    j->d.tuning = nullptr;
    j->I = d->n_instances;
    j->R = d->replicas_per_instance;
    j->G = j->I * j->R;
    j->K1 = d->n_samples;
    j->C = m->flat.n_cells;
    j->NR = std::max(1, m->flat.n_rules);
    j->shared_k = !(d->rate_table && m->flat.n_rules > 0);
    if (job_bytes(*j) > s->pool.bytes)
        return set_err(CWC_E_NOMEM, "job needs %zu bytes, the server pool has %zu", job_bytes(*j),
                       s->pool.bytes);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->policy == CWC_SCHED_RESIDENT && j->G > kRingItems * (j->layout == 0 ? 32 : 1))
        return set_err(CWC_E_UNSUPPORTED, "a resident-policy job takes at most %lld items (%lld "
                                          "trajectories)", kRingItems,
                       kRingItems * (j->layout == 0 ? 32 : 1));
    if (!s->error.empty()) return set_err(CWC_E_DEVICE, "server failed: %s", s->error.c_str());
    j->id = s->next_id++;
    j->t_submit = now_s(s->t0);
    *job_id = j->id;
    s->queue.push_back(j->id);
    s->jobs[j->id] = std::move(j);
    s->stats.jobs_submitted += 1;
    s->cv.notify_all();
    return CWC_OK;
}

cwc_status cwc_server_poll(cwc_server *s, uint64_t *done_ids, int32_t max, int32_t *n_done)
{
    if (!s || !n_done || (max > 0 && !done_ids)) return set_err(CWC_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->error.empty()) return set_err(CWC_E_DEVICE, "server failed: %s", s->error.c_str());
    int n = std::min<int>(max, (int)s->unreported.size());
    for (int i = 0; i < n; ++i) done_ids[i] = s->unreported[i];
    s->unreported.erase(s->unreported.begin(), s->unreported.begin() + n);
    *n_done = n;
    return CWC_OK;
}

cwc_status cwc_server_job_info(cwc_server *s, uint64_t job, cwc_job_info *info)
{
    if (!s || !info) return set_err(CWC_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return set_err(CWC_E_INVALID, "unknown job");
    const Job &j = *it->second;
    info->state = j.state;
    info->n_ticks = j.n_ticks;
    info->t_submit = j.t_submit;
    info->t_admit = j.t_admit;
    info->t_done = j.t_done;
    info->events = j.events;
    info->bytes = (int64_t)j.bytes;
    return CWC_OK;
}

cwc_status cwc_server_fetch_stats(cwc_server *s, uint64_t job, double *mean, double *var,
                                  int64_t *n, int dst_is_device)
{
    if (!s) return set_err(CWC_E_INVALID, "null server");
    cwc_status st = CWC_OK;
    Job *j;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        j = find_done(s, job, &st);
    }
    if (!j) return st;
    const size_t mom = (size_t)j->I * j->K1 * j->C;
    std::lock_guard<std::mutex> fk(s->fetch_mu);
    hipStream_t a = s->fetch;
    if ((st = copy_out(mean, j->mean, mom * 8, dst_is_device, a)) == CWC_OK &&
        (st = copy_out(var, j->var, mom * 8, dst_is_device, a)) == CWC_OK)
        st = copy_out(n, j->nk, (size_t)j->I * j->K1 * 8, dst_is_device, a);
    return st;
}

cwc_status cwc_server_fetch_counters(cwc_server *s, uint64_t job, int64_t *events,
                                     uint8_t *status, uint64_t *digest, double *t_final,
                                     int32_t *n_recorded, int32_t *final_counts,
                                     int dst_is_device)
{
    if (!s) return set_err(CWC_E_INVALID, "null server");
    cwc_status st = CWC_OK;
    Job *j;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        j = find_done(s, job, &st);
    }
    if (!j) return st;
    const size_t G = (size_t)j->G;
    std::lock_guard<std::mutex> fk(s->fetch_mu);
    hipStream_t a = s->fetch;
    int dv = dst_is_device;
    if ((st = copy_out(events, j->kp.events, G * 8, dv, a)) == CWC_OK &&
        (st = copy_out(status, j->kp.status, G, dv, a)) == CWC_OK &&
        (st = copy_out(digest, j->kp.digest, G * 8, dv, a)) == CWC_OK &&
        (st = copy_out(t_final, j->kp.t_final, G * 8, dv, a)) == CWC_OK &&
        (st = copy_out(n_recorded, j->kp.n_recorded, G * 4, dv, a)) == CWC_OK)
        st = copy_out(final_counts, j->kp.final_counts, G * j->C * 4, dv, a);
    return st;
}

cwc_status cwc_server_fetch_term(cwc_server *s, uint64_t job, int32_t *dst, int dst_is_device)
{
    if (!s || !dst) return set_err(CWC_E_INVALID, "null argument");
    cwc_status st = CWC_OK;
    Job *j;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        j = find_done(s, job, &st);
    }
    if (!j) return st;
    if (!j->term_ints) return set_err(CWC_E_INVALID, "not a general model: its term is fixed");
    std::lock_guard<std::mutex> fk(s->fetch_mu);
    hipStream_t a = s->fetch;
    st = copy_out(dst, j->kp.final_term, (size_t)j->term_ints * 4, dst_is_device, a);
    return st;
}

cwc_status cwc_server_release(cwc_server *s, uint64_t job)
{
    if (!s) return set_err(CWC_E_INVALID, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    cwc_status st = CWC_OK;
    Job *j = find_done(s, job, &st);
    if (!j) return st;
    drop(s, j);
    s->jobs.erase(job);
    s->cv.notify_all();            // freed memory may admit queued jobs
    return CWC_OK;
}

cwc_status cwc_server_wait_idle(cwc_server *s, double timeout_s)
{
    if (!s) return set_err(CWC_E_INVALID, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    bool ok = s->idle_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] {
        return (s->queue.empty() && s->active.empty()) || !s->error.empty();
    });
    if (!s->error.empty()) return set_err(CWC_E_DEVICE, "server failed: %s", s->error.c_str());
    if (!ok) return set_err(CWC_E_NOTREADY, "jobs still queued or active");
    return CWC_OK;
}

cwc_status cwc_server_get_stats(cwc_server *s, cwc_server_stats *st)
{
    if (!s || !st) return set_err(CWC_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->stats;
    st->pool_used = (int64_t)s->pool.used;
    st->pool_peak = (int64_t)s->pool.peak;
    return CWC_OK;
}

void cwc_server_destroy(cwc_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    (void)hipSetDevice(s->ctx->device);
    for (int i = 0; i < kStreams; ++i) {
        if (s->streams[i]) {
            (void)hipStreamSynchronize(s->streams[i]);
            (void)hipStreamDestroy(s->streams[i]);
        }
        if (s->d_wave_job[i]) (void)hipFree(s->d_wave_job[i]);
        if (s->d_wave_first[i]) (void)hipFree(s->d_wave_first[i]);
        if (s->ev_slice[i]) (void)hipEventDestroy(s->ev_slice[i]);
    }
    for (int i = 0; i < kRStreams; ++i) {
        if (s->rstreams[i]) {
            (void)hipStreamSynchronize(s->rstreams[i]);
            (void)hipStreamDestroy(s->rstreams[i]);
        }
        if (s->ev_res[i]) (void)hipEventDestroy(s->ev_res[i]);
    }
    if (s->aux) (void)hipStreamDestroy(s->aux);
    if (s->fetch) (void)hipStreamDestroy(s->fetch);
    if (s->d_jobs) (void)hipFree(s->d_jobs);
    if (s->d_done) (void)hipFree(s->d_done);
    for (auto &g : s->groups) {
        (void)hipHostFree(g->h_items);
        (void)hipHostFree(g->h_tail);
        (void)hipFree(g->d_head);
    }
    if (s->h_stop) (void)hipHostFree(s->h_stop);
    if (s->h_done) (void)hipHostFree(s->h_done);
    cwc_ctx *ctx = s->ctx;
    ctx->release(s->pool_mem);
    delete s;
    (void)hipGetLastError();   // errors of the teardown are not the next call's
    ctx_drop(ctx);
}

}  // extern "C"
