// Streamed runs: bounded-memory, windowed execution of a run (paper
// Sec. 5.2, schemas ii and iii).
//
// Schema ii makes every simulation instance an object that can be stopped
// and restarted, time-sliced at constant simulation time, with the
// scheduler guided by predictive heuristics from the instances' history.
// Schema iii pipelines the on-line reduction behind the simulation: since
// slicing keeps all trajectories nearly aligned in simulation time, a
// running window of the trajectories is reduced while later parts are
// still being produced, and the reduced part is dropped from memory.
//
// Here a run of K+1 sample points is cut into windows of W sample points.
// One time-sliced kernel launch per window advances every unfinished
// trajectory until it is about to record the window's first sample past
// the end (or finishes), and suspends it to a per-trajectory device
// checkpoint.  The moments of the window's W rows are then finalised into
// mean and variance, copied out on a second stream while the next window
// already runs, and the rows are cleared for reuse.  Device memory is
// O(G C + I W C) instead of O(I (K+1) C).  Before each window the
// wavefronts are ordered by the events their trajectories applied in the
// previous window (heaviest first; the first window by total propensity at
// t = 0), so the hardware dispatcher starts the slowest work first.
// Trajectories are bit-identical to an uninterrupted run: a suspended
// trajectory resumes with the same state and redraws the same
// counter-based random numbers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/cwcssa.h"
#include "runtime.h"
#include "stats.h"

using namespace cwc;

#define HIPCHK(call)                                                               \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return set_err(CWC_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

struct cwc_stream {
    cwc_ctx *ctx = nullptr;
    const cwc_model *m = nullptr;
    long long I = 0, R = 0, G = 0;
    int K1 = 0, C = 0, W = 0, n_windows = 0;
    int next_window = 0;                // window whose statistics next() returns
    int launched = 0;                   // windows launched so far
    int layout = 0, group = 1, per_wave = 64, wpb = 4;
    hipFunction_t fn = nullptr;
    unsigned lds = 0;
    std::string kernel;
    long long n_waves = 0;              // wavefronts of a window's launch (padded)
    std::vector<void *> bufs;
    size_t device_bytes = 0;
    // device state
    cwc_kparams *d_kp = nullptr;        // [2] parameters of alternate windows
    int *d_wave_job = nullptr;          // [n_waves] all zero (one job)
    long long *d_wave_first[2] = {};    // wave order of alternate windows
    double *mean[2] = {}, *var[2] = {}; // finalised rows, alternate windows
    long long *nrow[2] = {};            // contributor counts, alternate windows
    cwc_kparams kp{};                   // window 0's parameters (others differ
                                        // in k_base and k_stop only)
    // host state
    long long *h_wave_first[2] = {};    // pinned: the order uploaded per window
    cwc_kparams *h_kp = nullptr;        // pinned [2]: the parameters uploaded per window
    std::vector<long long> e_prev;      // applied events at the previous window's end
    std::vector<long long> e_now;
    std::vector<unsigned char> ck_state;
    std::vector<double> wave_cost;
    hipStream_t stream = nullptr;       // simulation stream (the caller's)
    hipStream_t copy = nullptr;         // output copies
    hipEvent_t ev_fin[2] = {}, ev_start = nullptr, ev_sim = nullptr;
    float last_ms = 0.0f;
    long long events_total = 0;
};

namespace {

template <class T>
cwc_status take(cwc_stream *s, T **p, size_t count)
{
    cwc_status st = CWC_OK;
    const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
    void *q = s->ctx->alloc(bytes, &st);
    if (!q) return st;
    s->bufs.push_back(q);
    s->device_bytes += bytes;
    *p = (T *)q;
    return CWC_OK;
}

void free_stream(cwc_stream *s)
{
    if (!s) return;
    cwc_ctx *ctx = s->ctx;
    (void)hipSetDevice(ctx->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->copy) {
        (void)hipStreamSynchronize(s->copy);
        (void)hipStreamDestroy(s->copy);
    }
    for (void *p : s->bufs) ctx->release(p);
    for (int i = 0; i < 2; ++i) {
        if (s->h_wave_first[i]) (void)hipHostFree(s->h_wave_first[i]);
        if (s->ev_fin[i]) (void)hipEventDestroy(s->ev_fin[i]);
    }
    if (s->h_kp) (void)hipHostFree(s->h_kp);
    if (s->ev_start) (void)hipEventDestroy(s->ev_start);
    if (s->ev_sim) (void)hipEventDestroy(s->ev_sim);
    delete s;
    (void)hipGetLastError();
    ctx_drop(ctx);
}

// Zero the window's accumulator rows (moments and contributor counts).
cwc_status clear_rows(cwc_stream *s, long long *nrow)
{
    const long long mom = s->I * (long long)s->W * s->C;
    HIPCHK(launch_fill_u64(s->kp.s1, 0, mom, s->stream));
    HIPCHK(launch_fill_u64(s->kp.s2_hi32, 0, mom, s->stream));
    HIPCHK(launch_fill_u64(s->kp.s2_lo32, 0, mom, s->stream));
    HIPCHK(launch_fill_u64((unsigned long long *)nrow, 0, s->I * (long long)s->W, s->stream));
    return CWC_OK;
}

// Wave order of window w: heaviest first by `cost` (events of the previous
// window, or the initial propensity), stable, padded to whole blocks with
// entries past the end.
void order_waves(cwc_stream *s, const std::vector<double> &cost, long long *out)
{
    const long long real = (s->G + s->per_wave - 1) / s->per_wave;
    std::vector<long long> idx(real);
    std::iota(idx.begin(), idx.end(), 0ll);
    std::stable_sort(idx.begin(), idx.end(),
                     [&](long long a, long long b) { return cost[a] > cost[b]; });
    for (long long i = 0; i < real; ++i) out[i] = idx[i] * s->per_wave;
    for (long long i = real; i < s->n_waves; ++i) out[i] = 1ll << 40;
}

// Enqueues window w: its wave order, the kernel, and (on the same stream,
// after it) nothing else; the caller finalises.
cwc_status launch_window(cwc_stream *s, int w)
{
    long long *h = s->h_wave_first[w & 1];
    HIPCHK(hipMemcpyAsync(s->d_wave_first[w & 1], h, s->n_waves * sizeof(long long),
                          hipMemcpyHostToDevice, s->stream));
    // this window's parameters (rows of its samples, where it stops); the
    // pinned slot was last read by window w - 2, which has finished
    cwc_kparams &k = s->h_kp[w & 1];
    k = s->kp;
    k.k_base = w * s->W;
    k.k_stop = std::min(s->K1, (w + 1) * s->W);
    k.n_rows = (unsigned long long *)s->nrow[w & 1];
    HIPCHK(hipMemcpyAsync(s->d_kp + (w & 1), &k, sizeof(cwc_kparams), hipMemcpyHostToDevice,
                          s->stream));
    cwc_kparams *jobs = s->d_kp + (w & 1);
    long long budget = 0x7FFFFFFFFFFFFFFFll;     // no draw limit: the window ends a slice
    void *args[] = {&jobs, &s->d_wave_job, &s->d_wave_first[w & 1], &budget};
    HIPCHK(hipEventRecord(s->ev_start, s->stream));
    HIPCHK(hipModuleLaunchKernel(s->fn, (unsigned)(s->n_waves / s->wpb), 1, 1, 64 * s->wpb, 1, 1,
                                 s->lds, s->stream, args, nullptr));
    HIPCHK(hipEventRecord(s->ev_sim, s->stream));
    s->launched = w + 1;
    return CWC_OK;
}

}  // namespace

extern "C" cwc_status cwc_stream_open(cwc_ctx *ctx, const cwc_model *m, const cwc_run_desc *d,
                                      int32_t window, void *hip_stream, cwc_stream **out)
{
    if (!ctx || !m || !d || !out) return set_err(CWC_E_INVALID, "null argument");
    *out = nullptr;
    if (m->ctx != ctx) return set_err(CWC_E_INVALID, "model belongs to another context");
    if (window < 1) return set_err(CWC_E_INVALID, "window must be >= 1 sample point");
    if (d->want_traj)
        return set_err(CWC_E_UNSUPPORTED, "a streamed run keeps statistics only: want_traj must be 0");
    std::vector<double> rates;
    std::vector<int> init;
    cwc_status st = validate_run(m, d, &rates, &init);
    if (st != CWC_OK) return st;
    const Flat &f = m->flat;
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(CWC_E_DEVICE, "hipSetDevice failed");

    auto s = new cwc_stream();
    s->ctx = ctx;
    ctx_retain(ctx);
    s->m = m;
    s->I = d->n_instances;
    s->R = d->replicas_per_instance;
    s->G = s->I * s->R;
    s->K1 = d->n_samples;
    s->C = f.n_cells;
    s->W = std::min<int>(window, d->n_samples);
    s->n_windows = (s->K1 + s->W - 1) / s->W;
    s->stream = (hipStream_t)hip_stream;
#define STCHK(expr)                     \
    do {                                \
        cwc_status st_ = (expr);        \
        if (st_ != CWC_OK) {            \
            free_stream(s);             \
            return st_;                 \
        }                               \
    } while (0)
#define SHIP(call)                                                                     \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            free_stream(s);                                                            \
            return set_err(CWC_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
        }                                                                              \
    } while (0)
    // layout: the model's own; lane-layout models run two lanes per
    // trajectory when they have two leaves, unless the tuning asks for one;
    // general models one wavefront per trajectory
    s->layout = f.layout;
    int lanes = d->tuning ? d->tuning->lanes_per_replica : 0;
    if (m->gen) {
        if (lanes != 0 && lanes != 64) {
            free_stream(s);
            return set_err(CWC_E_UNSUPPORTED, "a general model runs one wavefront per "
                                              "trajectory (lanes_per_replica 0 or 64)");
        }
    } else if (lanes == 64) {
        s->layout = 1;
    } else if (lanes == 1 || lanes == 2) {
        s->layout = 0;
    } else if (lanes != 0) {
        free_stream(s);
        return set_err(CWC_E_UNSUPPORTED, "a streamed run takes lanes_per_replica 0, 1, 2 or 64");
    }
    STCHK(ensure_layout(const_cast<cwc_model *>(m), s->layout));
    const bool shared = !(d->rate_table && f.n_rules > 0);
    if (s->layout == 2) {
        s->group = 64;
        s->per_wave = 1;
        s->fn = m->fn[2][shared ? 4 : 5];
        s->kernel = shared ? "cwc_gen_slice_shared" : "cwc_gen_slice_table";
    } else if (s->layout == 1) {
        s->group = 64;
        s->per_wave = 1;
        s->fn = m->fn[1][shared ? 4 : 5];
        s->kernel = shared ? "cwc_wave_slice_shared" : "cwc_wave_slice_table";
    } else if (lanes != 1 && m->pair_fn[4]) {
        s->group = 2;
        s->per_wave = 32;
        s->fn = m->pair_fn[shared ? 4 : 5];
        s->kernel = shared ? "cwc_pair_slice_shared" : "cwc_pair_slice_table";
    } else {
        s->group = 1;
        s->per_wave = 64;
        s->fn = m->fn[0][shared ? 4 : 5];
        s->kernel = shared ? "cwc_lane_slice_shared" : "cwc_lane_slice_table";
    }
    s->wpb = 4;
    while (s->layout == 0 && s->wpb > 1 &&
           cwc_lane_lds_bytes(s->C, s->wpb, kDefaultSampleSlots) > ctx->max_lds)
        s->wpb /= 2;
    s->lds = s->layout == 0 ? (unsigned)cwc_lane_lds_bytes(s->C, s->wpb, kDefaultSampleSlots) : 0u;
    const long long real = (s->G + s->per_wave - 1) / s->per_wave;
    s->n_waves = (real + s->wpb - 1) / s->wpb * s->wpb;

    // device buffers: per trajectory (checkpoint and terminal results), per
    // window row (moments, counts, finalised statistics)
    cwc_kparams &kp = s->kp;
    const long long G = s->G, C = s->C, rows = s->I * (long long)s->W;
    double *d_rates = nullptr;
    int *d_init = nullptr;
    STCHK(take(s, &d_rates, rates.size()));
    STCHK(take(s, &d_init, init.size()));
    STCHK(take(s, &kp.final_counts, G * C));
    STCHK(take(s, &kp.ck_counts, G * C));
    STCHK(take(s, &kp.events, G));
    STCHK(take(s, &kp.t_final, G));
    STCHK(take(s, &kp.digest, G));
    STCHK(take(s, &kp.status, G));
    STCHK(take(s, &kp.n_recorded, G));
    STCHK(take(s, &kp.ck_t, G));
    STCHK(take(s, &kp.ck_e, G));
    STCHK(take(s, &kp.ck_dig, G));
    STCHK(take(s, &kp.ck_kn, G));
    STCHK(take(s, &kp.ck_state, G));
    STCHK(take(s, &kp.done_count, 1));
    // general models: the term of each trajectory, its checkpoint while it
    // runs and its final term once it has ended
    if (m->gen)
        STCHK(take(s, &kp.final_term,
                   G * (long long)m->gen->max_comp * (3 + 2 * m->gen->n_species)));
    STCHK(take(s, &kp.s1, rows * C));
    STCHK(take(s, &kp.s2_hi32, rows * C));
    STCHK(take(s, &kp.s2_lo32, rows * C));
    for (int i = 0; i < 2; ++i) {
        STCHK(take(s, &s->nrow[i], rows));
        STCHK(take(s, &s->mean[i], rows * C));
        STCHK(take(s, &s->var[i], rows * C));
        STCHK(take(s, &s->d_wave_first[i], s->n_waves));
        SHIP(hipHostMalloc((void **)&s->h_wave_first[i], s->n_waves * sizeof(long long),
                           hipHostMallocDefault));
        SHIP(hipEventCreateWithFlags(&s->ev_fin[i], hipEventDisableTiming));
    }
    STCHK(take(s, &s->d_wave_job, s->n_waves));
    STCHK(take(s, &s->d_kp, 2));
    SHIP(hipHostMalloc((void **)&s->h_kp, 2 * sizeof(cwc_kparams), hipHostMallocDefault));
    SHIP(hipEventCreate(&s->ev_start));
    SHIP(hipEventCreate(&s->ev_sim));
    // the window copies must not queue behind the next window's kernel
    if (!own_queue_stream(ctx, &s->copy)) {
        free_stream(s);
        return set_err(CWC_E_DEVICE, "copy stream creation failed");
    }

    kp.seed = d->seed;
    kp.G = G;
    kp.R = s->R;
    kp.g_base = 0;
    kp.max_events = d->max_events;
    kp.dt = d->dt;
    kp.K1 = s->K1;
    kp.KR = s->W;
    kp.cap = (unsigned)d->count_cap;
    kp.rate_stride = shared ? 0 : (int)f.n_rules;
    kp.init_stride = d->init_table ? (int)C : 0;
    kp.want_traj = 0;
    kp.want_digest = d->want_digest ? 1 : 0;
    kp.rates = d_rates;
    kp.init = d_init;
    kp.nslot = kDefaultSampleSlots;
    kp.chunk = 1;
    kp.rec_hist = nullptr;
    kp.k_slice = 0;         // the window is the slice
    SHIP(hipMemcpy(d_rates, rates.data(), rates.size() * sizeof(double), hipMemcpyHostToDevice));
    SHIP(hipMemcpy(d_init, init.data(), init.size() * sizeof(int), hipMemcpyHostToDevice));
    SHIP(hipMemset(s->d_wave_job, 0, s->n_waves * sizeof(int)));
    SHIP(hipMemset(kp.ck_state, 0, G));
    SHIP(hipMemset(kp.done_count, 0, sizeof(unsigned long long)));

    // window 0: instances heaviest first by total propensity at t = 0
    {
        const std::vector<int> ord = instance_order(f, rates, init, (int)s->I, !shared,
                                                    d->init_table != nullptr);
        std::vector<double> rank(s->I);
        for (long long i = 0; i < s->I; ++i) rank[ord[i]] = (double)(s->I - i);
        std::vector<double> cost((size_t)real);
        for (long long wv = 0; wv < real; ++wv) {
            const long long g0 = wv * s->per_wave;
            cost[wv] = rank[g0 / s->R];
        }
        order_waves(s, cost, s->h_wave_first[0]);
    }
    s->e_prev.assign(G, 0);
    s->e_now.assign(G, 0);
    s->ck_state.assign(G, 0);
    s->wave_cost.assign((size_t)real, 0.0);
    STCHK(clear_rows(s, s->nrow[0]));
    STCHK(launch_window(s, 0));
#undef STCHK
#undef SHIP
    *out = s;
    return CWC_OK;
}

extern "C" cwc_status cwc_stream_next(cwc_stream *s, int32_t *k0, int32_t *rows, double *mean,
                                      double *var, int64_t *n, int dst_is_device)
{
    if (!s || !k0 || !rows) return set_err(CWC_E_INVALID, "null argument");
    HIPCHK(hipSetDevice(s->ctx->device));
    const int w = s->next_window;
    if (w >= s->n_windows) {
        *k0 = s->K1;
        *rows = 0;
        return CWC_OK;
    }
    // window w has been launched; wait for it and read the trajectories'
    // progress (the predictor of the next window's order)
    HIPCHK(hipEventSynchronize(s->ev_sim));
    HIPCHK(hipEventElapsedTime(&s->last_ms, s->ev_start, s->ev_sim));
    HIPCHK(hipMemcpy(s->e_now.data(), s->kp.ck_e, s->G * sizeof(long long), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(s->ck_state.data(), s->kp.ck_state, s->G, hipMemcpyDeviceToHost));
    // finalise window w's rows into its statistics buffers
    const int b = w & 1;
    const long long nr = s->I * (long long)s->W;
    HIPCHK(launch_finalize(s->nrow[b], s->kp.s1, s->kp.s2_hi32, s->kp.s2_lo32, nr, s->C,
                           s->mean[b], s->var[b], s->stream));
    HIPCHK(hipEventRecord(s->ev_fin[b], s->stream));
    // next window: clear the rows, order the waves by the events their
    // trajectories applied in window w (finished ones cost nothing), launch
    if (w + 1 < s->n_windows) {
        const long long real = (long long)s->wave_cost.size();
        for (long long wv = 0; wv < real; ++wv) {
            double c = 0.0;
            const long long g1 = std::min(s->G, (wv + 1) * s->per_wave);
            for (long long g = wv * s->per_wave; g < g1; ++g)
                if (s->ck_state[g] == 1) c += (double)(s->e_now[g] - s->e_prev[g]);
            s->wave_cost[wv] = c;
        }
        order_waves(s, s->wave_cost, s->h_wave_first[(w + 1) & 1]);
        cwc_status st = clear_rows(s, s->nrow[(w + 1) & 1]);
        if (st != CWC_OK) return st;
        st = launch_window(s, w + 1);
        if (st != CWC_OK) return st;
    }
    std::swap(s->e_prev, s->e_now);
    // window w's rows to the caller, behind the finalisation, beside the
    // next window's simulation
    const int k_base = w * s->W;
    const int nrows = std::min(s->K1, k_base + s->W) - k_base;
    HIPCHK(hipStreamWaitEvent(s->copy, s->ev_fin[b], 0));
    const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t C = (size_t)s->C;
    if (mean)
        HIPCHK(hipMemcpy2DAsync(mean, nrows * C * 8, s->mean[b], s->W * C * 8, nrows * C * 8,
                                s->I, kind, s->copy));
    if (var)
        HIPCHK(hipMemcpy2DAsync(var, nrows * C * 8, s->var[b], s->W * C * 8, nrows * C * 8, s->I,
                                kind, s->copy));
    if (n)
        HIPCHK(hipMemcpy2DAsync(n, nrows * 8, s->nrow[b], s->W * 8, nrows * 8, s->I, kind,
                                s->copy));
    HIPCHK(hipStreamSynchronize(s->copy));
    *k0 = k_base;
    *rows = nrows;
    s->next_window = w + 1;
    return CWC_OK;
}

extern "C" cwc_status cwc_stream_info(const cwc_stream *s, cwc_stream_info_t *info)
{
    if (!s || !info) return set_err(CWC_E_INVALID, "null argument");
    info->device_bytes = s->device_bytes;
    info->window = s->W;
    info->n_windows = s->n_windows;
    info->windows_done = s->next_window;
    info->last_window_ms = s->last_ms;
    std::snprintf(info->kernel, sizeof info->kernel, "%s", s->kernel.c_str());
    return CWC_OK;
}

extern "C" cwc_status cwc_stream_fetch_counters(cwc_stream *s, int64_t *events, uint8_t *status,
                                                uint64_t *digest, double *t_final,
                                                int32_t *n_recorded, int32_t *final_counts,
                                                int dst_is_device)
{
    if (!s) return set_err(CWC_E_INVALID, "null stream");
    if (s->next_window < s->n_windows)
        return set_err(CWC_E_NOTREADY, "the stream has windows left (%d of %d returned)",
                       s->next_window, s->n_windows);
    HIPCHK(hipSetDevice(s->ctx->device));
    HIPCHK(hipStreamSynchronize(s->stream));
    const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t G = (size_t)s->G;
    if (events) HIPCHK(hipMemcpy(events, s->kp.events, G * 8, kind));
    if (status) HIPCHK(hipMemcpy(status, s->kp.status, G, kind));
    if (digest) HIPCHK(hipMemcpy(digest, s->kp.digest, G * 8, kind));
    if (t_final) HIPCHK(hipMemcpy(t_final, s->kp.t_final, G * 8, kind));
    if (n_recorded) HIPCHK(hipMemcpy(n_recorded, s->kp.n_recorded, G * 4, kind));
    if (final_counts) HIPCHK(hipMemcpy(final_counts, s->kp.final_counts, G * s->C * 4, kind));
    return CWC_OK;
}

extern "C" cwc_status cwc_stream_fetch_term(cwc_stream *s, int32_t *dst, int dst_is_device)
{
    if (!s || !dst) return set_err(CWC_E_INVALID, "null argument");
    if (!s->m->gen) return set_err(CWC_E_INVALID, "not a general model: its term is fixed");
    if (s->next_window < s->n_windows)
        return set_err(CWC_E_NOTREADY, "the stream has windows left (%d of %d returned)",
                       s->next_window, s->n_windows);
    HIPCHK(hipSetDevice(s->ctx->device));
    HIPCHK(hipStreamSynchronize(s->stream));
    const GFlat &g = *s->m->gen;
    HIPCHK(hipMemcpy(dst, s->kp.final_term,
                     (size_t)s->G * g.max_comp * (3 + 2 * g.n_species) * sizeof(int32_t),
                     dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return CWC_OK;
}

extern "C" void cwc_stream_destroy(cwc_stream *s) { free_stream(s); }
