// Runs: validation, buffers, launch sequence (zero the accumulators ->
// simulation kernel -> contributor counts -> mean/variance), HIP-graph
// capture of the persistent form, completion and result fetches.
#include <hip/hip_runtime.h>
#include <thread>
#include <chrono>

#include <algorithm>
#include <cmath>
#include <cstring>
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

namespace {

template <class T>
cwc_status alloc_buf(cwc_run *r, T **p, size_t count)
{
    cwc_status st = CWC_OK;
    void *q = r->ctx->alloc(std::max<size_t>(1, count) * sizeof(T), &st);
    if (!q) return st;
    r->bufs.push_back(q);
    *p = (T *)q;
    return CWC_OK;
}

void free_run(cwc_run *r)
{
    if (!r) return;
    cwc_ctx *ctx = r->ctx;
    (void)hipSetDevice(ctx->device);
    if (r->launched && r->ev_end) (void)hipEventSynchronize(r->ev_end);
    if (r->graph) (void)hipGraphExecDestroy(r->graph);
    for (void *p : r->bufs) ctx->release(p);
    if (r->ev_start) (void)hipEventDestroy(r->ev_start);
    if (r->ev_sim) (void)hipEventDestroy(r->ev_sim);
    if (r->ev_end) (void)hipEventDestroy(r->ev_end);
    delete r;
    (void)hipGetLastError();   // errors of the teardown are not the next call's
    ctx_drop(ctx);
}

// Zero the accumulators and reset the queue cursor.
cwc_status enqueue_prologue(cwc_run *r, hipStream_t s)
{
    const long long mom = r->I * (long long)r->K1 * r->C;
    HIPCHK(launch_fill_u64(r->kp.s1, 0, mom, s));
    HIPCHK(launch_fill_u64(r->kp.s2_hi32, 0, mom, s));
    HIPCHK(launch_fill_u64(r->kp.s2_lo32, 0, mom, s));
    HIPCHK(launch_fill_u64(r->kp.rec_hist, 0, r->I * (long long)(r->K1 + 1), s));
    HIPCHK(launch_fill_u64(r->kp.cursor, r->n_threads, 1, s));
    return CWC_OK;
}

cwc_status enqueue_kernel(cwc_run *r, hipStream_t s)
{
    void *args[] = {&r->kp};
    HIPCHK(hipModuleLaunchKernel(r->fn, r->grid, 1, 1, r->block, 1, 1, r->lds, s, args, nullptr));
    return CWC_OK;
}

cwc_status enqueue_epilogue(cwc_run *r, hipStream_t s)
{
    HIPCHK(launch_hist_to_n(r->kp.rec_hist, r->nk, r->I, r->K1, s));
    HIPCHK(launch_finalize(r->nk, r->kp.s1, r->kp.s2_hi32, r->kp.s2_lo32, r->I * (long long)r->K1,
                           r->C, r->mean, r->var, s));
    return CWC_OK;
}

cwc_status capture_graph(cwc_run *r)
{
    hipStream_t cs = r->ctx->capture_stream;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    cwc_status st = enqueue_prologue(r, cs);
    if (st == CWC_OK) st = enqueue_kernel(r, cs);
    if (st == CWC_OK) st = enqueue_epilogue(r, cs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (st != CWC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return set_err(CWC_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&r->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return set_err(CWC_E_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    return CWC_OK;
}

cwc_status launch(cwc_run *r, hipStream_t s)
{
    HIPCHK(hipSetDevice(r->ctx->device));
    // a relaunch on another stream must not overlap the previous launch,
    // which uses the same buffers
    if (r->launched) HIPCHK(hipStreamWaitEvent(s, r->ev_end, 0));
    if (r->mode == CWC_MODE_PERSISTENT) {
        HIPCHK(hipEventRecord(r->ev_start, s));
        HIPCHK(hipGraphLaunch(r->graph, s));
        HIPCHK(hipEventRecord(r->ev_sim, s));
        HIPCHK(hipEventRecord(r->ev_end, s));
    } else {
        cwc_status st = enqueue_prologue(r, s);
        if (st != CWC_OK) return st;
        HIPCHK(hipEventRecord(r->ev_start, s));
        st = enqueue_kernel(r, s);
        if (st != CWC_OK) return st;
        HIPCHK(hipEventRecord(r->ev_sim, s));
        st = enqueue_epilogue(r, s);
        if (st != CWC_OK) return st;
        HIPCHK(hipEventRecord(r->ev_end, s));
    }
    r->stream = s;
    r->launched = true;
    return CWC_OK;
}


bool valid_rate(double k) { return std::isfinite(k) && k > 0.0 && k <= 1e250; }

// name of kernel k (plain/persistent x shared/table) of a run's family
std::string kernel_name(int layout, int group, int k)
{
    static const char *forms[4] = {"plain_shared", "plain_table", "persistent_shared",
                                   "persistent_table"};
    const char *fam = layout == 2 ? "cwc_gen" : layout == 1 ? "cwc_wave"
                                  : (group == 4 ? "cwc_quad" : (group == 2 ? "cwc_pair" : "cwc_lane"));
    return std::string(fam) + "_" + forms[k];
}

cwc_status ready(cwc_run *r)
{
    if (!r) return set_err(CWC_E_INVALID, "null run");
    if (!r->launched) return set_err(CWC_E_NOTREADY, "run not launched");
    hipError_t e = hipEventQuery(r->ev_end);
    if (e == hipErrorNotReady) return set_err(CWC_E_NOTREADY, "run still in flight");
    if (e != hipSuccess) return set_err(CWC_E_DEVICE, "run failed: %s", hipGetErrorString(e));
    return CWC_OK;
}

cwc_status copy_out(void *dst, const void *src, size_t bytes, int dst_is_device)
{
    if (!dst || bytes == 0) return CWC_OK;
    HIPCHK(hipMemcpy(dst, src, bytes, dst_is_device ? hipMemcpyDeviceToDevice
                                                    : hipMemcpyDeviceToHost));
    return CWC_OK;
}

}  // namespace

namespace cwc {

// Total propensity of each instance's initial state (host, for scheduling
// only) and the instance order by decreasing value.
std::vector<int> instance_order(const Flat &f, const std::vector<double> &rates,
                                const std::vector<int> &init, int I, bool rate_rows,
                                bool init_rows)
{
    std::vector<double> cost(I, 0.0);
    for (int i = 0; i < I; ++i) {
        const double *k = rates.data() + (rate_rows ? (size_t)i * f.n_rules : 0);
        const int *n = init.data() + (init_rows ? (size_t)i * f.n_cells : 0);
        double a0 = 0.0;
        for (const Slot &s : f.slots) {
            double h = 1.0;
            for (int t = 0; t < s.n_react; ++t) {
                const double x = n[s.react_cell[t]];
                h *= s.react_mult[t] == 2 ? x * std::max(x - 1.0, 0.0) * 0.5 : x;
            }
            a0 += k[s.rule] * h;
        }
        cost[i] = a0;
    }
    std::vector<int> order(I);
    for (int i = 0; i < I; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    return order;
}


// Checks a run descriptor against the model and returns host copies of the
// rate and initial-state tables (one shared row when not given).
cwc_status validate_run(const cwc_model *m, const cwc_run_desc *d, std::vector<double> *rates_out,
                        std::vector<int> *init_out)
{
    const Flat &f = m->flat;
    {
        cwc_status sst = validate_run_sizes(d);
        if (sst != CWC_OK) return sst;
    }
    const long long I = d->n_instances;
    const int C = f.n_cells;
    std::vector<double> &rates = *rates_out;
    std::vector<int> &init = *init_out;
    if (d->rate_table) {
        rates.assign(d->rate_table, d->rate_table + I * f.n_rules);
        for (double k : rates)
            if (!valid_rate(k)) return set_err(CWC_E_INVALID, "rate table entry not finite, > 0, <= 1e250");
        if (f.n_rules == 0) rates.assign(1, 1.0);
    } else {
        rates = f.k;
        if (rates.empty()) rates.assign(1, 1.0);
    }
    if (d->init_table && m->gen)
        return set_err(CWC_E_UNSUPPORTED,
                       "a general model starts from its own term: init_table must be NULL");
    if (d->init_table) {
        init.assign(d->init_table, d->init_table + I * C);
    } else {
        init = f.init;
    }
    for (int v : init)
        if (v < 0 || v > d->count_cap)
            return set_err(CWC_E_INVALID, "initial count outside [0, count_cap]");

    return CWC_OK;
}

// The scalar fields of a run descriptor: sizes, sample grid, caps.
cwc_status validate_run_sizes(const cwc_run_desc *d)
{
    if (d->n_instances < 1 || d->replicas_per_instance < 1)
        return set_err(CWC_E_INVALID, "n_instances and replicas_per_instance must be >= 1");
    if (d->n_instances > (1ll << 31) || d->replicas_per_instance > (1ll << 31) ||
        d->n_instances * d->replicas_per_instance > (1ll << 31))
        return set_err(CWC_E_INVALID, "at most 2^31 trajectories per run");
    if (!(std::isfinite(d->dt) && d->dt > 0.0))
        return set_err(CWC_E_INVALID, "dt must be finite and > 0");
    if (d->n_samples < 1 || d->n_samples > (1 << 24))
        return set_err(CWC_E_INVALID, "n_samples must be in [1, 2^24]");
    if (!std::isfinite(d->dt * (double)(d->n_samples - 1)))
        return set_err(CWC_E_INVALID, "last sample time is not finite");
    if (d->count_cap < 1) return set_err(CWC_E_INVALID, "count_cap must be >= 1");
    if (d->max_events < 0) return set_err(CWC_E_INVALID, "max_events must be >= 0");
    return CWC_OK;
}

// Launch shape of a run: tuning defaults and checks, layout (lanes per
// trajectory), block (narrowed until the lane layout's LDS fits), grid and
// kernel.  `tuned`: `tun` came from the autotuner's table.  `may_compile`:
// the layout's module may be compiled and loaded here; otherwise it must
// already be loaded.
cwc_status plan_launch(cwc_ctx *ctx, const cwc_model *m, const cwc_run_desc *d, cwc_tuning tun,
                       bool tuned, bool may_compile, LaunchPlan *out)
{
    const Flat &f = m->flat;
    const long long G = d->n_instances * d->replicas_per_instance;
    const int C = f.n_cells;
    if (tun.block_size <= 0) tun.block_size = 64;
    if (tun.block_size % 64 || tun.block_size > 256)
        return set_err(CWC_E_INVALID, "block_size must be a multiple of 64, at most 256");
    if (tun.waves_per_simd <= 0) tun.waves_per_simd = 2;
    if (tun.waves_per_simd > 16) return set_err(CWC_E_INVALID, "waves_per_simd must be <= 16");
    if (tun.refill_chunk <= 0) tun.refill_chunk = 64;
    if (tun.refill_chunk > 1 && tun.refill_chunk < 64)
        return set_err(CWC_E_INVALID, "refill_chunk must be 1 or at least 64");
    if (tun.sample_slots <= 0) tun.sample_slots = kDefaultSampleSlots;
    if (tun.sample_slots > 64 || (tun.sample_slots & (tun.sample_slots - 1)))
        return set_err(CWC_E_INVALID, "sample_slots must be a power of two, at most 64");
    int layout = f.layout;
    const bool pair = tun.lanes_per_replica == 2;
    const bool quad = tun.lanes_per_replica == 4;
    if (layout == 2) {
        // general terms: one wavefront per trajectory, lane = compartment slot
        if (tun.lanes_per_replica != 0 && tun.lanes_per_replica != 64)
            return set_err(CWC_E_UNSUPPORTED,
                           "a general model runs one wavefront per trajectory "
                           "(lanes_per_replica 0 or 64)");
    } else if (tun.lanes_per_replica == 1 || pair || quad) layout = 0;
    else if (tun.lanes_per_replica == 64) layout = 1;
    else if (tun.lanes_per_replica != 0)
        return set_err(CWC_E_UNSUPPORTED, "lanes_per_replica must be 0 (auto), 1, 2, 4 or 64");
    if (may_compile) {
        cwc_status lst = ensure_layout(const_cast<cwc_model *>(m), layout);
        if (lst != CWC_OK) return lst;
    } else if (!layout_loaded(m, layout)) {
        return set_err(CWC_E_INVALID,
                       "the model's code for the %s layout is not loaded (submit one run in "
                       "that layout with cwc_run_submit first)",
                       layout == 2 ? "general-term"
                                   : (layout == 1 ? "wavefront-per-replica" : "lane-per-replica"));
    }
    if (pair && !m->pair_fn[0])
        return set_err(CWC_E_UNSUPPORTED, "two lanes per trajectory need at least two leaves");
    if (quad && !m->quad_fn[0])
        return set_err(CWC_E_UNSUPPORTED, "four lanes per trajectory need at least four leaves");
    const int group = quad ? 4 : (pair ? 2 : 1);   // lanes per trajectory (lane module)
    tun.lanes_per_replica = layout >= 1 ? 64 : group;   // as launched

    const bool shared = !(d->rate_table && f.n_rules > 0);
    const bool wave = layout >= 1;
    if (wave && !tuned && (!d->tuning || d->tuning->block_size <= 0)) tun.block_size = 256;
    unsigned block = (unsigned)tun.block_size;
    // the lane layout's per-wavefront LDS (staging + accumulator cache)
    // grows with the cell count: narrow the block until it fits
    while (!wave && block > 64 &&
           cwc_lane_lds_bytes(C, (int)(block / 64), tun.sample_slots) > ctx->max_lds)
        block /= 2;
    if (!wave && cwc_lane_lds_bytes(C, 1, tun.sample_slots) > ctx->max_lds)
        return set_err(CWC_E_INVALID, "sample_slots too large for this model's cells");
    // lane layout: one trajectory per lane (two or four lanes per trajectory
    // in the pair and quad forms); wavefront layout: one per wave
    const long long per_block = wave ? block / 64 : block / group;
    const long long need_blocks = (G + per_block - 1) / per_block;
    unsigned grid;
    int k;
    if (d->mode == CWC_MODE_PERSISTENT) {
        long long resident = (long long)ctx->n_cu * 4 * tun.waves_per_simd * 64 / block;
        grid = (unsigned)std::max(1ll, std::min(need_blocks, resident));
        // a grid that already holds every trajectory has nothing to refill:
        // the queue would stay empty, so the kernel without the refill
        // bookkeeping runs the same computation, its blocks (dispatched as
        // others finish) taking the items in the same longest-first order
        const bool covers = (long long)grid * per_block >= G;
        k = covers ? (shared ? 0 : 1) : (shared ? 2 : 3);
    } else {
        k = shared ? 0 : 1;
        grid = (unsigned)need_blocks;
    }
    out->fn = quad ? m->quad_fn[k] : (pair ? m->pair_fn[k] : m->fn[layout][k]);
    out->kernel = kernel_name(layout, group, k);
    out->grid = grid;
    out->block = block;
    out->layout = layout;
    out->group = group;
    out->n_threads = (unsigned long long)grid * (unsigned long long)per_block;
    out->lds = wave ? 0u : (unsigned)cwc_lane_lds_bytes(C, (int)(block / 64), tun.sample_slots);
    out->tun = tun;
    return CWC_OK;
}

}  // namespace cwc

extern "C" {

cwc_status cwc_run_submit(cwc_ctx *ctx, const cwc_model *m, const cwc_run_desc *d,
                          void *hip_stream, cwc_run **out)
{
    if (!ctx || !m || !d || !out) return set_err(CWC_E_INVALID, "null argument");
    *out = nullptr;
    if (m->ctx != ctx) return set_err(CWC_E_INVALID, "model belongs to another context");
    if (d->mode != CWC_MODE_PLAIN && d->mode != CWC_MODE_PERSISTENT)
        return set_err(CWC_E_INVALID, "unknown mode %d", d->mode);
    const Flat &f = m->flat;
    std::vector<double> rates;
    std::vector<int> init;
    {
        cwc_status vst = validate_run(m, d, &rates, &init);
        if (vst != CWC_OK) return vst;
    }
    const long long I = d->n_instances, R = d->replicas_per_instance, G = I * R;
    const int C = f.n_cells, NR = std::max(1, f.n_rules), K1 = d->n_samples;

    // launch shape: the caller's, else the autotuner's stored choice, else
    // defaults
    cwc_tuning tun{};
    bool tuned = false;
    if (d->tuning) {
        tun = *d->tuning;
    } else {
        tuned = tuning_lookup(m, d, &tun);
    }
    LaunchPlan plan;
    {
        cwc_status pst = plan_launch(ctx, m, d, tun, tuned, true, &plan);
        if (pst != CWC_OK) return pst;
    }
    tun = plan.tun;

    auto r = new cwc_run();
    r->ctx = ctx;
    ctx_retain(ctx);                    // dropped by free_run
    r->m = m;
    r->I = I;
    r->R = R;
    r->G = G;
    r->K1 = K1;
    r->C = C;
    r->mode = d->mode;
    r->tun = tun;
    cwc_status st = CWC_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) {
        free_run(r);
        return set_err(CWC_E_DEVICE, "hipSetDevice failed");
    }
    double *d_rates = nullptr;
    int *d_init = nullptr;
    cwc_kparams &kp = r->kp;
    const long long mom = I * (long long)K1 * C;
#define ALLOC(ptr, n)                                   \
    do {                                                \
        st = alloc_buf(r, &(ptr), (size_t)(n));         \
        if (st != CWC_OK) {                             \
            free_run(r);                                \
            return st;                                  \
        }                                               \
    } while (0)
    ALLOC(d_rates, rates.size());
    ALLOC(d_init, init.size());
    ALLOC(kp.final_counts, G * C);
    ALLOC(kp.events, G);
    ALLOC(kp.t_final, G);
    ALLOC(kp.digest, G);
    ALLOC(kp.status, G);
    ALLOC(kp.n_recorded, G);
    if (d->want_traj) ALLOC(kp.traj, G * (long long)K1 * C);
    if (m->gen) ALLOC(kp.final_term, G * (long long)m->gen->max_comp * (3 + 2 * m->gen->n_species));
    ALLOC(kp.s1, mom);
    ALLOC(kp.s2_hi32, mom);
    ALLOC(kp.s2_lo32, mom);
    ALLOC(kp.rec_hist, I * (long long)(K1 + 1));
    ALLOC(kp.cursor, 1);
    int *d_order = nullptr;
    if (d->mode == CWC_MODE_PERSISTENT && I > 1) ALLOC(d_order, I);
    ALLOC(r->nk, I * (long long)K1);
    ALLOC(r->mean, mom);
    ALLOC(r->var, mom);
#undef ALLOC
    if (hipMemcpy(d_rates, rates.data(), rates.size() * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(d_init, init.data(), init.size() * sizeof(int), hipMemcpyHostToDevice) !=
            hipSuccess) {
        free_run(r);
        return set_err(CWC_E_DEVICE, "table upload failed");
    }
    kp.seed = d->seed;
    kp.G = G;
    kp.R = R;
    kp.g_base = 0;
    kp.max_events = d->max_events;
    kp.dt = d->dt;
    kp.K1 = K1;
    kp.KR = kp.K1;          // one accumulator row per sample
    kp.k_base = 0;
    kp.k_stop = 0x7FFFFFFF; // no window: trajectories run to the horizon
    kp.k_slice = 0;
    kp.n_rows = nullptr;
    kp.cap = (unsigned)d->count_cap;
    kp.rate_stride = (d->rate_table && f.n_rules > 0) ? NR : 0;
    kp.init_stride = d->init_table ? C : 0;
    kp.want_traj = d->want_traj ? 1 : 0;
    kp.want_digest = d->want_digest ? 1 : 0;
    kp.rates = d_rates;
    kp.init = d_init;
    kp.chunk = tun.refill_chunk;
    kp.nslot = tun.sample_slots;
    if (d_order) {
        // Longest-first claim order (the paper's predictive scheduling of
        // instances, Sec. 5.2 schema ii): instances are claimed in
        // decreasing order of their total propensity at t = 0, a proxy for
        // their event count, so the heaviest start first and the queue's
        // tail holds the lightest.  Trajectory results do not depend on it.
        std::vector<int> order = instance_order(f, rates, init, (int)I, d->rate_table != nullptr,
                                                d->init_table != nullptr);
        if (hipMemcpy(d_order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice) !=
            hipSuccess) {
            free_run(r);
            return set_err(CWC_E_DEVICE, "order upload failed");
        }
        kp.order = d_order;
    }

    r->block = plan.block;
    r->grid = plan.grid;
    r->fn = plan.fn;
    r->kernel = plan.kernel;
    r->n_threads = plan.n_threads;
    r->lds = plan.lds;

    if (hipEventCreate(&r->ev_start) != hipSuccess || hipEventCreate(&r->ev_sim) != hipSuccess ||
        hipEventCreate(&r->ev_end) != hipSuccess) {
        free_run(r);
        return set_err(CWC_E_DEVICE, "hipEventCreate failed");
    }
    if (d->mode == CWC_MODE_PERSISTENT) {
        st = capture_graph(r);
        if (st != CWC_OK) {
            free_run(r);
            return st;
        }
    }
    st = launch(r, (hipStream_t)hip_stream);
    if (st != CWC_OK) {
        free_run(r);
        return st;
    }
    *out = r;
    return CWC_OK;
}

cwc_status cwc_run_relaunch(cwc_run *r, void *hip_stream)
{
    if (!r) return set_err(CWC_E_INVALID, "null run");
    return launch(r, (hipStream_t)hip_stream);
}

cwc_status cwc_run_query(cwc_run *r, int *done)
{
    if (!r || !done) return set_err(CWC_E_INVALID, "null argument");
    cwc_status st = ready(r);
    if (st == CWC_E_NOTREADY) {
        *done = 0;
        return CWC_OK;
    }
    if (st != CWC_OK) return st;
    *done = 1;
    return CWC_OK;
}

cwc_status cwc_run_wait(cwc_run *r)
{
    if (!r) return set_err(CWC_E_INVALID, "null run");
    if (!r->launched) return set_err(CWC_E_NOTREADY, "run not launched");
    HIPCHK(hipEventSynchronize(r->ev_end));
    return ready(r);
}

cwc_status cwc_run_wait_for(cwc_run *r, double timeout_s)
{
    if (!r) return set_err(CWC_E_INVALID, "null run");
    if (!r->launched) return set_err(CWC_E_NOTREADY, "run not launched");
    if (!(timeout_s >= 0)) return set_err(CWC_E_INVALID, "timeout_s must be >= 0");
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipEventQuery(r->ev_end);
        if (e == hipSuccess) return ready(r);
        if (e != hipErrorNotReady)
            return set_err(CWC_E_DEVICE, "run failed: %s", hipGetErrorString(e));
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (el >= timeout_s)
            return set_err(CWC_E_NOTREADY, "run still in flight after %.3f s", timeout_s);
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
}

cwc_status cwc_run_kernel_name(const cwc_run *r, char *buf, size_t cap, size_t *len)
{
    if (!r) return set_err(CWC_E_INVALID, "null run");
    if (len) *len = r->kernel.size() + 1;
    if (buf && cap >= r->kernel.size() + 1) std::memcpy(buf, r->kernel.c_str(), r->kernel.size() + 1);
    return CWC_OK;
}

cwc_status cwc_run_elapsed(cwc_run *r, float *sim_ms, float *total_ms)
{
    cwc_status st = ready(r);
    if (st != CWC_OK) return st;
    if (sim_ms) HIPCHK(hipEventElapsedTime(sim_ms, r->ev_start, r->ev_sim));
    if (total_ms) HIPCHK(hipEventElapsedTime(total_ms, r->ev_start, r->ev_end));
    return CWC_OK;
}

cwc_status cwc_run_fetch_stats(cwc_run *r, double *mean, double *var, int64_t *n,
                               int dst_is_device)
{
    cwc_status st = ready(r);
    if (st != CWC_OK) return st;
    const size_t mom = (size_t)r->I * r->K1 * r->C;
    if ((st = copy_out(mean, r->mean, mom * sizeof(double), dst_is_device))) return st;
    if ((st = copy_out(var, r->var, mom * sizeof(double), dst_is_device))) return st;
    return copy_out(n, r->nk, (size_t)r->I * r->K1 * sizeof(int64_t), dst_is_device);
}

cwc_status cwc_run_fetch_moments(cwc_run *r, uint64_t *s1, uint64_t *s2_hi32, uint64_t *s2_lo32,
                                 int64_t *n, int dst_is_device)
{
    cwc_status st = ready(r);
    if (st != CWC_OK) return st;
    const size_t mom = (size_t)r->I * r->K1 * r->C * sizeof(uint64_t);
    if ((st = copy_out(s1, r->kp.s1, mom, dst_is_device))) return st;
    if ((st = copy_out(s2_hi32, r->kp.s2_hi32, mom, dst_is_device))) return st;
    if ((st = copy_out(s2_lo32, r->kp.s2_lo32, mom, dst_is_device))) return st;
    return copy_out(n, r->nk, (size_t)r->I * r->K1 * sizeof(int64_t), dst_is_device);
}

cwc_status cwc_run_fetch_trajectories(cwc_run *r, int32_t *dst, int dst_is_device)
{
    cwc_status st = ready(r);
    if (st != CWC_OK) return st;
    if (!r->kp.traj) return set_err(CWC_E_INVALID, "run was submitted without want_traj");
    return copy_out(dst, r->kp.traj, (size_t)r->G * r->K1 * r->C * sizeof(int32_t), dst_is_device);
}

cwc_status cwc_run_fetch_term(cwc_run *r, int32_t *dst, int dst_is_device)
{
    cwc_status st = ready(r);
    if (st != CWC_OK) return st;
    if (!r->m->gen) return set_err(CWC_E_INVALID, "not a general model: its term is fixed");
    const GFlat &g = *r->m->gen;
    return copy_out(dst, r->kp.final_term,
                    (size_t)r->G * g.max_comp * (3 + 2 * g.n_species) * sizeof(int32_t),
                    dst_is_device);
}

cwc_status cwc_run_fetch_counters(cwc_run *r, int64_t *events, uint8_t *status, uint64_t *digest,
                                  double *t_final, int32_t *n_recorded, int32_t *final_counts,
                                  int dst_is_device)
{
    cwc_status st = ready(r);
    if (st != CWC_OK) return st;
    const size_t G = (size_t)r->G;
    if ((st = copy_out(events, r->kp.events, G * 8, dst_is_device))) return st;
    if ((st = copy_out(status, r->kp.status, G, dst_is_device))) return st;
    if ((st = copy_out(digest, r->kp.digest, G * 8, dst_is_device))) return st;
    if ((st = copy_out(t_final, r->kp.t_final, G * 8, dst_is_device))) return st;
    if ((st = copy_out(n_recorded, r->kp.n_recorded, G * 4, dst_is_device))) return st;
    return copy_out(final_counts, r->kp.final_counts, G * r->C * 4, dst_is_device);
}

void cwc_run_destroy(cwc_run *r) { free_run(r); }

cwc_status cwc_stats_finalize(cwc_ctx *ctx, const int64_t *n, const uint64_t *s1,
                              const uint64_t *s2_hi32, const uint64_t *s2_lo32, int64_t rows,
                              int32_t n_cells, double *mean, double *var, void *hip_stream)
{
    if (!ctx || !n || !s1 || !s2_hi32 || !s2_lo32 || !mean || !var || rows < 0 || n_cells < 1)
        return set_err(CWC_E_INVALID, "bad argument");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(launch_finalize((const long long *)n, (const unsigned long long *)s1,
                           (const unsigned long long *)s2_hi32,
                           (const unsigned long long *)s2_lo32, rows, n_cells, mean, var,
                           (hipStream_t)hip_stream));
    return CWC_OK;
}

}  // extern "C"
