// The no-allocation run entry point (cwc_run_into) and its scratch memory.
//
// A run's intermediate device state -- the exact moment accumulators per
// (instance, sample, cell), the recorded-count histogram per (instance,
// sample) and the work-queue cursor -- lives here in one statically
// allocated device array per GPU instead of buffers allocated per run, so a
// caller that cannot allocate device memory can still run the whole path:
// it passes device tables and device outputs, the library enqueues the fill
// kernels, the simulation kernel and the two finalisation kernels on its
// stream, and nothing is allocated or freed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/cwcssa.h"
#include "runtime.h"
#include "stats.h"

using namespace cwc;

// Every GPU the library runs on holds its own copy until the process ends.
// Host code never uses this name as an address: the per-device address comes
// from hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) unsigned char scratch[CWC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }
}  // namespace

namespace cwc {

// Called by cwc_ctx_create with `device` current: looks up this device's
// address of the scratch array once and keeps it.
cwc_status scratch_address(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices)
        return set_err(CWC_E_INVALID, "device %d beyond the scratch table", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_err(CWC_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                           hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return CWC_OK;
}

}  // namespace cwc

#define HIPCHK(call)                                                               \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return set_err(CWC_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

extern "C" cwc_status cwc_run_into(cwc_ctx *ctx, const cwc_model *m, const cwc_run_desc *d,
                                   const cwc_run_outputs *o, void *hip_stream)
{
    if (!ctx || !m || !d || !o) return set_err(CWC_E_INVALID, "null argument");
    if (m->ctx != ctx) return set_err(CWC_E_INVALID, "model belongs to another context");
    if (d->mode != CWC_MODE_PLAIN && d->mode != CWC_MODE_PERSISTENT)
        return set_err(CWC_E_INVALID, "unknown mode %d", d->mode);
    if (d->want_traj)
        return set_err(CWC_E_INVALID, "cwc_run_into keeps no trajectories: want_traj must be 0");
    if (!o->mean || !o->var || !o->n || !o->events || !o->status || !o->digest || !o->t_final ||
        !o->n_recorded || !o->final_counts)
        return set_err(CWC_E_INVALID, "every output pointer must be set");
    {
        cwc_status st = validate_run_sizes(d);
        if (st != CWC_OK) return st;
    }
    if (!ctx->scratch) return set_err(CWC_E_DEVICE, "no scratch array on this device");
    const Flat &f = m->flat;
    const long long I = d->n_instances, R = d->replicas_per_instance, G = I * R;
    const int C = f.n_cells, K1 = d->n_samples;

    // scratch regions: S1, S2 high and low halves [I][K1][C] u64, the
    // recorded-count histogram [I][K1+1] u64, the queue cursor
    const size_t mom = (size_t)I * (size_t)K1 * (size_t)C;
    const size_t b_mom = align256(mom * 8), b_hist = align256((size_t)I * (K1 + 1) * 8);
    const size_t need = 3 * b_mom + b_hist + 256;
    if (mom > ((size_t)1 << 40) || need > (size_t)CWC_NOALLOC_SCRATCH_BYTES)
        return set_err(CWC_E_NOMEM,
                       "the run needs %zu bytes of scratch (24 bytes per instance, sample and "
                       "cell, 8 per instance and sample), more than the %zu bytes of "
                       "cwc_run_into; use cwc_run_submit",
                       need, (size_t)CWC_NOALLOC_SCRATCH_BYTES);

    const cwc_tuning tun = d->tuning ? *d->tuning : cwc_tuning{};
    LaunchPlan plan;
    {
        cwc_status st = plan_launch(ctx, m, d, tun, false, false, &plan);
        if (st != CWC_OK) return st;
    }

    unsigned char *base = (unsigned char *)ctx->scratch;
    cwc_kparams kp{};
    kp.s1 = (unsigned long long *)base;
    kp.s2_hi32 = (unsigned long long *)(base + b_mom);
    kp.s2_lo32 = (unsigned long long *)(base + 2 * b_mom);
    kp.rec_hist = (unsigned long long *)(base + 3 * b_mom);
    kp.cursor = (unsigned long long *)(base + 3 * b_mom + b_hist);
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
    const bool rate_rows = d->rate_table && f.n_rules > 0;
    kp.rate_stride = rate_rows ? f.n_rules : 0;
    kp.rates = rate_rows ? d->rate_table : m->d_k;
    kp.init_stride = d->init_table ? C : 0;
    kp.init = d->init_table ? d->init_table : m->d_init;
    kp.want_traj = 0;
    kp.want_digest = d->want_digest ? 1 : 0;
    kp.final_counts = o->final_counts;
    kp.events = (long long *)o->events;
    kp.t_final = o->t_final;
    kp.digest = (unsigned long long *)o->digest;
    kp.status = o->status;
    kp.n_recorded = o->n_recorded;
    kp.traj = nullptr;
    kp.order = nullptr;                     // natural order
    kp.chunk = plan.tun.refill_chunk;
    kp.nslot = plan.tun.sample_slots;

    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(hipSetDevice(ctx->device));
    // the array keeps the previous call's contents: clear what starts at 0
    HIPCHK(launch_fill_u64(kp.s1, 0, (long long)mom, s));
    HIPCHK(launch_fill_u64(kp.s2_hi32, 0, (long long)mom, s));
    HIPCHK(launch_fill_u64(kp.s2_lo32, 0, (long long)mom, s));
    HIPCHK(launch_fill_u64(kp.rec_hist, 0, I * (long long)(K1 + 1), s));
    HIPCHK(launch_fill_u64(kp.cursor, plan.n_threads, 1, s));
    void *args[] = {&kp};
    HIPCHK(hipModuleLaunchKernel(plan.fn, plan.grid, 1, 1, plan.block, 1, 1, plan.lds, s, args,
                                 nullptr));
    HIPCHK(launch_hist_to_n(kp.rec_hist, (long long *)o->n, I, K1, s));
    HIPCHK(launch_finalize((const long long *)o->n, kp.s1, kp.s2_hi32, kp.s2_lo32,
                           I * (long long)K1, C, o->mean, o->var, s));
    return CWC_OK;
}
