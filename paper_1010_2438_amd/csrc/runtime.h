// Internal definitions of the opaque C-ABI objects.
#ifndef CWC_RUNTIME_H
#define CWC_RUNTIME_H
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cwcssa.h"
#include "kparams.h"
#include "gmodel.h"
#include "model.h"

struct cwc_ctx {
    int device = 0;
    int n_cu = 0;
    size_t max_lds = 65536;             // dynamic LDS bytes a lane-layout block may allocate
    std::string arch;
    void *arena = nullptr;
    size_t arena_bytes = 0;
    size_t used = 0;
    std::map<size_t, size_t> free_blocks;     // arena offset -> size
    std::map<void *, size_t> sizes;           // live allocations
    std::mutex mu;
    hipStream_t capture_stream = nullptr;
    void *scratch = nullptr;            // this device's no-allocation scratch array
    // models, runs and servers hold the context: cwc_ctx_destroy marks it
    // closed and it is freed when the last of them is destroyed
    std::atomic<int> refs{0};
    bool closed = false;                // guarded by mu
    void *alloc(size_t bytes, cwc_status *st);
    void release(void *p);
};

namespace cwc {
void ctx_retain(cwc_ctx *ctx);
void ctx_drop(cwc_ctx *ctx);            // frees a closed context at the last drop
void ctx_drop_final(cwc_ctx *ctx);
}  // namespace cwc

struct cwc_model {
    cwc_ctx *ctx = nullptr;
    cwc::Flat flat;                     // flat.layout = the default layout
    int fits[3] = {0, 0, 0};            // layouts the model fits (lane, wave, general)
    std::string source[3];              // per layout, generated on demand
    hipModule_t module[3] = {nullptr, nullptr, nullptr};
    hipFunction_t fn[3][8] = {};        // [layout][plain/persistent/slice/resident x
                                        // shared/table]
    std::shared_ptr<cwc::GFlat> gen;    // general models (layout 2): the term and rules
    hipFunction_t quad_fn[4] = {};      // lane module's quad kernels (plain/persistent x
                                        // shared/table); null with fewer than four leaves
    hipFunction_t pair_fn[8] = {};      // lane module's pair kernels (plain/persistent/
                                        // slice/resident x shared/table); null with one leaf
    double *d_k = nullptr;              // device copies of the model's kinetic
    int *d_init = nullptr;              // constants and initial counts
    std::mutex mu;
};

namespace cwc {
// Dynamic LDS bytes of a lane-layout launch with `waves` wavefronts per
// block and `nslot` accumulator rows per wavefront: per wavefront a
// [cell][lane] int32 staging area and the accumulator cache of
// engine_lane.h (nslot tags + nslot x C x 2 sums, 64-bit).
inline size_t cwc_lane_lds_bytes(int n_cells, int waves, int nslot)
{
    return (size_t)waves * ((size_t)n_cells * 64 * 4 + (size_t)nslot * 8 +
                            2 * (size_t)nslot * (size_t)n_cells * 8);
}
constexpr int kDefaultSampleSlots = 16;
// static LDS of a lane-group kernel: the per-leaf (lane layout) or
// per-lane (pair and quad layouts) change table, and in the resident
// kernels the copies of the job parameters of a block's four wavefronts
constexpr size_t kLaneStaticLds =
    std::max(std::max(kLaneStaticLdsBytes, kPairStaticLdsBytes), kQuadStaticLdsBytes) +
    4 * sizeof(cwc_kparams);
// Compiles and loads the model's device code for `layout` if needed.
cwc_status ensure_layout(cwc_model *m, int layout);
// Directory of the compiled-code cache and the tuning table (created).
std::string cache_dir_path();
// Stored tuning for this model and run, if the autotuner recorded one.
bool tuning_lookup(const cwc_model *m, const cwc_run_desc *d, cwc_tuning *out);
// Checks a run descriptor; host copies of the rate / initial-state tables.
cwc_status validate_run(const cwc_model *m, const cwc_run_desc *d, std::vector<double> *rates,
                        std::vector<int> *init);
// Checks the scalar fields of a run descriptor (sizes, sample grid, caps).
cwc_status validate_run_sizes(const cwc_run_desc *d);
// Whether the model's code for `layout` is compiled and loaded.
bool layout_loaded(const cwc_model *m, int layout);
// Total propensity of each instance's initial state (host, for scheduling
// only) and the instance order by decreasing value.
std::vector<int> instance_order(const Flat &f, const std::vector<double> &rates,
                                const std::vector<int> &init, int I, bool rate_rows,
                                bool init_rows);
// Launch shape of a run (see run.cpp).
struct LaunchPlan {
    cwc_tuning tun{};                   // as launched
    int layout = 0, group = 1;          // module; lanes per trajectory
    hipFunction_t fn = nullptr;
    std::string kernel;
    unsigned grid = 0, block = 0, lds = 0;
    unsigned long long n_threads = 0;   // trajectory slots of the grid
};
cwc_status plan_launch(cwc_ctx *ctx, const cwc_model *m, const cwc_run_desc *d, cwc_tuning tun,
                       bool tuned, bool may_compile, LaunchPlan *out);
// Device address of the no-allocation entry point's scratch array on the
// current device (looked up once per device).
cwc_status scratch_address(int device, void **ptr);
}

struct cwc_run {
    cwc_ctx *ctx = nullptr;
    const cwc_model *m = nullptr;
    long long I = 0, R = 0, G = 0;
    int K1 = 0, C = 0, mode = 0;
    cwc_tuning tun{};
    cwc_kparams kp{};
    std::string kernel;                  // name of the simulation kernel dispatched
    hipFunction_t fn = nullptr;
    unsigned grid = 0, block = 0;
    unsigned lds = 0;                   // dynamic LDS bytes per block
    unsigned long long n_threads = 0;
    // device buffers
    std::vector<void *> bufs;
    long long *nk = nullptr;
    double *mean = nullptr, *var = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev_start = nullptr, ev_sim = nullptr, ev_end = nullptr;
    hipGraphExec_t graph = nullptr;
    bool launched = false;
};

namespace cwc {
extern thread_local std::string g_err;
cwc_status set_err(cwc_status code, const char *fmt, ...);
cwc_status compile_source(const std::string &src, const std::string &arch,
                          std::vector<char> *code);
std::string model_source(const Flat &f, int layout);
std::string gmodel_source(const GFlat &g);
// A non-blocking stream with a hardware queue of its own (created with a
// compute-unit mask covering the whole device, which the runtime serves
// from a queue of its own instead of one shared round-robin with the
// process's other streams): work on it never waits behind a long kernel
// on another stream.  Falls back to an ordinary non-blocking stream where
// the runtime has no masked streams.
bool own_queue_stream(cwc_ctx *ctx, hipStream_t *st);
}  // namespace cwc
#endif
