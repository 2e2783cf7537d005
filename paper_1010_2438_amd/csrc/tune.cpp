// Autotuner: picks the launch shape of a run by timing candidates on the
// run's own inputs over a shortened horizon, and keeps the choice in a
// small on-disk table (one line per key) next to the compiled-code cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/cwcssa.h"
#include "runtime.h"

using namespace cwc;

namespace {

std::mutex g_tune_mu;

uint64_t hash_str(const std::string &s)
{
    uint64_t h = 0xcbf29ce484222325ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 0x100000001b3ull;
    }
    return h;
}

// one line per key: key block waves_per_simd refill_chunk lanes_per_replica
// sample_slots milliseconds
std::string table_path() { return cache_dir_path() + "/tuning_v2.txt"; }

std::string tune_key(const cwc_model *m, const cwc_run_desc *d)
{
    const long long G = d->n_instances * d->replicas_per_instance;
    int lg = 0;
    while ((1ll << (lg + 1)) <= G) ++lg;
    char b[160];
    std::snprintf(b, sizeof b, "%016llx_m%d_t%d_g%d",
                  (unsigned long long)hash_str(m->gen ? gmodel_source(*m->gen)
                                                      : model_source(m->flat, m->flat.layout)),
                  d->mode,
                  d->rate_table ? 1 : 0, lg);
    return b;
}

}  // namespace

namespace cwc {

bool tuning_lookup(const cwc_model *m, const cwc_run_desc *d, cwc_tuning *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::ifstream f(table_path());
    if (!f) return false;
    const std::string key = tune_key(m, d);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        cwc_tuning t{};
        if (!(is >> k >> t.block_size >> t.waves_per_simd >> t.refill_chunk >> t.lanes_per_replica >>
              t.sample_slots))
            continue;
        if (k == key) {
            *out = t;                       // the last entry for a key wins
            found = true;
        }
    }
    return found;
}

}  // namespace cwc

namespace {

void tuning_store(const cwc_model *m, const cwc_run_desc *d, const cwc_tuning &t, double ms)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::ofstream f(table_path(), std::ios::app);
    if (!f) return;
    f << tune_key(m, d) << " " << t.block_size << " " << t.waves_per_simd << " " << t.refill_chunk
      << " " << t.lanes_per_replica << " " << t.sample_slots << " " << ms << "\n";
}

// Runs the descriptor once with tuning t; kernel milliseconds or < 0.
double trial(cwc_ctx *ctx, const cwc_model *m, const cwc_run_desc &d, const cwc_tuning &t,
             cwc_status *st)
{
    cwc_run_desc dd = d;
    dd.tuning = &t;
    dd.want_traj = 0;
    cwc_run *r = nullptr;
    *st = cwc_run_submit(ctx, m, &dd, nullptr, &r);
    if (*st != CWC_OK) return -1.0;
    *st = cwc_run_wait(r);
    float sim = 0, tot = 0;
    if (*st == CWC_OK) *st = cwc_run_elapsed(r, &sim, &tot);
    cwc_run_destroy(r);
    return *st == CWC_OK ? (double)sim : -1.0;
}

}  // namespace

extern "C" cwc_status cwc_autotune(cwc_ctx *ctx, const cwc_model *m, const cwc_run_desc *d,
                                   double budget_s, cwc_tuning *out)
{
    if (!ctx || !m || !d || !out) return set_err(CWC_E_INVALID, "null argument");
    if (!(budget_s > 0)) return set_err(CWC_E_INVALID, "budget_s must be > 0");
    if (m->gen) {
        // one layout: one wavefront per trajectory; only the block varies
        // little, so the library's choice stands
        *out = cwc_tuning{};
        out->block_size = 256;
        out->waves_per_simd = 8;
        out->lanes_per_replica = 64;
        return CWC_OK;
    }
    const bool persistent = d->mode == CWC_MODE_PERSISTENT;
    const int C = m->flat.n_cells;
    // stage 1 and 2 candidates: layout x block shape (x resident waves)
    // lanes per trajectory: 1, 2 (two or more leaves) and 4 (four or more)
    // in the lane layout's module, 64 in the wavefront layout
    std::vector<int> lprs;
    if (m->fits[0]) {
        lprs.push_back(1);
        if (m->flat.n_leaves >= 2) lprs.push_back(2);
        if (m->flat.n_leaves >= 4) lprs.push_back(4);
    }
    if (m->fits[1]) lprs.push_back(64);
    // The first shape of each layout is its strongest guess (largest block,
    // most waves), which stage 1 uses to compare the layouts.
    std::vector<cwc_tuning> cands;
    for (int lpr : lprs) {
        for (int bs : {256, 128, 64}) {
            if (persistent) {
                // up to 16 requested waves per SIMD: beyond what fits, the
                // extra blocks wait for the hardware dispatcher, and a grid
                // that holds every item runs the queue-free kernel (items
                // still longest-first), often the fastest for sweeps
                for (int wps : {16, 8, 4, 2, 1}) cands.push_back(cwc_tuning{bs, wps, 0, lpr, 0});
            } else {
                cands.push_back(cwc_tuning{bs, 2, 0, lpr, 0});
            }
        }
    }
    if (cands.empty()) return set_err(CWC_E_UNSUPPORTED, "model fits no layout");
    // lane layout, stage 3: sampling-buffer depths that fit in LDS
    std::vector<int> depths;
    for (int ds : {4, 64})
        if (cwc_lane_lds_bytes(C, 1, ds) <= ctx->max_lds) depths.push_back(ds);
    // stage 4 (persistent lane layout): refill chunk
    const std::vector<int> chunks = {1, 256};
    const size_t n_trials = cands.size() + depths.size() + (persistent ? chunks.size() : 0);

    // probe the default shape on a short horizon to size the trials
    cwc_run_desc probe = *d;
    cwc_status st = CWC_OK;
    const int K1 = d->n_samples;
    probe.n_samples = std::max(2, K1 / 16);
    double ms = trial(ctx, m, probe, cands[0], &st);
    if (ms < 0) return st;
    const double per_unit = ms / (double)(probe.n_samples - 1);      // per sample interval
    const double target = 1e3 * budget_s / (double)n_trials;
    int k1 = (int)std::floor(target / std::max(per_unit, 1e-6)) + 1;
    k1 = std::max(2, std::min(K1, k1));
    cwc_run_desc td = *d;
    td.n_samples = k1;

    // stage 1: the first shape of each layout (lanes per trajectory); a
    // layout more than 1.5x slower than the fastest one is not searched
    // further
    auto layout_of = [](const cwc_tuning &c) {
        switch (c.lanes_per_replica) {
        case 64: return 3;
        case 4: return 2;
        case 2: return 1;
        default: return 0;
        }
    };
    double lay_ms[4] = {-1.0, -1.0, -1.0, -1.0};
    size_t lay_first[4] = {cands.size(), cands.size(), cands.size(), cands.size()};
    for (size_t i = 0; i < cands.size(); ++i) {
        const int lay = layout_of(cands[i]);
        if (lay_first[lay] != cands.size()) continue;
        lay_first[lay] = i;
        lay_ms[lay] = trial(ctx, m, td, cands[i], &st);
        if (lay_ms[lay] < 0) return st;
    }
    double fastest = 1e300;
    for (int l = 0; l < 4; ++l)
        if (lay_ms[l] >= 0) fastest = std::min(fastest, lay_ms[l]);
    // stage 2: every shape of the remaining layouts
    double best = 1e300;
    cwc_tuning bt = cands[0];
    auto consider = [&](const cwc_tuning &c, double t) {
        if (t < best) {
            best = t;
            bt = c;
        }
    };
    for (size_t i = 0; i < cands.size(); ++i) {
        const int lay = layout_of(cands[i]);
        if (lay_ms[lay] > 1.5 * fastest) continue;
        double t = i == lay_first[lay] ? lay_ms[lay] : trial(ctx, m, td, cands[i], &st);
        if (t < 0) return st;
        consider(cands[i], t);
    }
    if (layout_of(bt) != 3) {
        // stages 3 and 4 move away from the defaults (16 accumulator rows,
        // chunks of 64) only for a gain above the trials' noise (1 %)
        auto consider_clear = [&](const cwc_tuning &c, double t) {
            if (t < 0.99 * best) {
                best = t;
                bt = c;
            }
        };
        // stage 3: sampling-buffer depth for the best shape
        const cwc_tuning shape = bt;
        for (int ds : depths) {
            cwc_tuning c = shape;
            c.sample_slots = ds;
            double t = trial(ctx, m, td, c, &st);
            if (t < 0) return st;
            consider_clear(c, t);
        }
        // stage 4: queue refill granularity
        if (persistent) {
            const cwc_tuning base = bt;
            for (int ch : chunks) {
                cwc_tuning c = base;
                c.refill_chunk = ch;
                double t = trial(ctx, m, td, c, &st);
                if (t < 0) return st;
                consider_clear(c, t);
            }
        }
    }
    tuning_store(m, d, bt, best);
    *out = bt;
    return CWC_OK;
}
