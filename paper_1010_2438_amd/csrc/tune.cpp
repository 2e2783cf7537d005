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

std::string table_path() { return cache_dir_path() + "/tuning.txt"; }

std::string tune_key(const cwc_model *m, const cwc_run_desc *d)
{
    const long long G = d->n_instances * d->replicas_per_instance;
    int lg = 0;
    while ((1ll << (lg + 1)) <= G) ++lg;
    char b[160];
    std::snprintf(b, sizeof b, "%016llx_m%d_t%d_g%d",
                  (unsigned long long)hash_str(model_source(m->flat, m->flat.layout)), d->mode,
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
        if (!(is >> k >> t.block_size >> t.waves_per_simd >> t.refill_chunk >> t.lanes_per_replica))
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
      << " " << t.lanes_per_replica << " " << ms << "\n";
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
    std::vector<cwc_tuning> cands;
    const int layouts[2] = {0, 1};
    for (int lay : layouts) {
        if (!m->fits[lay]) continue;
        for (int bs : {64, 128, 256}) {
            if (d->mode == CWC_MODE_PERSISTENT) {
                for (int wps : {1, 2, 4}) cands.push_back(cwc_tuning{bs, wps, 0, lay ? 64 : 1});
            } else {
                cands.push_back(cwc_tuning{bs, 2, 0, lay ? 64 : 1});
            }
        }
    }
    // probe the default shape on a short horizon to size the trials
    cwc_run_desc probe = *d;
    cwc_status st = CWC_OK;
    const int K1 = d->n_samples;
    probe.n_samples = std::max(2, K1 / 16);
    double ms = trial(ctx, m, probe, cands[0], &st);
    if (ms < 0) return st;
    const double per_unit = ms / (double)(probe.n_samples - 1);      // per sample interval
    const double target = 1e3 * budget_s / (double)cands.size();
    int k1 = (int)std::floor(target / std::max(per_unit, 1e-6)) + 1;
    k1 = std::max(2, std::min(K1, k1));
    cwc_run_desc td = *d;
    td.n_samples = k1;
    double best = 1e300;
    cwc_tuning bt = cands[0];
    for (const cwc_tuning &c : cands) {
        double t = trial(ctx, m, td, c, &st);
        if (t < 0) return st;
        if (t < best) {
            best = t;
            bt = c;
        }
    }
    tuning_store(m, d, bt, best);
    *out = bt;
    return CWC_OK;
}
