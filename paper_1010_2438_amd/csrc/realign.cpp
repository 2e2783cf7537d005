// Realignment of trajectories recorded at their own times onto the fixed
// sample grid (paper Sec. 5.2, schema i: trajectories sampled at fixed
// simulation-time steps make the on-line reduction simple; data recorded
// otherwise can be realigned while it is buffered).  The state of a
// stochastic simulation is piecewise constant and right-continuous, so the
// value on the grid at t_k = k dt is the last recorded state whose time is
// <= t_k -- the convention the kernels' own sampling follows.  Host-side.
#include <cmath>
#include <cstdint>

#include "../../include/cwcssa.h"
#include "runtime.h"

using namespace cwc;

extern "C" cwc_status cwc_realign(const double *times, const int32_t *values, int64_t n,
                                  int32_t n_cells, double dt, int32_t n_samples, int32_t fill,
                                  int32_t *out)
{
    if (n < 0 || n_cells < 1 || n_samples < 0) return set_err(CWC_E_INVALID, "bad sizes");
    if ((n > 0 && (!times || !values)) || (n_samples > 0 && !out))
        return set_err(CWC_E_INVALID, "null array");
    if (!(std::isfinite(dt) && dt > 0.0)) return set_err(CWC_E_INVALID, "dt must be finite and > 0");
    for (int64_t i = 0; i < n; ++i) {
        if (std::isnan(times[i])) return set_err(CWC_E_INVALID, "time %lld is NaN", (long long)i);
        if (i > 0 && times[i] < times[i - 1])
            return set_err(CWC_E_INVALID, "times must be non-decreasing (index %lld)",
                           (long long)i);
    }
    int64_t j = -1;   // last record with time <= t_k
    for (int32_t k = 0; k < n_samples; ++k) {
        const double tk = (double)k * dt;
        while (j + 1 < n && times[j + 1] <= tk) ++j;
        int32_t *row = out + (int64_t)k * n_cells;
        if (j < 0) {
            for (int32_t c = 0; c < n_cells; ++c) row[c] = fill;
        } else {
            const int32_t *v = values + j * (int64_t)n_cells;
            for (int32_t c = 0; c < n_cells; ++c) row[c] = v[c];
        }
    }
    return CWC_OK;
}
