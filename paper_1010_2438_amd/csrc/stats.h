// Host launchers for the model-independent library kernels (stats.hip).
#ifndef CWC_STATS_H
#define CWC_STATS_H
#include <hip/hip_runtime.h>

namespace cwc {
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, long long n,
                           hipStream_t s);
hipError_t launch_hist_to_n(const unsigned long long *hist, long long *n, long long n_inst,
                            int K1, hipStream_t s);
hipError_t launch_finalize(const long long *n, const unsigned long long *s1,
                           const unsigned long long *s2_hi32,
                           const unsigned long long *s2_lo32, long long rows, int C,
                           double *mean, double *var, hipStream_t s);
}  // namespace cwc
#endif
