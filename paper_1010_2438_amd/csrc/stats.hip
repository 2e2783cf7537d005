// Library kernels that do not depend on the model: buffer fills, the
// contributor count per (instance, sample) and the finalisation of exact
// moments into mean and unbiased variance (paper Sec. 3 and Sec. 5.2: the
// instances' trajectories are averaged at fixed sample times, with variance).
#include <hip/hip_runtime.h>

#include "stats.h"

typedef unsigned long long u64;
typedef long long i64;

__global__ void cwc_k_fill_u64(u64 *p, u64 v, i64 n)
{
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (i64)gridDim.x * blockDim.x)
        p[i] = v;
}

// n[i][k] = number of trajectories of instance i that recorded sample k,
// i.e. whose recorded-sample count exceeds k (suffix sum of the histogram).
__global__ void cwc_k_hist_to_n(const u64 *hist, i64 *n, i64 n_inst, int K1)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    const u64 *h = hist + i * (i64)(K1 + 1);
    u64 acc = h[K1];
    for (int k = K1 - 1; k >= 0; --k) {
        n[i * K1 + k] = (i64)acc;
        acc += h[k];
    }
}

struct u128 {
    u64 hi, lo;
};

__device__ __forceinline__ u128 mul64(u64 a, u64 b)
{
    return u128{__umul64hi(a, b), a * b};
}

__device__ __forceinline__ u128 sub128(u128 a, u128 b)
{
    u128 r;
    r.lo = a.lo - b.lo;
    r.hi = a.hi - b.hi - (a.lo < b.lo ? 1ull : 0ull);
    return r;
}

// Correctly rounded (nearest, ties to even) conversion of a 128-bit
// unsigned integer to binary64.
__device__ __forceinline__ double u128_to_f64(u128 v)
{
    if (v.hi == 0) return (double)v.lo;     // single rounding of hi*2^32 + lo
    const int s = __clzll((long long)v.hi);             // 0..63
    const u64 top = s ? ((v.hi << s) | (v.lo >> (64 - s))) : v.hi;
    const u64 rest = s ? (v.lo << s) : v.lo;
    u64 mant = top >> 11;                              // 53 bits, MSB set
    const u64 rb = top & 0x7FFull;
    const bool sticky = rest != 0;
    const bool up = rb > 0x400ull || (rb == 0x400ull && (sticky || (mant & 1ull)));
    mant += up ? 1ull : 0ull;                          // may reach 2^53: exact
    return ldexp((double)mant, 11 + 64 - s);
}

// mean = S1 / n; var = (n S2 - S1^2) / (n (n-1)), numerator exact in 128
// bits and rounded once; NaN for n < 1 (mean) and n < 2 (var).
// S2 = s2_hi32 * 2^32 + s2_lo32.
__global__ void cwc_k_finalize(const i64 *n, const u64 *s1, const u64 *s2_hi32,
                               const u64 *s2_lo32, i64 rows, int C,
                               double *mean, double *var)
{
    const i64 total = rows * (i64)C;
    for (i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (i64)gridDim.x * blockDim.x) {
        const u64 nn = (u64)n[idx / C];
        const double qnan = __longlong_as_double(0x7FF8000000000000ll);
        if (nn == 0) {
            mean[idx] = qnan;
            var[idx] = qnan;
            continue;
        }
        const u64 S1 = s1[idx];
        mean[idx] = (double)S1 / (double)nn;
        if (nn < 2) {
            var[idx] = qnan;
            continue;
        }
        const u64 hs = s2_hi32[idx], ls = s2_lo32[idx];
        // S2 = hs*2^32 + ls as 128 bits
        u128 S2;
        S2.lo = (hs << 32) + ls;
        S2.hi = (hs >> 32) + (S2.lo < ls ? 1ull : 0ull);
        // n * S2 (fits in 128 bits for n < 2^32)
        u128 a = mul64(nn, S2.lo);
        a.hi += nn * S2.hi;
        const u128 b = mul64(S1, S1);
        const u128 num = sub128(a, b);
        const double den = (double)(nn * (nn - 1ull));
        var[idx] = u128_to_f64(num) / den;
    }
}

namespace cwc {

static int blocks_for(i64 n, int bs)
{
    i64 b = (n + bs - 1) / bs;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (int)b;
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, long long n,
                           hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    (void)hipGetLastError();    // report this launch's error, not an earlier one
    hipLaunchKernelGGL(cwc_k_fill_u64, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_hist_to_n(const unsigned long long *hist, long long *n, long long n_inst,
                            int K1, hipStream_t s)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(cwc_k_hist_to_n, dim3(blocks_for(n_inst, 64)), dim3(64), 0, s, hist, n,
                       n_inst, K1);
    return hipGetLastError();
}

hipError_t launch_finalize(const long long *n, const unsigned long long *s1,
                           const unsigned long long *s2_hi32,
                           const unsigned long long *s2_lo32, long long rows, int C,
                           double *mean, double *var, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(cwc_k_finalize, dim3(blocks_for(rows * C, 256)), dim3(256), 0, s, n, s1,
                       s2_hi32, s2_lo32, rows, C, mean, var);
    return hipGetLastError();
}

}  // namespace cwc
