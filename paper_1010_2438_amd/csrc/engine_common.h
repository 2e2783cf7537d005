// Device primitives shared by both layouts (compiled per model together with
// the generated model section and one of engine_lane.h / engine_wave.h):
// Philox4x32-10, the 53-bit uniforms and ssa_log.  Compiled with
// contraction of a*b+c into FMA disabled: every binary64 operation rounds
// once, matching the contract in include/cwcssa.h.

typedef unsigned int u32;
typedef unsigned long long u64;
typedef int i32;
typedef long long i64;

// Keeps an updated count in a register as an opaque value: the in-place
// update n += d of an event is undone on its rare slow path by n -= d, and
// without this the compiler would fold n + d - d back to n and keep both
// the old and the new count alive through every event (an extra copy of
// every count per event).  Emits no instruction.
#define CWC_KEEP(v) __asm__("" : "+v"(v))

#define CWC_ST_OK 0
#define CWC_ST_ABSORBED 1
#define CWC_ST_OVERFLOW 2
#define CWC_ST_EVENT_CAP 3
#define CWC_ST_RUNNING (-1)
// suspended before recording sample k_stop (the end of a streamed run's
// window); the trajectory resumes from its checkpoint in the next window
#define CWC_ST_WINDOW (-2)

// ------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// multiplies; the key advances by the Weyl constants between rounds.
__device__ __forceinline__ void cwc_philox(u32 c0, u32 c1, u32 c2, u32 c3,
                                           u32 k0, u32 k1, u32 &x0, u32 &x1,
                                           u32 &x2, u32 &x3)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        u64 p0 = (u64)0xD2511F53u * (u64)c0;
        u64 p1 = (u64)0xCD9E8D57u * (u64)c2;
        u32 n0 = (u32)(p1 >> 32) ^ c1 ^ k0;
        u32 n2 = (u32)(p0 >> 32) ^ c3 ^ k1;
        c1 = (u32)p1;
        c3 = (u32)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    x0 = c0; x1 = c1; x2 = c2; x3 = c3;
}

// 53 random bits -> binary64, exact: with m = a 2^21 + (b >> 11), the value
// (m + 1) 2^-53 (resp. m 2^-53) is a 2^-32 + ((b >> 11) + 1) 2^-53.  Both
// terms are exact, and so is their sum (an integer of at most 53 bits times
// 2^-53), so a fused multiply-add returns it without any rounding and
// without assembling m in 64-bit integer arithmetic.
__device__ __forceinline__ double cwc_u_open0(u32 a, u32 b)   // (0, 1]
{
    return __builtin_fma((double)a, 0x1p-32, (double)((b >> 11) + 1u) * 0x1p-53);
}
__device__ __forceinline__ double cwc_u_open1(u32 a, u32 b)   // [0, 1)
{
    return __builtin_fma((double)a, 0x1p-32, (double)(b >> 11) * 0x1p-53);
}

// ------------------------------------------------------------- ssa_log
// Natural logarithm on [2^-53, 1]: u = 2^E f exactly from the bits, f
// folded into [sqrt2/2, sqrt2]; ln f = 2 atanh(s), s = (f-1)/(f+1), as
// 2s + 2 s z p(z), z = s^2, p(z) = sum_{j=0..10} z^j / (2j+3) by Horner;
// ln u = E*LN2_HI + (E*LN2_LO + ln f) with LN2_HI holding 32 significant
// bits of ln 2 (E*LN2_HI exact).  Only correctly rounded + - * /.
__device__ __forceinline__ double cwc_ssa_log(double u)
{
    const double SQRT2 = __longlong_as_double(0x3FF6A09E667F3BCDll);
    const double LN2_HI = __longlong_as_double(0x3FE62E42FF000000ll);
    const double LN2_LO = __longlong_as_double((long long)0xBDC718432A1B0E26ull);
    u64 b = (u64)__double_as_longlong(u);
    int E = (int)((b >> 52) & 0x7FFull) - 1023;
    double f = __longlong_as_double((long long)((b & 0x000FFFFFFFFFFFFFull) |
                                                0x3FF0000000000000ull));
    bool big = f > SQRT2;
    f = big ? f * 0.5 : f;
    E = big ? E + 1 : E;
    double s = (f - 1.0) / (f + 1.0);
    double z = s * s;
    double p = 1.0 / 23.0;
    p = p * z; p = p + 1.0 / 21.0;
    p = p * z; p = p + 1.0 / 19.0;
    p = p * z; p = p + 1.0 / 17.0;
    p = p * z; p = p + 1.0 / 15.0;
    p = p * z; p = p + 1.0 / 13.0;
    p = p * z; p = p + 1.0 / 11.0;
    p = p * z; p = p + 1.0 / 9.0;
    p = p * z; p = p + 1.0 / 7.0;
    p = p * z; p = p + 1.0 / 5.0;
    p = p * z; p = p + 1.0 / 3.0;
    double t = z * p;
    t = s * t;
    double lnf = (2.0 * s) + (2.0 * t);
    double Ed = (double)E;
    double lo = Ed * LN2_LO;
    lo = lo + lnf;
    double hi = Ed * LN2_HI;
    return hi + lo;
}

