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

// ------------------------------------------------- resident serving kernels
// A resident kernel stays on the device while the host keeps publishing
// (job, trajectory) items: each wavefront claims the next item, copies its
// job's parameters, runs the item's trajectories to their end, counts them
// toward the job and claims again, until the host asks it to stop or no
// item has come for a while.

// Claims the next item for the calling wavefront (lane 0 claims; the result
// is the same in every lane).  False once the host has asked for a stop,
// or when no item has been published for q.idle_ticks of wall-clock time.
// The acquire load of the host's tail orders the item's words and
// everything the host made visible before publishing it (the job's tables,
// zeroed accumulators, its parameters) before this wavefront's next loads.
__device__ __forceinline__ bool cwc_rq_claim(const cwc_rq &q, int &slot, i64 &first, i64 &job)
{
    i64 s = -1, f = 0, id = 0;
    if (__lane_id() == 0) {
        const u64 t0 = wall_clock64();
        for (;;) {
            if (__hip_atomic_load(q.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) break;
            u64 h = __hip_atomic_load(q.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const i64 t = __hip_atomic_load(q.tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
            if ((i64)h < t) {
                // another wavefront may take item h first: then try again
                // at once (every failure is some wavefront's claim)
                if (__hip_atomic_compare_exchange_strong(q.head, &h, h + 1ull, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)) {
                    const i64 *it = q.items + CWC_RQ_ITEM * (i64)(h & (u64)q.mask);
                    s = __hip_atomic_load(it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    f = __hip_atomic_load(it + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    id = __hip_atomic_load(it + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    break;
                }
                continue;
            }
            if ((i64)(wall_clock64() - t0) > q.idle_ticks) break;
            __builtin_amdgcn_s_sleep(127);
        }
    }
    s = __shfl(s, 0);
    f = __shfl(f, 0);
    id = __shfl(id, 0);
    slot = (int)s;
    first = f;
    job = id;
    return s >= 0;
}

// Copies a job's parameters into the wavefront's LDS copy with loads that
// bypass the caches: a slot's parameters change between jobs while the
// kernel runs.
__device__ __forceinline__ void cwc_rq_params(cwc_kparams *dst, const cwc_kparams *src)
{
    constexpr int W = (int)(sizeof(cwc_kparams) / sizeof(u32));
    const u32 *s = (const u32 *)src;
    u32 *d = (u32 *)dst;
    for (int i = (int)__lane_id(); i < W; i += 64)
        d[i] = __hip_atomic_load(s + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// After an item: its n finished trajectories count toward the job once
// their results are visible device-wide (release); the wavefront whose
// count completes the job publishes the job's id to the host.
__device__ __forceinline__ void cwc_rq_finish(const cwc_rq &q, const cwc_kparams &p, int slot,
                                              i64 job, u32 n)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (__lane_id() == 0 && n) {
        const u64 old = __hip_atomic_fetch_add(p.done_count, (u64)n, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
        if (old + n == (u64)p.G)
            __hip_atomic_store(q.done + slot, job, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

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

