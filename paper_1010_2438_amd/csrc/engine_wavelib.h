// Wavefront helpers shared by the engines that run one trajectory per
// wavefront (engine_wave.h: fixed compartment trees; engine_gen.h: general
// terms): lane reads and the butterfly that forms the compartment levels of
// the propensity tree.

__device__ __forceinline__ double cwc_rl(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Butterfly partner of level l (1..6) for a value that is uniform within
// each block of 2^(l-1) lanes: any lane of the sibling block will do, since
// the sum of the two blocks is the same in either order (IEEE addition
// commutes).  Levels 1-4 stay inside a row of 16 lanes (DPP: quad
// permutations, half-row and row mirrors); levels 5 and 6 use the row swaps
// of gfx950 (permlane16/permlane32 swap), which hand back both halves, so
// the level's sum is formed from the pair directly.
template <int CTRL>
__device__ __forceinline__ double cwc_dpp(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double cwc_bfly_sum(double v, int level)
{
    switch (level) {
    case 1: return v + cwc_dpp<0xB1>(v);     // quad_perm [1,0,3,2]: lane ^ 1
    case 2: return v + cwc_dpp<0x4E>(v);     // quad_perm [2,3,0,1]: lane ^ 2
    case 3: return v + cwc_dpp<0x141>(v);    // row_half_mirror: 7 - lane in 8
    case 4: return v + cwc_dpp<0x140>(v);    // row_mirror: 15 - lane in 16
    default: {
        const long long b = __double_as_longlong(v);
        const int lo = (int)b, hi = (int)(b >> 32);
        // the first result holds the even row (lower half) of each pair,
        // the second the odd row (upper half), in every lane
        const auto rl = level == 5 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                                   : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto rh = level == 5 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                                   : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        const double a = __longlong_as_double(((long long)rh[0] << 32) | (long long)(unsigned)rl[0]);
        const double c = __longlong_as_double(((long long)rh[1] << 32) | (long long)(unsigned)rl[1]);
        return a + c;
    }
    }
}

