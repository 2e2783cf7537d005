// Known-answer source for the oracle's Philox4x32-10: calls the block
// function of rocRAND's host-callable Philox engine (an implementation
// independent of this project).  Reads lines "c0 c1 c2 c3 k0 k1" (hex) on
// stdin, prints "x0 x1 x2 x3" (hex).  Built and run by the test suite only.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct probe : rocrand_device::philox4x32_10_engine
{
    uint4 block(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    probe eng;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = eng.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
