// Prints Philox4x32-10 blocks computed by rocRAND's host-callable engine, for
// counters/keys read from stdin ("c0 c1 c2 c3 k0 k1" per line, decimal).
// rocRAND's engine(seed, subsequence, offset) with offset a multiple of 4
// places the counter at (offset/4 lo, offset/4 hi, subsequence lo, hi) and its
// first next4() returns that counter's block, so any counter with c1 < 2^30
// is reachable through the public API.  Used only by the test suite.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subsequence = c2 | (c3 << 32);
        unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
        uint4 v = eng.next4();
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
