// Test-only third-party reference: rocRAND's Philox4x32-10 engine, run on the
// host.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal) and prints the four output
// words.  rocRAND's engine takes (seed, subsequence, offset): the seed is the
// 64-bit key, the subsequence is the upper counter half (c2, c3) and offset/4
// the lower half (c0, c1), so this maps a raw (counter, key) onto that API.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long sub = c2 | (c3 << 32);
        unsigned long long lower = c0 | (c1 << 32);
        rocrand_init(seed, sub, 4ull * (lower & ((1ull << 62) - 1)), &st);
        for (unsigned long long k = 0; k < 4ull * (lower >> 62); ++k)
            skipahead(1ull << 62, &st);   // 2^60 counter steps each
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
