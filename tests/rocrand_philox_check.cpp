// Host-only helper for the oracle's RNG test: prints rocRAND's Philox4x32-10
// output for the counters/keys read on stdin ("c0 c1 c2 c3 k0 k1" in hex), using
// rocRAND's documented mapping: key = seed (low, high word), counter words 2-3 =
// subsequence, counter words 0-1 = offset / 4.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
        unsigned long long offset = (((unsigned long long)c1 << 32) | c0) * 4ull;
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, offset, &st);
        uint4 r = rocrand4(&st);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
