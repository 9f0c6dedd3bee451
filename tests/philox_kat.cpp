// Known-answer generator for Philox4x32-10 from the rocRAND header-only
// engine (an implementation independent of the oracle's).  Reads lines
// "seed subsequence counter" (decimal u64) and prints the four output words
// of Philox4x32-10 for counter (counter lo, counter hi, subsequence lo,
// subsequence hi) and key (seed lo, seed hi).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long seed, sub, ctr;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &ctr) == 3) {
        rocrand_device::philox4x32_10_engine e;
        e.seed(seed, sub, 4ULL * ctr);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
