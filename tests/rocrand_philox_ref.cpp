// Reference Philox4x32-10 words from rocRAND's own engine (its header runs on the host).
// Reads lines "seed c0 c1 c2 c3" (decimal) from stdin and prints the four output words of
// the block at counter (c0, c1, c2, c3) under key = seed, one line per input line.
// rocRAND maps (seed, subsequence, offset) to key = seed, counter words 2-3 = subsequence,
// counter words 0-1 = offset / 4.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main()
{
    unsigned long long seed;
    unsigned int c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long subsequence = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, subsequence, offset);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
