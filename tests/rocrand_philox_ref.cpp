// Independent Philox4x32-10 reference for the tests: rocRAND's public header,
// built for the host only.  Reads "seed counter64 word2 word3" per line and
// prints the four output words of the block at that counter.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long seed, c64, w2, w3;
    while (std::scanf("%llu %llu %llu %llu", &seed, &c64, &w2, &w3) == 4) {
        rocrand_state_philox4x32_10 st;
        // rocRAND puts the subsequence in counter words 2-3 and offset/4 in words 0-1.
        rocrand_init(seed, w2 | (w3 << 32), 4ull * c64, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
