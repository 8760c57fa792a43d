// Host-side Philox4x32-10 outputs from rocRAND's header implementation, used
// by the test suite as an independent library reference for the oracle's
// own Philox.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal), prints the four
// output words.  rocRAND's engine keys on the 64-bit seed, puts the
// subsequence in counter words 2..3 and offset/4 in words 0..1, so an
// arbitrary counter with c1 < 2^30 is reached exactly.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subseq = c2 | (c3 << 32);
        unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
