// Independent Philox4x32-10 reference for the oracle's pin: rocRAND's
// header-only engine, run on the host.  Reads "seed c0 c1 c2 c3" lines and
// prints the four output words of Philox4x32-10(key = seed, counter = c).
// rocRAND places the 64-bit subsequence in counter words 2..3 and offset/4
// in words 0..1, so (subsequence, offset) select the counter exactly.
#include <cstdio>
#include <cinttypes>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long seed;
    unsigned int c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        // offset = 4 * (c0 + 2^32 c1) does not fit 64 bits when c1 >= 2^30:
        // add the low 30 bits of c1 at once and the top two bits in steps of
        // 2^62 numbers (2^28 in counter word 1) each.
        unsigned long long offset =
            4ull * ((unsigned long long)c0 | ((unsigned long long)(c1 & 0x3fffffffu) << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        for (unsigned int k = 0; k < 4u * (c1 >> 30); ++k) eng.discard(1ull << 62);
        uint4 v = eng.next4();
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
