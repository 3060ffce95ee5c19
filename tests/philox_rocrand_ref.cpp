// Host-only helper for the Philox pin: reads lines "c0 c1 c2 c3 k0 k1" (hex)
// from stdin and prints the four output words of rocRAND's philox4x32_10
// engine for that counter and key.  The engine's counter is the 128-bit
// integer (c0 + 2^32 c1) + 2^64 (c2 + 2^32 c3): "subsequence" sets the upper
// 64 bits, "offset" (in 32-bit outputs) the lower ones.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned c[4], k[2];
    while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        unsigned long long seed = (unsigned long long)k[0] | ((unsigned long long)k[1] << 32);
        unsigned long long subseq = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
        unsigned long long lo = (unsigned long long)c[0] | ((unsigned long long)c[1] << 32);
        rocrand_device::philox4x32_10_engine e(seed, subseq, 0);
        // advance the lower 64 counter bits by lo blocks (4 outputs each) in four
        // calls of lo outputs, so that the 64-bit offset argument cannot overflow
        for (int r = 0; r < 4; ++r) e.discard(lo);
        unsigned o0 = e(), o1 = e(), o2 = e(), o3 = e();
        std::printf("%08x %08x %08x %08x\n", o0, o1, o2, o3);
    }
    return 0;
}
