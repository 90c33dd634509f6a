// Host program: Philox4x32-10 outputs from rocRAND's open-source engine for
// counters/keys read from stdin ("c0 c1 c2 c3 k0 k1" in hex per line).
// Used only by the oracle's Philox test as an independent implementation.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c[4], k[2];
    while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        unsigned long long seed = (unsigned long long)k[0] | ((unsigned long long)k[1] << 32);
        unsigned long long sub = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
        // counter words 0/1 are reached by skipping 4 outputs per counter step
        rocrand_device::philox4x32_10_engine e(seed, sub, 4ull * c[0]);
        unsigned long long hi = c[1];
        while (hi) {
            unsigned long long h = hi > (1ull << 28) ? (1ull << 28) : hi;
            e.discard(h << 34);
            hi -= h;
        }
        unsigned r0 = e.next(), r1 = e.next(), r2 = e.next(), r3 = e.next();
        std::printf("%08x %08x %08x %08x\n", r0, r1, r2, r3);
    }
    return 0;
}
