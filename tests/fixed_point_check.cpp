// Host check of the exact fixed-point arithmetic of libmpcd (mpcd_dev.h):
// to_fixed(v) is v 2^32 truncated toward zero (computed here from the
// double value, which holds every float times 2^32 exactly), for random
// magnitudes from 2^-40 to the velocity limit, exact powers of two, both
// signs, zero, subnormals and non-finite values; the range check flags
// exactly the velocities at or beyond kVelocityLimit (and NaN); and at the
// limits a cell of kMaxCellCount - 1 terms m v 2^32 (masses up to kMassMax)
// cannot reach 2^63.  Prints "ok" or the first mismatch.  Built with hipcc
// as host code.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "mpcd_dev.h"

using namespace mpcd;

static unsigned long long rng = 88172645463325252ull;
static unsigned long long next()
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
}

// v 2^32 truncated toward zero as a two's-complement 64-bit word
static unsigned long long reference(float v)
{
    if (!std::isfinite(v) || std::fabs((double)v) >= 2147483648.0) return 0ull;
    const double t = std::trunc((double)v * 4294967296.0);   // exact: a float has 24 bits
    const long long q = (long long)t;
    return (unsigned long long)q;
}

static int check(float v)
{
    const unsigned long long got = to_fixed(v), want = reference(v);
    if (got != want) {
        printf("to_fixed(%.9g) = %llx, want %llx\n", (double)v, got, want);
        return 1;
    }
    return 0;
}

int main()
{
    // random magnitudes 2^-40 .. 2^8, both signs
    for (int i = 0; i < 2000000; ++i) {
        const unsigned long long r = next();
        const double mag = std::ldexp(1.0 + (double)(r & 0xffffff) / 16777216.0, (int)((r >> 24) % 48) - 40);
        const float v = (float)((r >> 40) & 1 ? -mag : mag);
        if (check(v)) return 1;
    }
    // every float bit pattern with a random significand, for each exponent
    for (unsigned e = 0; e < 256; ++e)
        for (int i = 0; i < 64; ++i) {
            const uint32_t bits = (uint32_t)((next() & 0x807fffffull) | ((unsigned long long)e << 23));
            float v;
            memcpy(&v, &bits, 4);
            const unsigned long long got = to_fixed(v);
            if (e == 255 || e == 0) {   // non-finite and subnormal: nothing
                if (got != 0ull) { printf("special exponent %u: %llx\n", e, got); return 1; }
                continue;
            }
            if (e > 157) continue;   // beyond 2^31: outside the range (flagged by the steps)
            if (check(v)) return 1;
        }
    // exact for |v| >= 2^-9: powers of two and their neighbours
    for (int p = -9; p <= 7; ++p) {
        const float v = std::ldexp(1.0f, p);
        if (to_fixed(v) != (1ull << (32 + p))) { printf("2^%d\n", p); return 1; }
        if (to_fixed(-v) != 0ull - (1ull << (32 + p))) { printf("-2^%d\n", p); return 1; }
        if (check(std::nextafter(v, 0.0f)) || check(std::nextafter(v, 1e9f))) return 1;
    }
    if (to_fixed(0.0f) != 0ull || to_fixed(-0.0f) != 0ull) { printf("zero\n"); return 1; }
    // the range check: |v| < kVelocityLimit passes, the limit and beyond fail
    const float below = std::nextafter(kVelocityLimit, 0.0f);
    const float cases[] = {0.0f, 1.0f, below, -below, kVelocityLimit, -kVelocityLimit, 1e30f, INFINITY, NAN};
    const int flagged[] = {0, 0, 0, 0, 1, 1, 1, 1, 1};
    for (int i = 0; i < 9; ++i) {
        long long d[kNumDiag] = {};
        diag_check(d, make_float3(0.5f, cases[i], -0.25f));
        if (d[5] != flagged[i]) { printf("range check of %g\n", (double)cases[i]); return 1; }
    }
    // the largest term m v 2^32 inside the range, and a cell of
    // kMaxCellCount - 1 of them, in 128-bit arithmetic
    const float vmax = below * kMassMax;   // m v rounds to FP32 before conversion
    const long long tmax = (long long)to_fixed(vmax);
    if (!(tmax > 0 && tmax < (1ll << 48))) { printf("largest term %lld\n", tmax); return 1; }
    const __int128 cell = (__int128)tmax * (kMaxCellCount - 1);
    if (!(cell < ((__int128)1 << 60))) { printf("cell sum bound\n"); return 1; }
    // the mass sum of such a cell
    const __int128 wsum = (__int128)to_fixed(kMassMax) * (kMaxCellCount - 1);
    if (!(wsum < ((__int128)1 << 63))) { printf("mass sum bound\n"); return 1; }
    printf("ok\n");
    return 0;
}
