// Host check of the brick-binning index arithmetic of libmpcd (mpcd_dev.h):
// aligned power-of-two bricks tile every dimension and brick_of inverts
// brick_lo; isqrt_ceil is exact; the neighbour
// group of a destination brick (brick_rel) maps back to it (brick_nbr) and is
// unique per source; bucket capacities with slack leave an overflow bucket
// that can take every particle; bucket_of_slot finds the bucket of every slot
// when some buckets are empty; interior bricks route by a shift of the next
// cell index exactly as the general form does; the counting sort's blocked cell order
// (sort_key) is a bijection that cell_of_key inverts.  Prints "ok" or the
// first mismatch.  Built
// with hipcc as host code.
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <set>
#include <vector>

#include "mpcd_dev.h"

using namespace mpcd;

static unsigned rng_state = 12345u;
static int rnd(int lo, int hi)
{
    rng_state = rng_state * 1664525u + 1013904223u;
    return lo + (int)((rng_state >> 8) % (unsigned)(hi - lo + 1));
}

int main()
{
    for (int trial = 0; trial < 400; ++trial) {
        int32_t L[3], want[3];
        for (int d = 0; d < 3; ++d) {
            L[d] = trial < 50 ? rnd(1, 6) : rnd(1, 300);
            want[d] = 1 << rnd(1, 6);   // 2 .. 64
        }
        const BrickGeom g = brick_geometry(L, want);
        int vol = 1;
        for (int d = 0; d < 3; ++d) {
            if ((1 << g.shift[d]) != want[d]) { printf("shift\n"); return 1; }
            int prev = 0;
            for (int i = 0; i < g.nb[d]; ++i) {
                const int lo = brick_lo(i, g.shift[d]);
                const int hi = std::min(brick_lo(i + 1, g.shift[d]), L[d]);
                if (lo != prev || hi <= lo || hi - lo > g.bmax[d]) {
                    printf("tiling L=%d nb=%d brick %d [%d,%d)\n", L[d], g.nb[d], i, lo, hi);
                    return 1;
                }
                for (int c = lo; c < hi; ++c)
                    if (brick_of(c, g.shift[d]) != i) {
                        printf("brick_of L=%d nb=%d c=%d\n", L[d], g.nb[d], c);
                        return 1;
                    }
                prev = hi;
            }
            if (prev != L[d]) { printf("tiling end\n"); return 1; }
            vol *= g.bmax[d];
        }
        if (vol != g.bvol) { printf("bvol\n"); return 1; }
    }
    // neighbour groups: every destination within one brick of the source has
    // an offset in {-1, 0, 1} that leads back to it, distinct destinations
    // have distinct offsets, and bricks farther away are reported as far
    for (int nb = 1; nb <= 9; ++nb)
        for (int s = 0; s < nb; ++s) {
            std::set<int> seen;
            for (int t = 0; t < nb; ++t) {
                const int r = brick_rel(s, t, nb);
                const int dist = std::min(std::abs(t - s), nb - std::abs(t - s));
                if (r <= 1) {
                    if (r < -1 || brick_nbr(s, r, nb) != t) { printf("rel/nbr nb=%d s=%d t=%d\n", nb, s, t); return 1; }
                    if (!seen.insert(r).second) { printf("two destinations share an offset\n"); return 1; }
                    if (dist > 1) { printf("near but far nb=%d s=%d t=%d\n", nb, s, t); return 1; }
                } else if (r != 2 || dist <= 1) {
                    printf("far nb=%d s=%d t=%d r=%d\n", nb, s, t, r);
                    return 1;
                }
            }
        }
    // integer square root (ceil) used by the bucket slack
    for (uint32_t n = 0; n < 300000u; ++n) {
        const uint32_t r = isqrt_ceil(n);
        if ((unsigned long long)r * r < n || (r > 0 && (unsigned long long)(r - 1) * (r - 1) >= n)) {
            printf("isqrt_ceil(%u) = %u\n", n, r);
            return 1;
        }
    }
    for (uint32_t n : {0xffffffffu, 0xfffe0001u, 0xfffe0000u, 1u << 30, (1u << 30) + 1u, 16777217u}) {
        const uint32_t r = isqrt_ceil(n);
        if ((unsigned long long)r * r < n || (r > 0 && (unsigned long long)(r - 1) * (r - 1) >= n)) {
            printf("isqrt_ceil(%u) = %u\n", n, r);
            return 1;
        }
    }
    // bucket layouts as re-bucketing builds them (counts plus slack, the
    // overflow bucket last), with empty buckets in runs
    for (int trial = 0; trial < 300; ++trial) {
        const int nbk = rnd(1, 400);
        std::vector<uint32_t> cnt(nbk);
        int64_t n = 0;
        for (int d = 0; d < nbk; ++d) {
            cnt[d] = (rnd(0, 3) == 0) ? 0u : (uint32_t)rnd(0, trial < 100 ? 40 : 5000);
            n += cnt[d];
        }
        const int64_t nslot = brick_slots(n, nbk);
        std::vector<uint32_t> start(nbk + 2);
        int64_t run = 0;
        for (int d = 0; d < nbk; ++d) {
            start[d] = (uint32_t)run;
            run += cnt[d] + bucket_slack(cnt[d]);
        }
        start[nbk] = (uint32_t)run;
        start[nbk + 1] = (uint32_t)nslot;
        if (nslot - run < n) { printf("overflow bucket smaller than n\n"); return 1; }
        // also the compact layout: everything in bucket 0
        std::vector<uint32_t> compact(nbk + 2, (uint32_t)n);
        compact[0] = 0;
        compact[nbk + 1] = (uint32_t)nslot;
        for (const std::vector<uint32_t>* st : {&start, &compact})
            for (int64_t i = 0; i < nslot; ++i) {
                const int b = bucket_of_slot(st->data(), nbk, i);
                if (b < 0 || b > nbk || (int64_t)(*st)[b] > i || (int64_t)(*st)[b + 1] <= i) {
                    printf("bucket_of_slot nbk=%d slot=%lld -> %d\n", nbk, (long long)i, b);
                    return 1;
                }
            }
    }
    // interior bricks of the brick step (a full brick below and above, itself
    // full, along the axis): for every next-step cell index c in [-1, L] (L
    // and -1 are the periodic images of cells 0 and L-1), a neighbour that
    // (c >> shift) - b names is the one the exact form gives for the wrapped
    // cell (anything else goes to the exact slow path, which is always
    // right), and every cell of the three bricks is named
    for (int trial = 0; trial < 2000; ++trial) {
        const int L = rnd(1, 300), sh = rnd(1, 6);
        const int nb = (L + (1 << sh) - 1) >> sh;
        for (int b = 0; b < nb; ++b) {
            if (!(b >= 1 && ((b + 2) << sh) <= L)) continue;
            for (int c = -1; c <= L; ++c) {
                const int fast = (c >> sh) - b;
                const int wrapped = c < 0 ? c + L : (c >= L ? c - L : c);
                const int exact = brick_rel(b, brick_of(wrapped, sh), nb);
                const bool fast_nbr = fast >= -1 && fast <= 1;
                const bool near = c >= ((b - 1) << sh) && c < ((b + 2) << sh);
                if ((fast_nbr && fast != exact) || (near && !fast_nbr)) {
                    printf("interior routing L=%d shift=%d brick=%d cell=%d: %d vs %d\n", L, sh, b, c, fast, exact);
                    return 1;
                }
            }
        }
    }
    // the counting sort's blocked cell order: a bijection of the cells onto
    // [0, L0 L1 L2) that cell_of_key inverts (every cell of small boxes,
    // random cells of large ones, blocks from 1 to 32 cells per edge)
    for (int trial = 0; trial < 300; ++trial) {
        int32_t L[3], sh[3];
        for (int d = 0; d < 3; ++d) {
            L[d] = trial < 200 ? rnd(1, 40) : rnd(1, 1200);
            sh[d] = rnd(0, 5);
        }
        const uint64_t nc = (uint64_t)L[0] * L[1] * L[2];
        if (trial < 200) {
            std::vector<char> seen(nc, 0);
            for (int iz = 0; iz < L[2]; ++iz)
                for (int iy = 0; iy < L[1]; ++iy)
                    for (int ix = 0; ix < L[0]; ++ix) {
                        const uint32_t key = sort_key(L, sh, ix, iy, iz);
                        const uint32_t c = (uint32_t)(ix + L[0] * (iy + L[1] * iz));
                        if (key >= nc || seen[key] || cell_of_key(L, sh, key) != c) {
                            printf("sort_key L=%d,%d,%d sh=%d,%d,%d cell %d,%d,%d -> %u\n", L[0], L[1], L[2], sh[0],
                                   sh[1], sh[2], ix, iy, iz, key);
                            return 1;
                        }
                        seen[key] = 1;
                    }
        } else {
            for (int q = 0; q < 20000; ++q) {
                const int ix = rnd(0, L[0] - 1), iy = rnd(0, L[1] - 1), iz = rnd(0, L[2] - 1);
                const uint32_t key = sort_key(L, sh, ix, iy, iz);
                if (key >= nc || cell_of_key(L, sh, key) != (uint32_t)(ix + L[0] * (iy + L[1] * iz))) {
                    printf("sort_key (large) L=%d,%d,%d cell %d,%d,%d -> %u\n", L[0], L[1], L[2], ix, iy, iz, key);
                    return 1;
                }
            }
        }
    }
    printf("ok\n");
    return 0;
}
