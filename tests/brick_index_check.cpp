// Host check of the brick-binning index arithmetic of libmpcd (mpcd_dev.h):
// every (brick, window slot) an accumulating workgroup can write maps to one
// canonical cell, and the per-cell gather enumerates exactly those slots; the
// bucket offsets used for re-bucketing round-trip.  Prints "ok" or the first
// mismatch.  Built with hipcc as host code.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <tuple>
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
            L[d] = trial < 50 ? rnd(1, 6) : rnd(1, 70);
            want[d] = rnd(2, 16);
        }
        const BrickGeom g = brick_geometry(L, want);
        const int m = g.margin;
        for (int d = 0; d < 3; ++d) {
            // bricks tile the dimension, sizes within one of each other, >= margin
            int prev = 0;
            for (int i = 0; i < g.nb[d]; ++i) {
                const int lo = brick_lo(i, L[d], g.nb[d]), hi = brick_lo(i + 1, L[d], g.nb[d]);
                if (lo != prev || hi <= lo || hi - lo > g.bmax[d] || hi - lo < m) {
                    printf("tiling L=%d nb=%d brick %d [%d,%d)\n", L[d], g.nb[d], i, lo, hi);
                    return 1;
                }
                for (int c = lo; c < hi; ++c)
                    if (brick_of(c, L[d], g.nb[d]) != i) {
                        printf("brick_of L=%d nb=%d c=%d\n", L[d], g.nb[d], c);
                        return 1;
                    }
                prev = hi;
            }
            if (prev != L[d]) { printf("tiling end\n"); return 1; }
            // slots an accumulating brick can write (l < size + 2m, offset taken mod L)
            std::set<std::pair<int, int>> written;   // (brick, l) reached by some cell
            for (int i = 0; i < g.nb[d]; ++i) {
                const int lo = brick_lo(i, L[d], g.nb[d]);
                const int ext = brick_lo(i + 1, L[d], g.nb[d]) - lo + 2 * m;
                if (ext > g.wdim[d]) { printf("window overflow\n"); return 1; }
                for (int c = 0; c < L[d]; ++c) {
                    const int l = window_offset(c, lo, m, L[d]);
                    if (l < 0 || l >= L[d]) { printf("offset range\n"); return 1; }
                    if (l < ext) written.insert({i, l});
                }
            }
            // the gather of each cell enumerates exactly its slots
            std::set<std::pair<int, int>> gathered;
            for (int c = 0; c < L[d]; ++c) {
                int bi[3], li[3];
                const int n = windows_of(c, L[d], g.nb[d], m, bi, li);
                for (int k = 0; k < n; ++k) {
                    const int lo = brick_lo(bi[k], L[d], g.nb[d]);
                    if (window_offset(c, lo, m, L[d]) != li[k]) { printf("gather offset\n"); return 1; }
                    if (!gathered.insert({bi[k], li[k]}).second) { printf("slot gathered twice\n"); return 1; }
                }
                // every brick whose window holds c must be listed
                for (int i = 0; i < g.nb[d]; ++i) {
                    const int lo = brick_lo(i, L[d], g.nb[d]);
                    const int ext = brick_lo(i + 1, L[d], g.nb[d]) - lo + 2 * m;
                    if (window_offset(c, lo, m, L[d]) < ext) {
                        bool found = false;
                        for (int k = 0; k < n; ++k) found |= (bi[k] == i);
                        if (!found) {
                            printf("missed window L=%d nb=%d c=%d brick=%d\n", L[d], g.nb[d], c, i);
                            return 1;
                        }
                    }
                }
            }
            if (gathered != written) { printf("written != gathered L=%d nb=%d\n", L[d], g.nb[d]); return 1; }
            // neighbour offsets round-trip
            for (int s = 0; s < g.nb[d]; ++s)
                for (int t = 0; t < g.nb[d]; ++t) {
                    const int r = brick_rel(s, t, g.nb[d]);
                    if (r <= 1) {
                        if (r < -1 || (s + r + g.nb[d]) % g.nb[d] != t) { printf("rel\n"); return 1; }
                    } else if (g.nb[d] <= 3) {
                        printf("far in small grid\n");
                        return 1;
                    }
                }
        }
    }
    // bucket group layout: group q of bucket d comes from brick d - off(q) and
    // every (source, q) pair lands in exactly one bucket group
    for (int nb = 1; nb <= 6; ++nb) {
        for (int d = 0; d < nb; ++d) {
            std::set<int> srcs;
            for (int r = -1; r <= 1; ++r) {
                const int src = brick_nbr(d, -r, nb);
                if (src < 0) continue;
                if (brick_nbr(src, r, nb) != d) { printf("nbr inverse nb=%d\n", nb); return 1; }
                if (brick_rel(src, d, nb) != r) { printf("rel vs nbr nb=%d d=%d r=%d\n", nb, d, r); return 1; }
                if (!srcs.insert(src).second && nb >= 3) { printf("duplicate source\n"); return 1; }
            }
        }
        for (int s = 0; s < nb; ++s)
            for (int t = 0; t < nb; ++t) {
                const int r = brick_rel(s, t, nb);
                if (r <= 1 && brick_nbr(s, r, nb) != t) { printf("rel/nbr mismatch\n"); return 1; }
            }
    }
    printf("ok\n");
    return 0;
}
