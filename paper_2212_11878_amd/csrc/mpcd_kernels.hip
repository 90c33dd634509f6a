// mpcd_kernels.hip -- HIP kernels of the SRD step for gfx950 (MI355X).
//
// One step of a box (paper Sec. 2; shifted grid of Sec. 3.1, Listing 1;
// mass-weighted cell velocity of Sec. 3.3, Listing 4) runs as:
//
//   ATOMIC binning (particles bucketed by brick of cells)
//     k_brick_accumulate  per brick: stream, bin into the brick's window,
//                         LDS-atomic exact cell sums, write window partials,
//                         count next-step buckets
//     k_brick_sizes/scan/offsets  next bucket sizes and starts, and where
//                         each source brick's movers start in them
//     k_brick_finalize    per cell: add the window partials (and escapes),
//                         u_c = sum v / n, axis n_c from Philox
//     k_brick_rotate      per brick: stream again (same arithmetic), rotate
//                         v <- u_c + R(n_c, alpha)(v - u_c), write the
//                         particle into its next bucket; FP64 diagnostics
//     k_box_finish        per box: reduce diagnostics, VACF sample, k++
//
//   SORT binning (counting sort by collision cell every step)
//     zero, k_count (streamed collision cell + rank), scan, k_scatter (streams
//     while moving), flip, k_cell_rotate (one thread per cell over its
//     contiguous run), k_box_finish
//
// Both paths sum the momentum of a cell exactly (64-bit fixed point), so
// they produce bit-identical velocities whatever the order of the atomics.
// All kernels grid over "tiles" (contiguous particle, cell or brick ranges of
// one box), which lets one launch advance many boxes of different sizes.
#include "mpcd_dev.h"
#include "mpcd_launch.h"

namespace mpcd {

// --------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ bool box_idle(const BoxState& s) { return s.remaining == 0; }

// The counting sort runs every step for SORT boxes, and once for brick
// boxes whose particles are not bucketed yet (after admission / set_state).
__device__ __forceinline__ bool sort_due(const BoxDev& b, const BoxState& s)
{
    return b.binning == 2 || s.rebucket != 0;
}

__device__ __forceinline__ bool vacf_due(const BoxDev& b, const BoxState& s)
{
    return b.vacf_stride > 0 && ((s.k + 1 - s.vacf_origin) % b.vacf_stride) == 0;
}

__device__ __forceinline__ long long wave_sum(long long v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Block sum of kNumDiag exact partials; threads 0..kNumDiag-1 write out[].
__device__ __forceinline__ void block_diag(long long (&d)[kNumDiag], long long* out)
{
    __shared__ long long red[kBlock / kWave][kNumDiag];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < kNumDiag; ++j) {
        const long long v = wave_sum(d[j]);
        if (lane == 0) red[w][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < kNumDiag) {
        long long v = 0;
        for (int i = 0; i < kBlock / kWave; ++i) v += red[i][threadIdx.x];
        out[threadIdx.x] = v;
    }
}

// Block-wide exclusive scan of one uint32 per thread; returns the prefix and
// the block total in *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total)
{
    __shared__ uint32_t wsum[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += t;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        const uint32_t s = wsum[i];
        if (i < w) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

// --------------------------------------------------------------------------
// ATOMIC (brick) path

__global__ __launch_bounds__(kBlock) void k_brick_accumulate(const Tile* __restrict__ tiles,
                                                              const BoxDev* __restrict__ boxes,
                                                              const BoxState* __restrict__ st)
{
    extern __shared__ CellAcc win[];
    __shared__ uint32_t cnt[27];
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (box_idle(s) || b.binning != 1) return;
    const int brick = (int)tl.begin;
    const int bx = brick % b.nb[0], by = (brick / b.nb[0]) % b.nb[1], bz = brick / (b.nb[0] * b.nb[1]);
    const int m = b.margin;
    const int lox = b.blo[0][bx], loy = b.blo[1][by], loz = b.blo[2][bz];
    const int ex = b.blo[0][bx + 1] - lox + 2 * m;   // window extents
    const int ey = b.blo[1][by + 1] - loy + 2 * m;
    const int ez = b.blo[2][bz + 1] - loz + 2 * m;
    const int wx = b.wdim[0], wy = b.wdim[1];
    for (int i = threadIdx.x; i < b.wsize; i += kBlock) {
        CellAcc z = {0ull, 0ull, 0ull, 0ull};
        win[i] = z;
    }
    if (threadIdx.x < 27) cnt[threadIdx.x] = 0u;
    __syncthreads();

    const int par = s.parity;
    const MPCD_G float* __restrict__ x = gp(b.p[par][0]);
    const MPCD_G float* __restrict__ y = gp(b.p[par][1]);
    const MPCD_G float* __restrict__ z = gp(b.p[par][2]);
    const MPCD_G float* __restrict__ vx = gp(b.p[par][3]);
    const MPCD_G float* __restrict__ vy = gp(b.p[par][4]);
    const MPCD_G float* __restrict__ vz = gp(b.p[par][5]);
    const float* __restrict__ mp = b.m[par];
    MPCD_G CellAcc* __restrict__ esc = gp(b.esc);
    MPCD_G uint32_t* __restrict__ bcount = gp(b.bcount);
    const float3 sh = grid_shift(b, s.k);
    const float dt = b.dt;
    const uint32_t stamp = (uint32_t)(s.k + 1);
    const int64_t beg = b.bstart[par][brick], end = b.bstart[par][brick + 1];
    constexpr int kU = 8;   // particles per thread in flight
    for (int64_t base = beg; base < end; base += (int64_t)kBlock * kU) {
        float qx[kU], qy[kU], qz[kU], qvx[kU], qvy[kU], qvz[kU], qm[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {   // issue every load first
            const int64_t i = base + u * kBlock + threadIdx.x;
            const bool ok = i < end;
            const int64_t j = ok ? i : beg;
            qx[u] = x[j];
            qy[u] = y[j];
            qz[u] = z[j];
            qvx[u] = vx[j];
            qvy[u] = vy[j];
            qvz[u] = vz[j];
            qm[u] = mp ? gp(mp)[j] : 1.0f;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = base + u * kBlock + threadIdx.x;
            if (i >= end) continue;
            const float ux = qvx[u], uy = qvy[u], uz = qvz[u];
            const float px = fold(fmaf(ux, dt, qx[u]), b.len[0]);
            const float py = fold(fmaf(uy, dt, qy[u]), b.len[1]);
            const float pz = fold(fmaf(uz, dt, qz[u]), b.len[2]);
            const int cx = axis_cell(px, sh.x, b.inv_a, b.L[0]);
            const int cy = axis_cell(py, sh.y, b.inv_a, b.L[1]);
            const int cz = axis_cell(pz, sh.z, b.inv_a, b.L[2]);
            const int lx = window_offset(cx, lox, m, b.L[0]);
            const int ly = window_offset(cy, loy, m, b.L[1]);
            const int lz = window_offset(cz, loz, m, b.L[2]);
            const float mi = qm[u];
            const unsigned long long fx = to_fixed(mi * ux), fy = to_fixed(mi * uy), fz = to_fixed(mi * uz);
            const unsigned long long fw = to_fixed(mi);
            if (lx < ex && ly < ey && lz < ez) {
                CellAcc* w = &win[lx + wx * (ly + wy * lz)];
                atomicAdd(&w->sx, fx);
                atomicAdd(&w->sy, fy);
                atomicAdd(&w->sz, fz);
                atomicAdd(&w->w, fw);
            } else {   // left the window: exact global sums, flag the owner brick
                const uint32_t c = (uint32_t)cx + (uint32_t)b.L[0] * ((uint32_t)cy + (uint32_t)b.L[1] * (uint32_t)cz);
                gatomic_add(&esc[c].sx, fx);
                gatomic_add(&esc[c].sy, fy);
                gatomic_add(&esc[c].sz, fz);
                gatomic_add(&esc[c].w, fw);
                const int ob = b.bof[0][cx] + b.nb[0] * (b.bof[1][cy] + b.nb[1] * b.bof[2][cz]);
                gp(b.eflag)[ob] = stamp;
            }
            // bucket of the streamed position for the next step
            const int3 d = brick_of_pos(b, px, py, pz);
            const int rx = brick_rel(bx, d.x, b.nb[0]), ry = brick_rel(by, d.y, b.nb[1]),
                      rz = brick_rel(bz, d.z, b.nb[2]);
            if (rx <= 1 && ry <= 1 && rz <= 1)
                atomicAdd(&cnt[(rx + 1) + 3 * ((ry + 1) + 3 * (rz + 1))], 1u);
            else
                gatomic_add(&bcount[d.x + b.nb[0] * (d.y + b.nb[1] * d.z)], 1u);
        }
    }
    __syncthreads();
    MPCD_G CellAcc* __restrict__ out = gp(b.part) + (size_t)brick * b.wsize;
    for (int i = threadIdx.x; i < b.wsize; i += kBlock) store_acc(out + i, win[i]);
    if (threadIdx.x < 27) gp(b.outcnt)[(size_t)brick * 27 + threadIdx.x] = cnt[threadIdx.x];
}

// bucket sizes of the next step: the neighbour groups plus the far particles
__global__ __launch_bounds__(kBlock) void k_brick_sizes(const Tile* __restrict__ tiles, int ntiles,
                                                         const BoxDev* __restrict__ boxes,
                                                         const BoxState* __restrict__ st)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (box_idle(s) || b.binning != 1) return;
    const int d = (int)tl.begin;
    const int dx = d % b.nb[0], dy = (d / b.nb[0]) % b.nb[1], dz = d / (b.nb[0] * b.nb[1]);
    uint32_t n = gp(b.bcount)[d];
    for (int r = 0; r < 27; ++r) {   // source of group r of bucket d: d - offset(r)
        const int sx = brick_nbr(dx, 1 - r % 3, b.nb[0]);
        const int sy = brick_nbr(dy, 1 - (r / 3) % 3, b.nb[1]);
        const int sz = brick_nbr(dz, 1 - r / 9, b.nb[2]);
        if (sx < 0 || sy < 0 || sz < 0) continue;
        n += gp(b.outcnt)[(size_t)(sx + b.nb[0] * (sy + b.nb[1] * sz)) * 27 + r];
    }
    gp(b.bsize)[d] = n;
}

// per box: bucket starts of the next buffer, far-particle cursors, reset
__global__ __launch_bounds__(kBlock) void k_brick_scan(const int32_t* __restrict__ active,
                                                        const BoxDev* __restrict__ boxes,
                                                        const BoxState* __restrict__ st)
{
    const int bx = active[blockIdx.x];
    const BoxState s = st[bx];
    const BoxDev& b = boxes[bx];
    if (box_idle(s) || b.binning != 1) return;
    const int nb = b.nbrick;
    const int per = (nb + kBlock - 1) / kBlock;
    const int lo = min(nb, (int)threadIdx.x * per), hi = min(nb, ((int)threadIdx.x + 1) * per);
    uint32_t v = 0;
    for (int i = lo; i < hi; ++i) v += gp(b.bsize)[i];
    uint32_t total;
    uint32_t run = block_exclusive_scan(v, &total);
    MPCD_G uint32_t* __restrict__ next = gp(b.bstart[s.parity ^ 1]);
    for (int i = lo; i < hi; ++i) {
        const uint32_t c = gp(b.bsize)[i];
        next[i] = run;
        gp(b.bcursor)[i] = run + c - gp(b.bcount)[i];   // far particles fill the bucket's end
        gp(b.bcount)[i] = 0u;
        run += c;
    }
    if (threadIdx.x == 0) next[nb] = total;
}

// where the particles of source brick b heading for neighbour r start in
// that neighbour's bucket: groups are laid out in r order
__global__ __launch_bounds__(kBlock) void k_brick_offsets(const Tile* __restrict__ tiles, int ntiles,
                                                           const BoxDev* __restrict__ boxes,
                                                           const BoxState* __restrict__ st)
{
    const int g = blockIdx.x * kBlock + threadIdx.x;   // (brick tile, r) pairs
    const int t = g / 27, r = g % 27;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (box_idle(s) || b.binning != 1) return;
    const int src = (int)tl.begin;
    const int sx = src % b.nb[0], sy = (src / b.nb[0]) % b.nb[1], sz = src / (b.nb[0] * b.nb[1]);
    const int dx = brick_nbr(sx, r % 3 - 1, b.nb[0]);
    const int dy = brick_nbr(sy, (r / 3) % 3 - 1, b.nb[1]);
    const int dz = brick_nbr(sz, r / 9 - 1, b.nb[2]);
    uint32_t off = 0;
    if (dx >= 0 && dy >= 0 && dz >= 0) {
        const int d = dx + b.nb[0] * (dy + b.nb[1] * dz);
        off = gp(b.bstart[s.parity ^ 1])[d];
        for (int q = 0; q < r; ++q) {   // earlier groups of bucket d
            const int ex = brick_nbr(dx, 1 - q % 3, b.nb[0]);
            const int ey = brick_nbr(dy, 1 - (q / 3) % 3, b.nb[1]);
            const int ez = brick_nbr(dz, 1 - q / 9, b.nb[2]);
            if (ex < 0 || ey < 0 || ez < 0) continue;
            off += gp(b.outcnt)[(size_t)(ex + b.nb[0] * (ey + b.nb[1] * ez)) * 27 + q];
        }
    }
    gp(b.outbase)[(size_t)src * 27 + r] = off;
}

__global__ __launch_bounds__(kBlock) void k_brick_finalize(const Tile* __restrict__ tiles,
                                                            const BoxDev* __restrict__ boxes,
                                                            const BoxState* __restrict__ st)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (box_idle(s) || b.binning != 1) return;
    const int m = b.margin;
    const uint32_t stamp = (uint32_t)(s.k + 1);
    const uint32_t L0 = (uint32_t)b.L[0], L01 = (uint32_t)b.L[0] * (uint32_t)b.L[1];
    for (int64_t c = tl.begin + threadIdx.x; c < tl.end; c += kBlock) {
        const uint32_t cu = (uint32_t)c;
        const int cz = (int)(cu / L01);
        const uint32_t rem = cu - (uint32_t)cz * L01;
        const int cy = (int)(rem / L0);
        const int cx = (int)(rem - (uint32_t)cy * L0);
        int bxs[3], lxs[3], bys[3], lys[3], bzs[3], lzs[3];
        const int nx = windows_of_tab(cx, b.L[0], b.nb[0], m, b.bof[0], b.blo[0], bxs, lxs);
        const int ny = windows_of_tab(cy, b.L[1], b.nb[1], m, b.bof[1], b.blo[1], bys, lys);
        const int nz = windows_of_tab(cz, b.L[2], b.nb[2], m, b.bof[2], b.blo[2], bzs, lzs);
        unsigned long long sx = 0, sy = 0, sz = 0, sw = 0;
        for (int iz = 0; iz < nz; ++iz)
            for (int iy = 0; iy < ny; ++iy)
                for (int ix = 0; ix < nx; ++ix) {
                    const int br = bxs[ix] + b.nb[0] * (bys[iy] + b.nb[1] * bzs[iz]);
                    const int sl = lxs[ix] + b.wdim[0] * (lys[iy] + b.wdim[1] * lzs[iz]);
                    const CellAcc r = load_acc(gp(b.part) + (size_t)br * b.wsize + sl);
                    sx += r.sx;
                    sy += r.sy;
                    sz += r.sz;
                    sw += r.w;
                }
        const int ob = b.bof[0][cx] + b.nb[0] * (b.bof[1][cy] + b.nb[1] * b.bof[2][cz]);
        if (gp(b.eflag)[ob] == stamp) {
            const CellAcc e = load_acc(gp(b.esc) + c);
            if (e.w) {
                sx += e.sx;
                sy += e.sy;
                sz += e.sz;
                sw += e.w;
                CellAcc zero = {0ull, 0ull, 0ull, 0ull};
                store_acc(gp(b.esc) + c, zero);
            }
        }
        if (sw == 0) continue;
        CellUN u;
        u.ux = fixed_mean(sx, sw);
        u.uy = fixed_mean(sy, sw);
        u.uz = fixed_mean(sz, sw);
        const float3 ax = cell_axis(b, s.k, (uint32_t)c);
        u.nx = ax.x;
        u.ny = ax.y;
        u.nz = ax.z;
        u.kappa = axis_kappa(ax);
        u.pad1 = 0.0f;
        store_un(gp(b.un) + c, u);
    }
}

__global__ __launch_bounds__(kBlock) void k_brick_rotate(const Tile* __restrict__ tiles,
                                                          const BoxDev* __restrict__ boxes,
                                                          const BoxState* __restrict__ st,
                                                          long long* __restrict__ partials)
{
    extern __shared__ CellUN wun[];   // u_c and axis of the brick's window cells
    __shared__ uint32_t cnt[27];
    __shared__ uint32_t base[27];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const Tile tl = tiles[t];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (box_idle(s) || b.binning != 1) return;
    const int brick = (int)tl.begin;
    const int bx = brick % b.nb[0], by = (brick / b.nb[0]) % b.nb[1], bz = brick / (b.nb[0] * b.nb[1]);
    const int m = b.margin;
    const int lox = b.blo[0][bx], loy = b.blo[1][by], loz = b.blo[2][bz];
    const int ex = b.blo[0][bx + 1] - lox + 2 * m;
    const int ey = b.blo[1][by + 1] - loy + 2 * m;
    const int ez = b.blo[2][bz + 1] - loz + 2 * m;
    const int wx = b.wdim[0], wy = b.wdim[1];
    // stage the window's cell data in LDS (cells of empty slots are never read)
    for (int i = threadIdx.x; i < b.wsize; i += kBlock) {
        const int lx = i % wx, ly = (i / wx) % wy, lz = i / (wx * wy);
        if (lx < ex && ly < ey && lz < ez) {
            int cx = lox - m + lx, cy = loy - m + ly, cz = loz - m + lz;
            cx = ((cx % b.L[0]) + b.L[0]) % b.L[0];
            cy = ((cy % b.L[1]) + b.L[1]) % b.L[1];
            cz = ((cz % b.L[2]) + b.L[2]) % b.L[2];
            wun[i] = load_un(gp(b.un) + ((uint32_t)cx + (uint32_t)b.L[0] * ((uint32_t)cy + (uint32_t)b.L[1] * (uint32_t)cz)));
        }
    }
    __syncthreads();
    const int src = s.parity, dst = s.parity ^ 1;
    const float3 sh = grid_shift(b, s.k);
    const float dt = b.dt;
    const double ca = b.ca, sa = b.sa;
    const bool track = b.vacf_stride > 0;
    const bool vacf = vacf_due(b, s);
    const int64_t beg = b.bstart[src][brick], end = b.bstart[src][brick + 1];
    const MPCD_G float* __restrict__ ix = gp(b.p[src][0]);
    const MPCD_G float* __restrict__ iy = gp(b.p[src][1]);
    const MPCD_G float* __restrict__ iz = gp(b.p[src][2]);
    const MPCD_G float* __restrict__ ivx = gp(b.p[src][3]);
    const MPCD_G float* __restrict__ ivy = gp(b.p[src][4]);
    const MPCD_G float* __restrict__ ivz = gp(b.p[src][5]);
    const MPCD_G int32_t* __restrict__ iid = gp(b.pid[src]);
    MPCD_G float* __restrict__ ox = gp(b.p[dst][0]);
    MPCD_G float* __restrict__ oy = gp(b.p[dst][1]);
    MPCD_G float* __restrict__ oz = gp(b.p[dst][2]);
    MPCD_G float* __restrict__ ovx = gp(b.p[dst][3]);
    MPCD_G float* __restrict__ ovy = gp(b.p[dst][4]);
    MPCD_G float* __restrict__ ovz = gp(b.p[dst][5]);
    MPCD_G int32_t* __restrict__ oid = gp(b.pid[dst]);
    const MPCD_G float* __restrict__ im = b.m[src] ? gp(b.m[src]) : nullptr;
    MPCD_G float* __restrict__ om = b.m[dst] ? gp(b.m[dst]) : nullptr;
    const MPCD_G CellUN* __restrict__ un = gp(b.un);
    MPCD_G uint32_t* __restrict__ bcursor = gp(b.bcursor);
    // running ranks within each destination group; group starts precomputed
    if (threadIdx.x < 27) {
        cnt[threadIdx.x] = 0u;
        base[threadIdx.x] = gp(b.outbase)[(size_t)brick * 27 + threadIdx.x];
    }
    __syncthreads();
    long long d[kNumDiag] = {0, 0, 0, 0, 0, 0};
    const int lane = threadIdx.x & (kWave - 1);
    for (int64_t c0 = beg; c0 < end; c0 += (int64_t)kBlock * kItems) {
        float px[kItems], py[kItems], pz[kItems], qx[kItems], qy[kItems], qz[kItems], qm[kItems];
        int32_t id[kItems];
#pragma unroll
        for (int it = 0; it < kItems; ++it) {   // issue every load first
            const int64_t i = c0 + it * kBlock + threadIdx.x;
            const int64_t j = (i < end) ? i : beg;
            px[it] = ix[j];
            py[it] = iy[j];
            pz[it] = iz[j];
            qx[it] = ivx[j];
            qy[it] = ivy[j];
            qz[it] = ivz[j];
            qm[it] = im ? im[j] : 1.0f;
            id[it] = iid[j];
        }
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const int64_t i = c0 + it * kBlock + threadIdx.x;
            const bool ok = i < end;
            const float ux = qx[it], uy = qy[it], uz = qz[it];
            const float fx = fold(fmaf(ux, dt, px[it]), b.len[0]);
            const float fy = fold(fmaf(uy, dt, py[it]), b.len[1]);
            const float fz = fold(fmaf(uz, dt, pz[it]), b.len[2]);
            const int cx = axis_cell(fx, sh.x, b.inv_a, b.L[0]);
            const int cy = axis_cell(fy, sh.y, b.inv_a, b.L[1]);
            const int cz = axis_cell(fz, sh.z, b.inv_a, b.L[2]);
            const int lx = window_offset(cx, lox, m, b.L[0]);
            const int ly = window_offset(cy, loy, m, b.L[1]);
            const int lz = window_offset(cz, loz, m, b.L[2]);
            CellUN u;
            if (lx < ex && ly < ey && lz < ez)
                u = wun[lx + wx * (ly + wy * lz)];
            else
                u = load_un(un + ((uint32_t)cx + (uint32_t)b.L[0] * ((uint32_t)cy + (uint32_t)b.L[1] * (uint32_t)cz)));
            const float3 v = rotate_about(u, ux, uy, uz, ca, sa);
            const int3 db = brick_of_pos(b, fx, fy, fz);
            const int rx = brick_rel(bx, db.x, b.nb[0]), ry = brick_rel(by, db.y, b.nb[1]),
                      rz = brick_rel(bz, db.z, b.nb[2]);
            const bool near = rx <= 1 && ry <= 1 && rz <= 1;
            const int r = near ? (rx + 1) + 3 * ((ry + 1) + 3 * (rz + 1)) : 27;
            // rank in the destination group; particles that stay in this brick
            // (most of them) take consecutive ranks per wave, so stores coalesce
            const bool stay = ok && r == 13;
            const unsigned long long mask = __ballot(stay);
            uint32_t slot = 0;
            if (mask) {
                const int leader = __ffsll((long long)mask) - 1;
                uint32_t wbase = 0;
                if (lane == leader) wbase = atomicAdd(&cnt[13], (uint32_t)__popcll(mask));
                wbase = __shfl(wbase, leader, kWave);
                slot = base[13] + wbase + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
            }
            if (!ok) continue;
            if (r == 27)
                slot = gatomic_add(&bcursor[db.x + b.nb[0] * (db.y + b.nb[1] * db.z)], 1u);
            else if (r != 13)
                slot = base[r] + atomicAdd(&cnt[r], 1u);
            const int64_t j = slot;
            ox[j] = fx;
            oy[j] = fy;
            oz[j] = fz;
            ovx[j] = v.x;
            ovy[j] = v.y;
            ovz[j] = v.z;
            oid[j] = id[it];
            if (om) om[j] = qm[it];
            if (track) {
                gp(b.v0[dst][0])[j] = gp(b.v0[src][0])[i];
                gp(b.v0[dst][1])[j] = gp(b.v0[src][1])[i];
                gp(b.v0[dst][2])[j] = gp(b.v0[src][2])[i];
            }
            diag_particle(d, v, qm[it]);
            if (vacf) diag_vacf(d, v, gp(b.v0[src][0])[i], gp(b.v0[src][1])[i], gp(b.v0[src][2])[i]);
        }
    }
    block_diag(d, partials + (size_t)t * kNumDiag);
}

// --------------------------------------------------------------------------
// counting sort: by collision cell every step (SORT), or by brick once to
// bucket a brick box's particles (after admission / set_state)

__global__ __launch_bounds__(kBlock) void k_zero_counts(const Tile* __restrict__ tiles,
                                                         const BoxDev* __restrict__ boxes,
                                                         const BoxState* __restrict__ st)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (box_idle(s) || !sort_due(b, s)) return;
    for (int64_t c = tl.begin + threadIdx.x; c < tl.end; c += kBlock) b.cstart[c] = 0u;
    if (tl.end == b.ncell && threadIdx.x == 0) b.cstart[b.ncell] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_count(const Tile* __restrict__ tiles,
                                                   const BoxDev* __restrict__ boxes,
                                                   const BoxState* __restrict__ st)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (box_idle(s) || !sort_due(b, s)) return;
    const float* __restrict__ x = b.p[s.parity][0];
    const float* __restrict__ y = b.p[s.parity][1];
    const float* __restrict__ z = b.p[s.parity][2];
    const float* __restrict__ vx = b.p[s.parity][3];
    const float* __restrict__ vy = b.p[s.parity][4];
    const float* __restrict__ vz = b.p[s.parity][5];
    const bool collide_key = (b.binning == 2);
    const float3 sh = collide_key ? grid_shift(b, s.k) : make_float3(0.0f, 0.0f, 0.0f);
    const float dt = b.dt;
    for (int64_t i = tl.begin + threadIdx.x; i < tl.end; i += kBlock) {
        float px = x[i], py = y[i], pz = z[i];
        uint32_t key;
        if (collide_key) {
            px = fold(fmaf(vx[i], dt, px), b.len[0]);
            py = fold(fmaf(vy[i], dt, py), b.len[1]);
            pz = fold(fmaf(vz[i], dt, pz), b.len[2]);
            key = collision_cell(b, px, py, pz, sh);
        } else {
            const int3 d = brick_of_pos(b, px, py, pz);
            key = (uint32_t)(d.x + b.nb[0] * (d.y + b.nb[1] * d.z));
        }
        b.cell[i] = key;
        b.rank[i] = atomicAdd(&b.cstart[key], 1u);
    }
}

// per cell tile: total count
__global__ __launch_bounds__(kBlock) void k_scan_tilesum(const Tile* __restrict__ tiles,
                                                          const BoxDev* __restrict__ boxes,
                                                          const BoxState* __restrict__ st,
                                                          uint32_t* __restrict__ tilesum)
{
    const int t = blockIdx.x;
    const Tile tl = tiles[t];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (box_idle(s) || !sort_due(b, s)) return;
    uint32_t v = 0;
    for (int64_t c = tl.begin + threadIdx.x; c < tl.end; c += kBlock) v += b.cstart[c];
    uint32_t total;
    block_exclusive_scan(v, &total);
    if (threadIdx.x == 0) tilesum[t] = total;
}

// per box: exclusive scan of its tiles' totals (in place)
__global__ __launch_bounds__(kBlock) void k_scan_box(const int32_t* __restrict__ active,
                                                      const BoxDev* __restrict__ boxes,
                                                      const BoxState* __restrict__ st,
                                                      uint32_t* __restrict__ tilesum)
{
    const int bx = active[blockIdx.x];
    const BoxState s = st[bx];
    const BoxDev& b = boxes[bx];
    if (box_idle(s) || !sort_due(b, s)) return;
    const int t0 = b.ctile0, nt = b.ctile1 - b.ctile0;
    const int per = (nt + kBlock - 1) / kBlock;
    const int lo = t0 + min(nt, (int)threadIdx.x * per), hi = t0 + min(nt, ((int)threadIdx.x + 1) * per);
    uint32_t v = 0;
    for (int t = lo; t < hi; ++t) v += tilesum[t];
    uint32_t total;
    uint32_t run = block_exclusive_scan(v, &total);
    for (int t = lo; t < hi; ++t) {
        const uint32_t c = tilesum[t];
        tilesum[t] = run;
        run += c;
    }
}

// per cell tile: exclusive scan of counts into starts
__global__ __launch_bounds__(kBlock) void k_scan_apply(const Tile* __restrict__ tiles,
                                                        const BoxDev* __restrict__ boxes,
                                                        const BoxState* __restrict__ st,
                                                        const uint32_t* __restrict__ tilesum)
{
    constexpr int kPer = kCellTile / kBlock;
    const int t = blockIdx.x;
    const Tile tl = tiles[t];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (box_idle(s) || !sort_due(b, s)) return;
    const int64_t c0 = tl.begin + (int64_t)threadIdx.x * kPer;
    uint32_t loc[kPer];
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        loc[j] = (c0 + j < tl.end) ? b.cstart[c0 + j] : 0u;
        v += loc[j];
    }
    uint32_t total;
    const uint32_t start = tilesum[t] + block_exclusive_scan(v, &total);
    // brick boxes: the keys are bricks; their starts are also the bucket
    // starts of the buffer the scatter fills
    uint32_t* __restrict__ next = (b.binning == 1) ? b.bstart[s.parity ^ 1] : nullptr;
    uint32_t run = start;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t c = c0 + j;
        if (c < tl.end) {
            b.cstart[c] = run;
            if (next && c <= b.nbrick) next[c] = run;
        }
        run += loc[j];
    }
    if (tl.end == b.ncell && threadIdx.x == 0) {
        b.cstart[b.ncell] = (uint32_t)b.n;
        if (next && b.nbrick == b.ncell) next[b.nbrick] = (uint32_t)b.n;
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter(const Tile* __restrict__ tiles,
                                                     const BoxDev* __restrict__ boxes,
                                                     const BoxState* __restrict__ st)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (box_idle(s) || !sort_due(b, s)) return;
    const int src = s.parity, dst = s.parity ^ 1;
    const bool stream = (b.binning == 2);
    const bool vacf = b.vacf_stride > 0;
    const float dt = b.dt;
    for (int64_t i = tl.begin + threadIdx.x; i < tl.end; i += kBlock) {
        const int64_t j = (int64_t)b.cstart[b.cell[i]] + b.rank[i];
        const float vx = b.p[src][3][i], vy = b.p[src][4][i], vz = b.p[src][5][i];
        float px = b.p[src][0][i], py = b.p[src][1][i], pz = b.p[src][2][i];
        if (stream) {
            px = fold(fmaf(vx, dt, px), b.len[0]);
            py = fold(fmaf(vy, dt, py), b.len[1]);
            pz = fold(fmaf(vz, dt, pz), b.len[2]);
        }
        b.p[dst][0][j] = px;
        b.p[dst][1][j] = py;
        b.p[dst][2][j] = pz;
        b.p[dst][3][j] = vx;
        b.p[dst][4][j] = vy;
        b.p[dst][5][j] = vz;
        b.pid[dst][j] = b.pid[src][i];
        if (b.m[src]) b.m[dst][j] = b.m[src][i];
        if (vacf) {
            b.v0[dst][0][j] = b.v0[src][0][i];
            b.v0[dst][1][j] = b.v0[src][1][i];
            b.v0[dst][2][j] = b.v0[src][2][i];
        }
    }
}

__global__ void k_flip(const int32_t* __restrict__ active, int nactive,
                       const BoxDev* __restrict__ boxes, BoxState* __restrict__ st)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nactive) return;
    const int bx = active[i];
    BoxState& s = st[bx];
    const bool due = !box_idle(s) && sort_due(boxes[bx], s);
    if (due) s.parity ^= 1;
    s.rebucket = 0;
}

// Angular-momentum-conserving collision of one cell whose particles occupy
// [beg, end) of the current buffer (streamed, SORT binning): the plain
// rotation followed by the rigid-body velocity omega x r' that restores the
// cell's angular momentum about its centre of mass, omega = -I^+ dL.  All
// cell sums are exact fixed point (independent of particle order); the
// per-cell algebra is FP64.
__device__ __forceinline__ void collide_cell_am(const BoxDev& b, int par, long long k, uint32_t c,
                                                uint32_t beg, uint32_t end, float3 sh, double ca,
                                                double sa, long long (&d)[kNumDiag], bool vacf)
{
    const float* __restrict__ px = b.p[par][0];
    const float* __restrict__ py = b.p[par][1];
    const float* __restrict__ pz = b.p[par][2];
    float* __restrict__ vx = b.p[par][3];
    float* __restrict__ vy = b.p[par][4];
    float* __restrict__ vz = b.p[par][5];
    const float* __restrict__ mp = b.m[par];
    const double a = b.a;
    // position inside the shifted cell, each component in [0, a)
    auto local = [&](uint32_t j, double r[3]) {
        const double q[3] = {(double)px[j] - sh.x, (double)py[j] - sh.y, (double)pz[j] - sh.z};
#pragma unroll
        for (int e = 0; e < 3; ++e) r[e] = q[e] - a * floor(q[e] / a);
    };
    // pass 1: mass, momentum, first and second position moments
    long long sw = 0, sv[3] = {0, 0, 0}, s1[3] = {0, 0, 0}, s2[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t j = beg; j < end; ++j) {
        const double mj = mass_of(mp, j);
        double r[3];
        local(j, r);
        sw += fixed_term(mj);
        sv[0] += fixed_term(mj * vx[j]);
        sv[1] += fixed_term(mj * vy[j]);
        sv[2] += fixed_term(mj * vz[j]);
#pragma unroll
        for (int e = 0; e < 3; ++e) s1[e] += fixed_term(mj * r[e]);
        s2[0] += fixed_term(mj * r[0] * r[0]);
        s2[1] += fixed_term(mj * r[0] * r[1]);
        s2[2] += fixed_term(mj * r[0] * r[2]);
        s2[3] += fixed_term(mj * r[1] * r[1]);
        s2[4] += fixed_term(mj * r[1] * r[2]);
        s2[5] += fixed_term(mj * r[2] * r[2]);
    }
    const double M = fixed_to_double((unsigned long long)sw);
    double u[3], rc[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        u[e] = fixed_to_double((unsigned long long)sv[e]) / M;
        rc[e] = fixed_to_double((unsigned long long)s1[e]) / M;
    }
    // sums are in units of 2^-32: Mt is the true mass; u and rc are ratios
    const double k2 = 2.3283064365386963e-10;
    const double Mt = M * k2;
    double Q[3][3];   // second moment of position about the centre of mass
    Q[0][0] = fixed_to_double((unsigned long long)s2[0]) * k2 - Mt * rc[0] * rc[0];
    Q[0][1] = fixed_to_double((unsigned long long)s2[1]) * k2 - Mt * rc[0] * rc[1];
    Q[0][2] = fixed_to_double((unsigned long long)s2[2]) * k2 - Mt * rc[0] * rc[2];
    Q[1][1] = fixed_to_double((unsigned long long)s2[3]) * k2 - Mt * rc[1] * rc[1];
    Q[1][2] = fixed_to_double((unsigned long long)s2[4]) * k2 - Mt * rc[1] * rc[2];
    Q[2][2] = fixed_to_double((unsigned long long)s2[5]) * k2 - Mt * rc[2] * rc[2];
    Q[1][0] = Q[0][1];
    Q[2][0] = Q[0][2];
    Q[2][1] = Q[1][2];
    const float3 ax = cell_axis(b, k, c);
    double nx = ax.x, ny = ax.y, nz = ax.z;
    const double inv = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
    nx *= inv;
    ny *= inv;
    nz *= inv;
    // pass 2: change of the cell's angular momentum under the plain rotation
    long long sl[3] = {0, 0, 0};
    for (uint32_t j = beg; j < end; ++j) {
        const double mj = mass_of(mp, j);
        double r[3], w[3], rw[3];
        local(j, r);
        w[0] = (double)vx[j] - u[0];
        w[1] = (double)vy[j] - u[1];
        w[2] = (double)vz[j] - u[2];
        rotate_w(nx, ny, nz, ca, sa, w, rw);
        const double rp[3] = {r[0] - rc[0], r[1] - rc[1], r[2] - rc[2]};
        const double dw[3] = {rw[0] - w[0], rw[1] - w[1], rw[2] - w[2]};
        sl[0] += fixed_term(mj * (rp[1] * dw[2] - rp[2] * dw[1]));
        sl[1] += fixed_term(mj * (rp[2] * dw[0] - rp[0] * dw[2]));
        sl[2] += fixed_term(mj * (rp[0] * dw[1] - rp[1] * dw[0]));
    }
    const double dL[3] = {fixed_to_double((unsigned long long)sl[0]) * k2,
                          fixed_to_double((unsigned long long)sl[1]) * k2,
                          fixed_to_double((unsigned long long)sl[2]) * k2};
    double I[3][3], Ip[3][3];
    const double tr = Q[0][0] + Q[1][1] + Q[2][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) I[i][j] = (i == j ? tr : 0.0) - Q[i][j];
    sym3_pinv(I, 1e-10, Ip);
    double om[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) om[i] = -(Ip[i][0] * dL[0] + Ip[i][1] * dL[1] + Ip[i][2] * dL[2]);
    // pass 3: rotated relative velocity plus the rigid-body correction
    for (uint32_t j = beg; j < end; ++j) {
        double r[3], w[3], rw[3];
        local(j, r);
        w[0] = (double)vx[j] - u[0];
        w[1] = (double)vy[j] - u[1];
        w[2] = (double)vz[j] - u[2];
        rotate_w(nx, ny, nz, ca, sa, w, rw);
        const double rp[3] = {r[0] - rc[0], r[1] - rc[1], r[2] - rc[2]};
        const float3 v = make_float3((float)(u[0] + rw[0] + (om[1] * rp[2] - om[2] * rp[1])),
                                     (float)(u[1] + rw[1] + (om[2] * rp[0] - om[0] * rp[2])),
                                     (float)(u[2] + rw[2] + (om[0] * rp[1] - om[1] * rp[0])));
        if (vacf) diag_vacf(d, v, b.v0[par][0][j], b.v0[par][1][j], b.v0[par][2][j]);
        vx[j] = v.x;
        vy[j] = v.y;
        vz[j] = v.z;
        diag_particle(d, v, mass_of(mp, j));
    }
}

// SORT path: particles of cell c occupy [cstart[c], cstart[c+1]) in the
// current buffer, already streamed.  One thread per cell.
__global__ __launch_bounds__(kBlock) void k_cell_rotate(const Tile* __restrict__ tiles,
                                                         const BoxDev* __restrict__ boxes,
                                                         const BoxState* __restrict__ st,
                                                         long long* __restrict__ partials)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const Tile tl = tiles[t];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (box_idle(s) || b.binning != 2) return;
    float* __restrict__ vx = b.p[s.parity][3];
    float* __restrict__ vy = b.p[s.parity][4];
    float* __restrict__ vz = b.p[s.parity][5];
    const bool vacf = vacf_due(b, s);
    const float* __restrict__ w0x = b.v0[s.parity][0];
    const float* __restrict__ w0y = b.v0[s.parity][1];
    const float* __restrict__ w0z = b.v0[s.parity][2];
    const float* __restrict__ mp = b.m[s.parity];
    const double ca = b.ca, sa = b.sa;
    long long d[kNumDiag] = {0, 0, 0, 0, 0, 0};
    if (b.conserve_l) {
        const float3 sh = grid_shift(b, s.k);
        for (int64_t c = tl.begin + threadIdx.x; c < tl.end; c += kBlock) {
            const uint32_t beg = b.cstart[c], end = b.cstart[c + 1];
            if (beg != end) collide_cell_am(b, s.parity, s.k, (uint32_t)c, beg, end, sh, ca, sa, d, vacf);
        }
        block_diag(d, partials + (size_t)t * kNumDiag);
        return;
    }
    for (int64_t c = tl.begin + threadIdx.x; c < tl.end; c += kBlock) {
        const uint32_t beg = b.cstart[c], end = b.cstart[c + 1];
        if (beg == end) continue;
        unsigned long long sx = 0, sy = 0, sz = 0, sw = 0;
        for (uint32_t j = beg; j < end; ++j) {
            const float mj = mass_of(mp, j);
            sx += to_fixed(mj * vx[j]);
            sy += to_fixed(mj * vy[j]);
            sz += to_fixed(mj * vz[j]);
            sw += to_fixed(mj);
        }
        CellUN u;
        u.ux = fixed_mean(sx, sw);
        u.uy = fixed_mean(sy, sw);
        u.uz = fixed_mean(sz, sw);
        const float3 ax = cell_axis(b, s.k, (uint32_t)c);
        u.nx = ax.x;
        u.ny = ax.y;
        u.nz = ax.z;
        u.kappa = axis_kappa(ax);
        for (uint32_t j = beg; j < end; ++j) {
            const float3 v = rotate_about(u, vx[j], vy[j], vz[j], ca, sa);
            vx[j] = v.x;
            vy[j] = v.y;
            vz[j] = v.z;
            diag_particle(d, v, mass_of(mp, j));
            if (vacf) diag_vacf(d, v, w0x[j], w0y[j], w0z[j]);
        }
    }
    block_diag(d, partials + (size_t)t * kNumDiag);
}

// --------------------------------------------------------------------------
// end of step: per-box reduction of the partials in a fixed order

__global__ __launch_bounds__(kBlock) void k_box_finish(const int32_t* __restrict__ active,
                                                        const BoxDev* __restrict__ boxes,
                                                        BoxState* __restrict__ st,
                                                        const long long* __restrict__ partials_b,
                                                        const long long* __restrict__ partials_c)
{
    const int bx = active[blockIdx.x];
    BoxState* sp = &st[bx];
    if (box_idle(*sp)) return;
    const BoxDev& b = boxes[bx];
    const bool by_cell = (b.binning == 2);
    const int t0 = by_cell ? b.ctile0 : b.btile0;
    const int t1 = by_cell ? b.ctile1 : b.btile1;
    const long long* __restrict__ partials = by_cell ? partials_c : partials_b;
    // exact sum of the 64-bit tile partials as (high, low) 32-bit halves
    long long hi[kNumDiag] = {0, 0, 0, 0, 0, 0}, lo[kNumDiag] = {0, 0, 0, 0, 0, 0};
    for (int t = t0 + (int)threadIdx.x; t < t1; t += kBlock) {
#pragma unroll
        for (int j = 0; j < kNumDiag; ++j) {
            const long long v = partials[(size_t)t * kNumDiag + j];
            hi[j] += v >> 32;
            lo[j] += (long long)(unsigned long long)(unsigned)(v & 0xffffffffll);
        }
    }
    __shared__ long long thi[kNumDiag], tlo[kNumDiag];
    block_diag(hi, thi);
    __syncthreads();
    block_diag(lo, tlo);
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[kNumDiag];
        for (int j = 0; j < kNumDiag; ++j)   // (hi 2^32 + lo) 2^-32, one rounding
            tot[j] = (double)thi[j] + (double)tlo[j] * 2.3283064365386963e-10;
        const bool vac = vacf_due(b, *sp);
        sp->diag[0] = tot[0];
        sp->diag[1] = tot[1];
        sp->diag[2] = tot[2];
        sp->diag[3] = tot[3];
        if (thi[5] != 0 || tlo[5] != 0) sp->status = -5;   // velocity out of range / not finite
        if (vac && sp->vacf_len < b.vacf_cap && b.n > 0)
            b.vacf[sp->vacf_len++] = tot[4] / (double)b.n;
        sp->k += 1;
        if (sp->remaining > 0) sp->remaining -= 1;
        if (!by_cell) sp->parity ^= 1;   // the brick rotation wrote the other buffer
    }
}

// --------------------------------------------------------------------------
// initial state on the device (not part of the step)

__global__ __launch_bounds__(kBlock) void k_init_maxwell(const Tile* __restrict__ tiles,
                                                          const BoxDev* __restrict__ boxes,
                                                          const BoxState* __restrict__ st,
                                                          float vscale, long long* __restrict__ partials)
{
    const int t = blockIdx.x;
    const Tile tl = tiles[t];
    const BoxDev& b = boxes[tl.box];
    const int par = st[tl.box].parity;
    long long d[kNumDiag] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = tl.begin + threadIdx.x; i < tl.end; i += kBlock) {
        const uint32_t lo = (uint32_t)i, hi = (uint32_t)((uint64_t)i >> 32);
        const uint4 r = philox4x32_10(make_uint4(lo, hi, 0u, 2u), b.key0, b.key1);
        b.p[par][0][i] = fold(b.len[0] * unit24(r.x), b.len[0]);
        b.p[par][1][i] = fold(b.len[1] * unit24(r.y), b.len[1]);
        b.p[par][2][i] = fold(b.len[2] * unit24(r.z), b.len[2]);
        const uint4 q = philox4x32_10(make_uint4(lo, hi, 0u, 3u), b.key0, b.key1);
        const float r1 = sqrtf(-2.0f * logf(1.0f - unit24(q.x)));
        const float r2 = sqrtf(-2.0f * logf(1.0f - unit24(q.z)));
        float s1, c1, s2, c2;
        sincosf(6.2831853071795864769f * unit24(q.y), &s1, &c1);
        sincosf(6.2831853071795864769f * unit24(q.w), &s2, &c2);
        const float vx = vscale * r1 * c1, vy = vscale * r1 * s1, vz = vscale * r2 * c2;
        b.p[par][3][i] = vx;
        b.p[par][4][i] = vy;
        b.p[par][5][i] = vz;
        b.pid[par][i] = (int32_t)i;
        diag_particle(d, make_float3(vx, vy, vz), 1.0f);
    }
    block_diag(d, partials + (size_t)t * kNumDiag);
}

// v <- (v - V) * scale; partial sums of v^2 before scaling and of v after
__global__ __launch_bounds__(kBlock) void k_init_adjust(const Tile* __restrict__ tiles,
                                                         const BoxDev* __restrict__ boxes,
                                                         const BoxState* __restrict__ st,
                                                         float mx, float my, float mz, float scale,
                                                         long long* __restrict__ partials)
{
    const int t = blockIdx.x;
    const Tile tl = tiles[t];
    const BoxDev& b = boxes[tl.box];
    const int par = st[tl.box].parity;
    long long d[kNumDiag] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = tl.begin + threadIdx.x; i < tl.end; i += kBlock) {
        const float vx = (b.p[par][3][i] - mx) * scale;
        const float vy = (b.p[par][4][i] - my) * scale;
        const float vz = (b.p[par][5][i] - mz) * scale;
        b.p[par][3][i] = vx;
        b.p[par][4][i] = vy;
        b.p[par][5][i] = vz;
        diag_particle(d, make_float3(vx, vy, vz), 1.0f);
    }
    block_diag(d, partials + (size_t)t * kNumDiag);
}

// v0 <- v, and the FP64 partials of the current state (sum v, sum v^2, sum v.v0)
__global__ __launch_bounds__(kBlock) void k_snapshot(const Tile* __restrict__ tiles,
                                                      const BoxDev* __restrict__ boxes,
                                                      const BoxState* __restrict__ st,
                                                      int set_v0, long long* __restrict__ partials)
{
    const int t = blockIdx.x;
    const Tile tl = tiles[t];
    const BoxDev& b = boxes[tl.box];
    const int par = st[tl.box].parity;
    const bool has_v0 = b.vacf_stride > 0;
    long long d[kNumDiag] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = tl.begin + threadIdx.x; i < tl.end; i += kBlock) {
        const float vx = b.p[par][3][i], vy = b.p[par][4][i], vz = b.p[par][5][i];
        if (has_v0 && set_v0) {
            b.v0[par][0][i] = vx;
            b.v0[par][1][i] = vy;
            b.v0[par][2][i] = vz;
        }
        diag_particle(d, make_float3(vx, vy, vz), mass_of(b.m[par], i));
        if (has_v0) diag_vacf(d, make_float3(vx, vy, vz), b.v0[par][0][i], b.v0[par][1][i], b.v0[par][2][i]);
    }
    block_diag(d, partials + (size_t)t * kNumDiag);
}

__global__ __launch_bounds__(kBlock) void k_fill_iota(int32_t* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_fill_f32(float* __restrict__ p, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

// dst[i] = src[pid[i]] (gather_by_id) or dst[pid[i]] = src[i] (scatter_by_id);
// pid is a permutation of [0, n)
__global__ __launch_bounds__(kBlock) void k_permute_f32(float* __restrict__ dst, const float* __restrict__ src,
                                                         const int32_t* __restrict__ pid, int64_t n,
                                                         int scatter)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int64_t j = pid[i];
        if (j < 0 || j >= n) continue;
        if (scatter)
            dst[j] = src[i];
        else
            dst[i] = src[j];
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_zero_u32(uint32_t* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = 0u;
}

// --------------------------------------------------------------------------
// host launchers

#define MPCD_LAUNCH(kern, grid, block, stream, ...)                              \
    do {                                                                          \
        if ((grid) > 0) hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, stream, __VA_ARGS__); \
    } while (0)

void launch_brick_accumulate(const Tables& T, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {   // allow windows above the default 64 KiB of dynamic LDS
        (void)hipFuncSetAttribute((const void*)k_brick_accumulate,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  max_window_records() * (int)sizeof(CellAcc));
        attr = true;
    }
    const size_t lds = (size_t)T.max_wsize * sizeof(CellAcc);
    if (T.nbtiles > 0)
        hipLaunchKernelGGL(k_brick_accumulate, dim3(T.nbtiles), dim3(kBlock), lds, s, T.btiles, T.boxes,
                           T.state);
}
void launch_brick_scan(const Tables& T, hipStream_t s)
{
    MPCD_LAUNCH(k_brick_sizes, (T.nbtiles + kBlock - 1) / kBlock, kBlock, s, T.btiles, T.nbtiles, T.boxes,
                T.state);
    MPCD_LAUNCH(k_brick_scan, T.nactive, kBlock, s, T.active, T.boxes, T.state);
    MPCD_LAUNCH(k_brick_offsets, (T.nbtiles * 27 + kBlock - 1) / kBlock, kBlock, s, T.btiles, T.nbtiles,
                T.boxes, T.state);
}
void launch_brick_finalize(const Tables& T, hipStream_t s)
{
    MPCD_LAUNCH(k_brick_finalize, T.nctiles, kBlock, s, T.ctiles, T.boxes, T.state);
}
void launch_brick_rotate(const Tables& T, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)k_brick_rotate, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  max_window_records() * (int)sizeof(CellUN));
        attr = true;
    }
    const size_t lds = (size_t)T.max_wsize * sizeof(CellUN);
    if (T.nbtiles > 0)
        hipLaunchKernelGGL(k_brick_rotate, dim3(T.nbtiles), dim3(kBlock), lds, s, T.btiles, T.boxes, T.state,
                           T.partials_b);
}
void launch_box_finish(const Tables& T, hipStream_t s)
{
    MPCD_LAUNCH(k_box_finish, T.nactive, kBlock, s, T.active, T.boxes, T.state, T.partials_b,
                T.partials_c);
}
void launch_zero_counts(const Tables& T, hipStream_t s)
{
    MPCD_LAUNCH(k_zero_counts, T.nctiles, kBlock, s, T.ctiles, T.boxes, T.state);
}
void launch_count(const Tables& T, hipStream_t s)
{
    MPCD_LAUNCH(k_count, T.nptiles, kBlock, s, T.ptiles, T.boxes, T.state);
}
void launch_scan(const Tables& T, hipStream_t s)
{
    MPCD_LAUNCH(k_scan_tilesum, T.nctiles, kBlock, s, T.ctiles, T.boxes, T.state, T.tilesum);
    MPCD_LAUNCH(k_scan_box, T.nactive, kBlock, s, T.active, T.boxes, T.state, T.tilesum);
    MPCD_LAUNCH(k_scan_apply, T.nctiles, kBlock, s, T.ctiles, T.boxes, T.state, T.tilesum);
}
void launch_scatter(const Tables& T, hipStream_t s)
{
    MPCD_LAUNCH(k_scatter, T.nptiles, kBlock, s, T.ptiles, T.boxes, T.state);
}
void launch_flip(const Tables& T, hipStream_t s)
{
    MPCD_LAUNCH(k_flip, (T.nactive + kBlock - 1) / kBlock, kBlock, s, T.active, T.nactive, T.boxes,
                T.state);
}
void launch_cell_rotate(const Tables& T, hipStream_t s)
{
    MPCD_LAUNCH(k_cell_rotate, T.nctiles, kBlock, s, T.ctiles, T.boxes, T.state, T.partials_c);
}

// Largest window (in records) one brick workgroup may hold in LDS.
int max_window_records() { return (int)(96 * 1024 / sizeof(CellAcc)); }

// The init/snapshot launchers take a sub-range of T.ptiles (one box); their
// partials land at the same tile indices as the step's.
static long long* partials_at(const Tile* tiles, const Tables& T)
{
    return T.partials + (size_t)(tiles - T.ptiles) * kNumDiag;
}
void launch_init_maxwell(const Tile* tiles, int ntiles, const Tables& T, float vscale, hipStream_t s)
{
    MPCD_LAUNCH(k_init_maxwell, ntiles, kBlock, s, tiles, T.boxes, T.state, vscale, partials_at(tiles, T));
}
void launch_init_adjust(const Tile* tiles, int ntiles, const Tables& T, float mx, float my, float mz,
                        float scale, hipStream_t s)
{
    MPCD_LAUNCH(k_init_adjust, ntiles, kBlock, s, tiles, T.boxes, T.state, mx, my, mz, scale,
                partials_at(tiles, T));
}
void launch_snapshot(const Tile* tiles, int ntiles, const Tables& T, int set_v0, hipStream_t s)
{
    MPCD_LAUNCH(k_snapshot, ntiles, kBlock, s, tiles, T.boxes, T.state, set_v0, partials_at(tiles, T));
}
void launch_fill_iota(int32_t* p, int64_t n, hipStream_t s)
{
    const int64_t g = (n + kBlock - 1) / kBlock;
    MPCD_LAUNCH(k_fill_iota, (int)(g < 65536 ? g : 65536), kBlock, s, p, n);
}
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s)
{
    const int64_t g = (n + kBlock - 1) / kBlock;
    MPCD_LAUNCH(k_fill_f32, (int)(g < 65536 ? g : 65536), kBlock, s, p, n, v);
}
void launch_permute_f32(float* dst, const float* src, const int32_t* pid, int64_t n, int scatter, hipStream_t s)
{
    const int64_t g = (n + kBlock - 1) / kBlock;
    MPCD_LAUNCH(k_permute_f32, (int)(g < 65536 ? g : 65536), kBlock, s, dst, src, pid, n, scatter);
}
void launch_fill_zero_u32(uint32_t* p, int64_t n, hipStream_t s)
{
    const int64_t g = (n + kBlock - 1) / kBlock;
    MPCD_LAUNCH(k_fill_zero_u32, (int)(g < 65536 ? g : 65536), kBlock, s, p, n);
}

}  // namespace mpcd
