// mpcd_kernels.hip -- HIP kernels of the SRD step for gfx950 (MI355X).
//
// One step of a box (paper Sec. 2; shifted grid of Sec. 3.1, Listing 1;
// mass-weighted cell velocity of Sec. 3.3, Listing 4) runs as:
//
//   ATOMIC binning (particles bucketed by the brick of their collision cell)
//     k_brick_step        per brick, one pass: stream, exact LDS cell sums,
//                         u_c = sum(m v)/sum(m) and axis n_c from Philox,
//                         v <- u_c + R(n_c, alpha)(v - u_c), then the particle
//                         goes straight into the bucket of the brick holding
//                         its next-step collision cell; range check and VACF
//                         terms.  Instances: per-particle masses (kMass), the
//                         angular-momentum rule (kAM: moment, angular-momentum
//                         and omega passes), 64-bit store offsets (kWide)
//     k_box_finish        per box: particles of the overflow bucket (rare),
//                         reduce diagnostics, VACF sample, k++
//   Re-bucketing (after admission / set_state, or when a bucket overflowed):
//     k_mark_holes, k_rebucket_clear, then the counting sort below keyed by
//     brick, which also sets the bucket capacities
//
//   SORT binning (counting sort by collision cell every step)
//     zero, k_count (streamed collision cell + rank), scan, k_scatter (the
//     permutation; under the angular-momentum rule the particles themselves,
//     streamed), flip, k_cell_rotate (gathers runs of cells through the
//     permutation and streams them, one thread per cell for the sums),
//     k_box_finish
//
// Per box, outside the step: k_init_maxwell / k_init_adjust (initial state),
// k_snapshot (exact momentum and energy on demand), k_box_stats(_tiles)
// (exact 128-bit reduction of their per-tile partials on the device).
//
// Both paths sum the momentum of a cell exactly (64-bit fixed point), so
// they produce bit-identical velocities whatever the order of the atomics.
// All kernels grid over "tiles" (contiguous slot, cell or brick ranges of one
// box), which lets one launch advance many boxes of different sizes.
#include <type_traits>

#include "mpcd_dev.h"
#include "mpcd_launch.h"

namespace mpcd {

// --------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ bool box_idle(const BoxState& s) { return s.remaining == 0; }

// Values the whole workgroup shares (read from the box tables), made
// explicitly uniform so that addresses derived from them stay in scalar
// registers.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uniform(long long v)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffll));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}
// A box array's global address, made wavefront-uniform so that it stays in
// scalar registers (the address of each access is then that base plus a
// 32-bit lane offset, with no per-lane 64-bit add).
template <class T>
__device__ __forceinline__ MPCD_G T* ugp(T* p)
{
    return (MPCD_G T*)(uintptr_t)(unsigned long long)uniform((long long)(uintptr_t)p);
}

// The counting sort runs every step for SORT boxes, and once for brick
// boxes whose particles are not bucketed yet (after admission / set_state).
__device__ __forceinline__ bool sort_due(const BoxDev& b, const BoxState& s)
{
    return b.binning == 2 || s.rebucket != 0;
}

// Slots the counting sort reserves for key c holding n particles: n for
// cells (SORT), n plus slack for bricks (brick boxes re-bucketing).
__device__ __forceinline__ uint32_t key_capacity(const BoxDev& b, int64_t c, uint32_t n)
{
    return (b.binning == 1 && c < b.nbrick) ? n + bucket_slack(n) : n;
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

// Particle tile blockIdx.x of one box (per-box launches): slots
// [t kPartTile, (t + 1) kPartTile) clipped to the box's slot count.
__device__ __forceinline__ Tile box_tile(const BoxDev* __restrict__ boxes, int box)
{
    const int64_t begin = (int64_t)blockIdx.x * kPartTile;
    return Tile{box, 0, begin, min(boxes[box].nslot, begin + (int64_t)kPartTile)};
}

// Block sum of kNumDiag exact partials; threads 0..kNumDiag-1 write out[].
template <int kT = kBlock>
__device__ __forceinline__ void block_diag(long long (&d)[kNumDiag], long long* out)
{
    __shared__ long long red[kT / kWave][kNumDiag];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < kNumDiag; ++j) {
        const long long v = wave_sum(d[j]);
        if (lane == 0) red[w][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < kNumDiag) {
        long long v = 0;
        for (int i = 0; i < kT / kWave; ++i) v += red[i][threadIdx.x];
        out[threadIdx.x] = v;
    }
}

// End of a step kernel's workgroup: add its exact VACF partial (on sampled
// steps) and a range-violation mark to the box's accumulators.  Atomic
// integer adds are exact, so the order does not matter; the workgroups are
// spread over kAccLanes lanes per box (high and low 32-bit halves of the
// VACF sum, so no lane can overflow).
template <int kT = kBlock>
__device__ __forceinline__ void step_flush(const long long (&d)[kNumDiag], bool vacf, long long* acc, int lane_sel)
{
    __shared__ long long red[kT / kWave];
    const int any = __syncthreads_or(d[5] != 0);
    long long* a = acc + (size_t)(lane_sel & (kAccLanes - 1)) * 3;
    if (vacf) {
        const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
        const long long v = wave_sum(d[4]);
        if (lane == 0) red[w] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            long long t = 0;
            for (int i = 0; i < kT / kWave; ++i) t += red[i];
            gatomic_add(gp(a), t >> 32);
            gatomic_add(gp(a) + 1, (long long)(unsigned long long)(unsigned)(t & 0xffffffffll));
        }
    }
    if (any && threadIdx.x == 0) gatomic_add(gp(a) + 2, 1ll);
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

// Element at byte offset o of a global array (a 32-bit offset from a
// uniform base lets one address register serve every array of a slot).
template <class T>
__device__ __forceinline__ T ldg(const MPCD_G T* p, uint32_t o)
{
    return *(const MPCD_G T*)((const MPCD_G char*)p + o);
}
template <class T>
__device__ __forceinline__ void stg(MPCD_G T* p, uint32_t o, T v)
{
    *(MPCD_G T*)((MPCD_G char*)p + o) = v;
}
// the same with a 64-bit byte offset (buffers of 2^30 slots or more)
template <class T>
__device__ __forceinline__ void stg(MPCD_G T* p, unsigned long long o, T v)
{
    *(MPCD_G T*)((MPCD_G char*)p + o) = v;
}

// Collision cell, at step k+1, of a particle at (x, y, z) that leaves step k
// with velocity v: the stream of step k+1 and its shifted grid (the same
// arithmetic the next step applies).
__device__ __forceinline__ int3 next_cell(const BoxDev& b, float x, float y, float z, float3 v, float3 sh1)
{
    const float qx = fold(fmaf(v.x, b.dt, x), b.len[0]);
    const float qy = fold(fmaf(v.y, b.dt, y), b.len[1]);
    const float qz = fold(fmaf(v.z, b.dt, z), b.len[2]);
    return make_int3(axis_cell(qx, sh1.x, b.inv_a, b.L[0]), axis_cell(qy, sh1.y, b.inv_a, b.L[1]),
                     axis_cell(qz, sh1.z, b.inv_a, b.L[2]));
}

__device__ __forceinline__ int3 brick_of_cell(const BoxDev& b, int3 c)
{
    return make_int3(brick_of(c.x, b.bshift[0]), brick_of(c.y, b.bshift[1]), brick_of(c.z, b.bshift[2]));
}

// One slot of bucket `dest` of buffer `dst`, reserved alone; false when the
// bucket is full.
__device__ __forceinline__ bool place_single(const BoxDev& b, int dst, uint32_t dest, uint32_t* j)
{
    const uint32_t p = gatomic_add(gp(b.bsize[dst]) + dest, 1u);
    const uint32_t b0 = gp(b.bstart)[dest];
    if (p < gp(b.bstart)[dest + 1] - b0) {
        *j = b0 + p;
        return true;
    }
    return false;
}

// A slot of the overflow bucket of buffer `dst` for a particle whose bucket
// is full.  Its share of the next step's cell sums (cell nc, mass m, velocity
// v) goes to the exact escape sums of step k+1, and the brick owning nc is
// flagged to add them.  False only when the overflow bucket is full, which
// its capacity (every particle of the box) rules out.
__device__ __forceinline__ bool place_overflow(const BoxDev& b, int dst, long long k, int3 nc, float m,
                                               float3 v, uint32_t* j)
{
    const uint32_t nbk = (uint32_t)b.nbrick;
    const uint32_t o = gatomic_add(gp(b.bsize[dst]) + nbk, 1u);
    const uint32_t ob = gp(b.bstart)[nbk];
    if (o >= gp(b.bstart)[nbk + 1] - ob) return false;
    *j = ob + o;
    const uint32_t c = (uint32_t)nc.x + (uint32_t)b.L[0] * ((uint32_t)nc.y + (uint32_t)b.L[1] * (uint32_t)nc.z);
    MPCD_G CellAcc* e = gp(b.esc[(k + 1) & 1]) + c;
    gatomic_add(&e->sx, to_fixed(m * v.x));
    gatomic_add(&e->sy, to_fixed(m * v.y));
    gatomic_add(&e->sz, to_fixed(m * v.z));
    gatomic_add(&e->w, to_fixed(m));
    if (b.ecnt[0]) gatomic_add(gp(b.ecnt[(k + 1) & 1]) + c, 1u);   // masses: w is no count
    const int3 br = brick_of_cell(b, nc);
    gp(b.eflag)[(size_t)((k + 1) & 1) * b.nbrick + br.x + b.nb[0] * (br.y + b.nb[1] * br.z)] = (uint32_t)(k + 2);
    return true;
}

// Store particle state at slot j of buffer dst.
__device__ __forceinline__ void put_particle(const BoxDev& b, int dst, uint32_t j, float x, float y, float z,
                                             float3 v, int32_t id, float m, bool has_m)
{
    const unsigned long long o = (unsigned long long)j * 4u;
    stg(gp(b.p[dst][0]), o, x);
    stg(gp(b.p[dst][1]), o, y);
    stg(gp(b.p[dst][2]), o, z);
    stg(gp(b.p[dst][3]), o, v.x);
    stg(gp(b.p[dst][4]), o, v.y);
    stg(gp(b.p[dst][5]), o, v.z);
    if (b.pid[dst]) stg(gp(b.pid[dst]), o, id);
    if (has_m) stg(gp(b.m[dst]), o, m);
}

// VACF term of particle `id` with new velocity v.  The reference velocities
// v(0) stay in particle-id order (one 16-byte record each), so particles can
// move between slots without carrying them; they are read only on the steps
// that take a sample.
__device__ __forceinline__ void vacf_term(const BoxDev& b, int32_t id, float3 v, long long (&d)[kNumDiag])
{
    const f32x4 w = *((const MPCD_G f32x4*)gp(b.v0) + id);
    diag_vacf(d, v, w.x, w.y, w.z);
}

// One SRD step of one brick (paper Sec. 2; the shifted grid of Sec. 3.1;
// the mass-weighted cell velocity of Sec. 3.3).  The workgroup owns every
// particle whose collision cell lies in its brick, so the whole step is one
// pass over them, held in registers (kS per thread; larger buckets take
// several chunks, re-read from memory):
//   1. stream, collision cell, exact fixed-point cell sums in LDS
//      (+ escape sums of overflow particles, when flagged)
//   2. per cell: u_c = sum(m v)/sum(m), axis n_c from Philox (in place)
//   3. rotate v about n_c relative to u_c; collision cell of the next step;
//      rank in the destination group (27 neighbour bricks: wave ballots for
//      the particles that stay, LDS counters for the others)
//   4. one global reservation per group in the destination buckets, then
//      stores.  Per step only the range check (and the VACF sum when a
//      sample is due) is reduced; momentum and energy are summed on demand.
// The instance for equal masses without particle ids (the benchmark's) is
// held to 5 waves per SIMD (96 registers, a few spilled): measured 6 %
// faster than 4 waves with no spill, while 6 waves (80 registers) and the
// instances with ids at 5 waves are slower.
template <int kT, int kS, bool kMass, bool kAM, bool kWide, bool kIds>
__global__ __launch_bounds__(kT)
__attribute__((amdgpu_waves_per_eu(kMass || kAM ? 1 : (kIds || kS > 6 ? 4 : 5), kMass || kAM || kIds || kS > 6 ? 8 : 5)))
void k_brick_step(const Tile* __restrict__ tiles, int one_box, const BoxDev* __restrict__ boxes,
                  const BoxState* __restrict__ st, long long* __restrict__ dacc)
{
    // LDS, per cell of the brick: exact sums of m v (3 x 64 bit) and of m (64
    // bit, or a 32-bit count for equal masses) in 40-byte records, then u_c,
    // n_c and kappa in 48-byte records (two 16-byte reads); both strides
    // spread neighbouring cells over the LDS banks.  Boxes with the
    // angular-momentum rule (kAM instances only) use kAmWords per cell instead.
    extern __shared__ __align__(16) unsigned long long lds64[];
    __shared__ uint32_t gcnt[27], gpos[27], gbeg[27], gcap[27];
    constexpr uint32_t kChunk = (uint32_t)kT * kS;
    constexpr uint32_t kNone = 0xffffffffu;   // no particle / no cell
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    // with a single brick box the brick tiles are its bricks in order, and
    // the tile record need not be loaded before the box's
    const Tile tl = one_box >= 0 ? Tile{one_box, 0, t, t + 1} : tiles[t];
    const BoxState s = st[uniform(tl.box)];
    const BoxDev& b = boxes[uniform(tl.box)];
    if (box_idle(s) || b.binning != 1) return;
    const int brick = uniform((int)tl.begin);
    const long long k = uniform(s.k);
    const int src = uniform(s.parity), dst = src ^ 1;
    const bool vacf = b.vacf_stride > 0 && ((k + 1 - uniform(s.vacf_origin)) % b.vacf_stride) == 0;
    const int nb0 = b.nb[0], nb1 = b.nb[1], nb2 = b.nb[2];
    const int bx = brick % nb0, by = (brick / nb0) % nb1, bz = brick / (nb0 * nb1);
    const int lox = brick_lo(bx, b.bshift[0]), loy = brick_lo(by, b.bshift[1]), loz = brick_lo(bz, b.bshift[2]);
    const int ex = min(1 << b.bshift[0], b.L[0] - lox);
    const int ey = min(1 << b.bshift[1], b.L[1] - loy);
    const int ez = min(1 << b.bshift[2], b.L[2] - loz);
    const int ncl = ex * ey * ez;
    const bool am = kAM && b.conserve_l != 0;
    unsigned long long* const acc = lds64;   // [ncl][kAccWords]: sx, sy, sz, w
    float* const fu = reinterpret_cast<float*>(lds64 + ((kAccWords * ncl + 1) & ~1));   // [ncl][kUnWords]
    for (int i = threadIdx.x; i < (am ? kAmWords : kAccWords) * ncl; i += kT) lds64[i] = 0ull;
    const uint32_t beg = (uint32_t)uniform((int)gp(b.bstart)[brick]);
    // escape sums for this brick (overflow particles of the previous step):
    // flagged during that step, in the half of eflag this step only reads,
    // so the load goes out with the bucket's and is not waited for here
    const uint32_t stamp = (uint32_t)(k + 1);
    const uint32_t eflag_k = gp(b.eflag)[(size_t)(k & 1) * b.nbrick + brick];
    // the bucket's fill, read by every wave (this workgroup alone reads it and
    // clears it at the end, since this buffer is the next step's destination)
    const uint32_t cnt = min((uint32_t)uniform((int)gp(b.bsize[src])[brick]),
                             (uint32_t)uniform((int)gp(b.bstart)[brick + 1]) - beg);
    __syncthreads();
    const int nch = (int)((cnt + kChunk - 1) / kChunk);

    // bucket-relative bases (uniform): a lane's offset is its index in the bucket
    const MPCD_G float* __restrict__ ix = ugp(b.p[src][0]) + beg;
    const MPCD_G float* __restrict__ iy = ugp(b.p[src][1]) + beg;
    const MPCD_G float* __restrict__ iz = ugp(b.p[src][2]) + beg;
    const MPCD_G float* __restrict__ ivx = ugp(b.p[src][3]) + beg;
    const MPCD_G float* __restrict__ ivy = ugp(b.p[src][4]) + beg;
    const MPCD_G float* __restrict__ ivz = ugp(b.p[src][5]) + beg;
    const bool has_mass = kMass && b.m[src] != nullptr;   // uniform
    const MPCD_G float* __restrict__ im = has_mass ? ugp(b.m[src]) + beg : nullptr;
    const float3 sh = grid_shift(b, k);
    const float dt = b.dt;
    const float inv_a = b.inv_a;

    float px[kS], py[kS], pz[kS], vx[kS], vy[kS], vz[kS], pm[kS];
    uint32_t meta[kS];   // cell in the brick after loading; destination group << 24 | rank later
    long long d[kNumDiag] = {};
    // load and stream chunk ch; meta <- cell inside the brick, kNone past the
    // end of the bucket or for a particle in the wrong bucket (never happens:
    // both sides use the same arithmetic; flagged if it does)
    // slots of chunk ch that hold particles for some thread (uniform)
    auto used_slots = [&](int ch) -> int {
        const uint32_t rem = cnt - (uint32_t)ch * kChunk;
        return (int)min((uint32_t)kS, (rem + kT - 1) / kT);
    };
    auto load = [&](int ch) {
        const int nu = used_slots(ch);
#pragma unroll
        for (int u = 0; u < kS; ++u) {   // issue every load first
            if (u >= nu) break;
            const uint32_t i = (uint32_t)ch * kChunk + (uint32_t)(u * kT) + threadIdx.x;
            const uint32_t o = (i < cnt ? i : 0u) * 4u;   // byte offset inside the bucket
            px[u] = ldg(ix, o);
            py[u] = ldg(iy, o);
            pz[u] = ldg(iz, o);
            vx[u] = ldg(ivx, o);
            vy[u] = ldg(ivy, o);
            vz[u] = ldg(ivz, o);
            pm[u] = has_mass ? ldg(im, o) : 1.0f;
        }
#pragma unroll
        for (int u = 0; u < kS; ++u) {
            if (u >= nu) {
                meta[u] = kNone;
                continue;
            }
            const uint32_t i = (uint32_t)ch * kChunk + (uint32_t)(u * kT) + threadIdx.x;
            px[u] = fold(fmaf(vx[u], dt, px[u]), b.len[0]);
            py[u] = fold(fmaf(vy[u], dt, py[u]), b.len[1]);
            pz[u] = fold(fmaf(vz[u], dt, pz[u]), b.len[2]);
            const int cx = axis_cell_raw(px[u], sh.x, inv_a, b.L[0]) - lox;   // range-checked below
            const int cy = axis_cell_raw(py[u], sh.y, inv_a, b.L[1]) - loy;
            const int cz = axis_cell_raw(pz[u], sh.z, inv_a, b.L[2]) - loz;
            const bool in = (unsigned)cx < (unsigned)ex && (unsigned)cy < (unsigned)ey && (unsigned)cz < (unsigned)ez;
            meta[u] = (i < cnt && in) ? (uint32_t)(cx + ex * (cy + ey * cz)) : kNone;
            if (i < cnt && !in) d[5] += 1;
        }
    };

    // 1. cell sums; the last chunk first, so that chunk 0 stays in registers
    for (int ch = nch - 1; ch >= 0; --ch) {
        load(ch);
#pragma unroll
        for (int u = 0; u < kS; ++u) {
            const uint32_t c = meta[u];
            if (c == kNone) continue;
            if (kAM && am) {   // moments of the angular-momentum rule
                double rl[3];
                long long tm[kAmMoments];
                am_local(b.a, px[u], py[u], pz[u], sh, rl);
                am_moments((double)pm[u], vx[u], vy[u], vz[u], rl, tm);
                unsigned long long* const ra = acc + (size_t)c * kAmWords;
#pragma unroll
                for (int q = 0; q < kAmMoments; ++q) atomicAdd(&ra[q], (unsigned long long)tm[q]);
                atomicAdd(&ra[kAmMoments], 1ull);   // particle count (free until pass 2a)
                continue;
            }
            unsigned long long* const r = acc + (size_t)c * kAccWords;
            if (kMass) {
                const float mi = pm[u];
                atomicAdd(&r[0], to_fixed(mi * vx[u]));
                atomicAdd(&r[1], to_fixed(mi * vy[u]));
                atomicAdd(&r[2], to_fixed(mi * vz[u]));
                atomicAdd(&r[3], to_fixed(mi));
                atomicAdd(reinterpret_cast<uint32_t*>(&r[4]), 1u);   // particle count
            } else {   // equal masses: r[3] counts particles
                atomicAdd(&r[0], to_fixed(vx[u]));
                atomicAdd(&r[1], to_fixed(vy[u]));
                atomicAdd(&r[2], to_fixed(vz[u]));
                atomicAdd(reinterpret_cast<uint32_t*>(&r[3]), 1u);
            }
        }
    }
    __syncthreads();
    const bool flagged = eflag_k == stamp;
    const uint32_t L0 = (uint32_t)b.L[0], L01 = (uint32_t)b.L[0] * (uint32_t)b.L[1];
    // Angular-momentum rule, flagged brick: the particles of this step's
    // overflow bucket whose collision cell lies here are read directly (pass
    // 1: moments, pass 2: angular-momentum change), as their escape sums
    // carry no moments.
    auto am_overflow = [&](int pass) {
        const uint32_t nbk = (uint32_t)b.nbrick;
        const uint32_t ob = gp(b.bstart)[nbk];
        const uint32_t ocnt = min(gp(b.bsize[src])[nbk], gp(b.bstart)[nbk + 1] - ob);
        for (uint32_t q = threadIdx.x; q < ocnt; q += kT) {
            const uint32_t si = ob + q;
            const float ux = gp(b.p[src][3])[si], uy = gp(b.p[src][4])[si], uz = gp(b.p[src][5])[si];
            const float qx = fold(fmaf(ux, dt, gp(b.p[src][0])[si]), b.len[0]);
            const float qy = fold(fmaf(uy, dt, gp(b.p[src][1])[si]), b.len[1]);
            const float qz = fold(fmaf(uz, dt, gp(b.p[src][2])[si]), b.len[2]);
            const int cx = axis_cell(qx, sh.x, inv_a, b.L[0]) - lox;
            const int cy = axis_cell(qy, sh.y, inv_a, b.L[1]) - loy;
            const int cz = axis_cell(qz, sh.z, inv_a, b.L[2]) - loz;
            if ((unsigned)cx >= (unsigned)ex || (unsigned)cy >= (unsigned)ey || (unsigned)cz >= (unsigned)ez) continue;
            const int c = cx + ex * (cy + ey * cz);
            const double mj = has_mass ? (double)gp(b.m[src])[si] : 1.0;
            double rl[3];
            am_local(b.a, qx, qy, qz, sh, rl);
            unsigned long long* const ra = acc + (size_t)c * kAmWords;
            if (pass == 1) {
                long long tm[kAmMoments];
                am_moments(mj, ux, uy, uz, rl, tm);
                for (int e = 0; e < kAmMoments; ++e) atomicAdd(&ra[e], (unsigned long long)tm[e]);
                atomicAdd(&ra[kAmMoments], 1ull);
            } else {
                const double* const rec = reinterpret_cast<const double*>(ra);
                long long tl3[3];
                if (!am_dl(mj, ux, uy, uz, rl, rec, rec + 3, rec + 6, b.ca, b.sa, tl3)) d[5] += 1;
                for (int e = 0; e < 3; ++e) atomicAdd(&ra[15 + e], (unsigned long long)tl3[e]);
            }
        }
    };
    if (flagged) {   // overflow particles of this step whose cells lie here
        MPCD_G CellAcc* __restrict__ esc = gp(b.esc[k & 1]);
        for (int c = threadIdx.x; c < ncl; c += kT) {
            const int lx = c % ex, ly = (c / ex) % ey, lz = c / (ex * ey);
            const uint32_t gc = (uint32_t)(lox + lx) + L0 * (uint32_t)(loy + ly) + L01 * (uint32_t)(loz + lz);
            const CellAcc e = load_acc(esc + gc);
            if (e.w) {
                if (!(kAM && am)) {
                    unsigned long long* const r = acc + (size_t)c * kAccWords;
                    r[0] += e.sx;
                    r[1] += e.sy;
                    r[2] += e.sz;
                    r[3] += kMass ? e.w : (e.w >> 32);   // escape weights are 2^32 m
                    if (kMass && has_mass) {   // and their count
                        MPCD_G uint32_t* const ec = gp(b.ecnt[k & 1]) + gc;
                        *reinterpret_cast<uint32_t*>(&r[4]) += *ec;
                        *ec = 0u;
                    }
                }
                CellAcc z = {0ull, 0ull, 0ull, 0ull};
                store_acc(esc + gc, z);
            }
        }
        if (kAM && am) am_overflow(1);
        __syncthreads();
    }

    if (kAM && am) {
        // 2a. per cell: u, r_c, axis n, second moment Q (FP64, in place of
        // the moment sums; an empty cell keeps n = 0)
        for (int c = threadIdx.x; c < ncl; c += kT) {
            unsigned long long* const ra = acc + (size_t)c * kAmWords;
            const long long* const sm = reinterpret_cast<const long long*>(ra);
            if (sm[0] == 0) continue;
            if (ra[kAmMoments] >= kMaxCellCount) d[5] += 1;   // the cell's sums may have wrapped
            const int lx = c % ex, ly = (c / ex) % ey, lz = c / (ex * ey);
            const uint32_t gc = (uint32_t)(lox + lx) + L0 * (uint32_t)(loy + ly) + L01 * (uint32_t)(loz + lz);
            double uc[3], rc[3], Q[6], n[3];
            am_cell(b, k, gc, sm, uc, rc, Q, n);
            double* const rec = reinterpret_cast<double*>(ra);
            for (int e = 0; e < 3; ++e) {
                rec[e] = uc[e];
                rec[3 + e] = rc[e];
                rec[6 + e] = n[e];
            }
            for (int e = 0; e < 6; ++e) rec[9 + e] = Q[e];
        }
        __syncthreads();
        // 2b. angular-momentum change of each particle under the plain rotation
        for (int ch = nch - 1; ch >= 0; --ch) {
            if (nch > 1) load(ch);
#pragma unroll
            for (int u = 0; u < kS; ++u) {
                const uint32_t c = meta[u];
                if (c == kNone) continue;
                unsigned long long* const ra = acc + (size_t)c * kAmWords;
                const double* const rec = reinterpret_cast<const double*>(ra);
                double rl[3];
                long long tl3[3];
                am_local(b.a, px[u], py[u], pz[u], sh, rl);
                if (!am_dl((double)pm[u], vx[u], vy[u], vz[u], rl, rec, rec + 3, rec + 6, b.ca, b.sa, tl3)) d[5] += 1;
                for (int e = 0; e < 3; ++e) atomicAdd(&ra[15 + e], (unsigned long long)tl3[e]);
            }
        }
        if (flagged) am_overflow(2);
        __syncthreads();
        // 2c. per cell: omega (in place of Q); flagged bricks publish the
        // cell data for the overflow particles
        for (int c = threadIdx.x; c < ncl; c += kT) {
            unsigned long long* const ra = acc + (size_t)c * kAmWords;
            double* const rec = reinterpret_cast<double*>(ra);
            if (rec[6] == 0.0 && rec[7] == 0.0 && rec[8] == 0.0) continue;   // empty
            double om[3];
            am_omega(rec + 9, reinterpret_cast<const long long*>(ra + 15), om);
            for (int e = 0; e < 3; ++e) rec[9 + e] = om[e];
            if (flagged) {
                const int lx = c % ex, ly = (c / ex) % ey, lz = c / (ex * ey);
                const uint32_t gc = (uint32_t)(lox + lx) + L0 * (uint32_t)(loy + ly) + L01 * (uint32_t)(loz + lz);
                CellAm* const g = b.uam + gc;
                for (int e = 0; e < 3; ++e) {
                    g->u[e] = rec[e];
                    g->rc[e] = rec[3 + e];
                    g->n[e] = rec[6 + e];
                    g->om[e] = om[e];
                }
            }
        }
        __syncthreads();
    } else {
        // 2. cell velocity and axis
        for (int c = threadIdx.x; c < ncl; c += kT) {
            const unsigned long long* const r = acc + (size_t)c * kAccWords;
            const unsigned long long w = kMass ? r[3] : ((r[3] & 0xffffffffull) << 32);
            if (w == 0) continue;
            const uint32_t count = kMass ? (uint32_t)r[4] : (uint32_t)r[3];
            if (count >= kMaxCellCount) d[5] += 1;   // the cell's sums may have wrapped
            const int lx = c % ex, ly = (c / ex) % ey, lz = c / (ex * ey);
            const uint32_t gc = (uint32_t)(lox + lx) + L0 * (uint32_t)(loy + ly) + L01 * (uint32_t)(loz + lz);
            double uc[3];
            fixed_mean3(r[0], r[1], r[2], w, uc);
            const CellRot cr = cell_rotation(uc[0], uc[1], uc[2], cell_axis(b, k, gc), b.ca, b.sa);
            float4* const q = reinterpret_cast<float4*>(fu + (size_t)c * kUnWords);
            q[0] = make_float4(cr.m[0], cr.m[1], cr.m[2], cr.m[3]);
            q[1] = make_float4(cr.m[4], cr.m[5], cr.m[6], cr.m[7]);
            q[2] = make_float4(cr.m[8], cr.t[0], cr.t[1], cr.t[2]);
            if (flagged) store_rot(gp(b.un) + gc, cr);   // read by the overflow particles
        }
        __syncthreads();
    }

    // 3./4. rotate, route to the next step's buckets, store
    const float3 sh1 = grid_shift(b, k + 1);
    // Interior bricks (a full brick below and above this one, itself full,
    // along every axis): a particle that stays inside the box needs no
    // periodic fold, and the brick of its next cell c = floor((x' - s1)/a),
    // c in [-1, L], is c >> shift, a neighbour exactly when that is within
    // one of this brick's index (c = -1 and c = L, the images of cells L-1
    // and 0, then fall outside the three); everything else takes the exact
    // general form.
    const bool interior = bx >= 1 && ((bx + 2) << b.bshift[0]) <= b.L[0] && by >= 1 &&
                          ((by + 2) << b.bshift[1]) <= b.L[1] && bz >= 1 && ((bz + 2) << b.bshift[2]) <= b.L[2];
    MPCD_G float* const ox = ugp(b.p[dst][0]);
    MPCD_G float* const oy = ugp(b.p[dst][1]);
    MPCD_G float* const oz = ugp(b.p[dst][2]);
    MPCD_G float* const ovx = ugp(b.p[dst][3]);
    MPCD_G float* const ovy = ugp(b.p[dst][4]);
    MPCD_G float* const ovz = ugp(b.p[dst][5]);
    const bool has_id = kIds && b.pid[src] != nullptr;   // uniform
    MPCD_G int32_t* const oid = has_id ? ugp(b.pid[dst]) : nullptr;
    const MPCD_G int32_t* const iid = has_id ? ugp(b.pid[src]) + beg : nullptr;   // bucket-relative
    const bool has_m = kMass && b.m[src] != nullptr;
    const int lane = threadIdx.x & (kWave - 1);
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int ch = 0; ch < nch; ++ch) {
        if (ch > 0) load(ch);
        const int nu = used_slots(ch);
        if (threadIdx.x < 27) gcnt[threadIdx.x] = 0u;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kS; ++u) {
            if (u >= nu) {
                meta[u] = 28u << 24;
                continue;
            }
            const uint32_t i = (uint32_t)ch * kChunk + (uint32_t)(u * kT) + threadIdx.x;
            uint32_t r = 28u;   // no particle
            if (i < cnt) {
                const uint32_t c = meta[u];
                if (kAM && am && c != kNone) {
                    const double* const rec = reinterpret_cast<const double*>(acc + (size_t)c * kAmWords);
                    double rl[3];
                    am_local(b.a, px[u], py[u], pz[u], sh, rl);
                    const float3 v = am_velocity(vx[u], vy[u], vz[u], rl, rec, rec + 3, rec + 6, rec + 9, b.ca, b.sa);
                    vx[u] = v.x;
                    vy[u] = v.y;
                    vz[u] = v.z;
                } else if (c != kNone) {
                    const float4* const q = reinterpret_cast<const float4*>(fu + (size_t)c * kUnWords);
                    const float4 q0 = q[0], q1 = q[1], q2 = q[2];
                    CellRot cr;
                    cr.m[0] = q0.x; cr.m[1] = q0.y; cr.m[2] = q0.z; cr.m[3] = q0.w;
                    cr.m[4] = q1.x; cr.m[5] = q1.y; cr.m[6] = q1.z; cr.m[7] = q1.w;
                    cr.m[8] = q2.x; cr.t[0] = q2.y; cr.t[1] = q2.z; cr.t[2] = q2.w;
                    const float3 v = apply_rotation(cr, vx[u], vy[u], vz[u]);
                    vx[u] = v.x;
                    vy[u] = v.y;
                    vz[u] = v.z;
                }
                const float3 v = make_float3(vx[u], vy[u], vz[u]);
                diag_check(d, v);
                if (vacf) vacf_term(b, ldg(iid, i * 4u), v, d);
                // brick of the next collision cell (a non-finite position
                // lands far away and takes the clamped slow path below)
                const float qx = fmaf(v.x, dt, px[u]), qy = fmaf(v.y, dt, py[u]), qz = fmaf(v.z, dt, pz[u]);
                int rx, ry, rz;
                if (interior && qx >= 0.0f && qx < b.len[0] && qy >= 0.0f && qy < b.len[1] && qz >= 0.0f &&
                    qz < b.len[2]) {
                    rx = ((int)floorf((qx - sh1.x) * inv_a) >> b.bshift[0]) - bx;
                    ry = ((int)floorf((qy - sh1.y) * inv_a) >> b.bshift[1]) - by;
                    rz = ((int)floorf((qz - sh1.z) * inv_a) >> b.bshift[2]) - bz;
                } else {
                    const int dbx = brick_of(axis_cell_raw(fold(qx, b.len[0]), sh1.x, inv_a, b.L[0]), b.bshift[0]);
                    const int dby = brick_of(axis_cell_raw(fold(qy, b.len[1]), sh1.y, inv_a, b.L[1]), b.bshift[1]);
                    const int dbz = brick_of(axis_cell_raw(fold(qz, b.len[2]), sh1.z, inv_a, b.L[2]), b.bshift[2]);
                    rx = brick_rel(bx, dbx, nb0);
                    ry = brick_rel(by, dby, nb1);
                    rz = brick_rel(bz, dbz, nb2);
                }
                r = ((unsigned)(rx + 1) <= 2u && (unsigned)(ry + 1) <= 2u && (unsigned)(rz + 1) <= 2u)
                        ? (uint32_t)((rx + 1) + 3 * ((ry + 1) + 3 * (rz + 1)))
                        : 27u;
            }
            // particles that stay in the brick (most) take consecutive ranks
            // per wave, so their stores coalesce
            const unsigned long long mask = __ballot(r == 13u);
            uint32_t rank = 0u;
            if (mask) {
                const int leader = __ffsll((long long)mask) - 1;
                uint32_t wb = 0u;
                if (lane == leader) wb = atomicAdd(&gcnt[13], (uint32_t)__popcll(mask));
                wb = __builtin_amdgcn_readlane(wb, leader);
                rank = wb + (uint32_t)__popcll(mask & below);
            }
            if (r < 27u && r != 13u) rank = atomicAdd(&gcnt[r], 1u);
            meta[u] = (r << 24) | rank;
        }
        // identities (only needed for the store): load while the groups reserve
        int32_t id[kS];
#pragma unroll
        for (int u = 0; u < kS; ++u) {
            if (u >= nu || !has_id) break;
            const uint32_t i = (uint32_t)ch * kChunk + (uint32_t)(u * kT) + threadIdx.x;
            id[u] = ldg(iid, (i < cnt ? i : 0u) * 4u);
        }
        __syncthreads();
        if (threadIdx.x < 27) {
            const int q = threadIdx.x;
            const uint32_t n = gcnt[q];
            if (n) {
                const int dx = brick_nbr(bx, q % 3 - 1, nb0), dy = brick_nbr(by, (q / 3) % 3 - 1, nb1),
                          dz = brick_nbr(bz, q / 9 - 1, nb2);
                const uint32_t dest = (uint32_t)(dx + nb0 * (dy + nb1 * dz));
                gpos[q] = gatomic_add(gp(b.bsize[dst]) + dest, n);
                const uint32_t b0 = gp(b.bstart)[dest];
                gbeg[q] = b0;
                gcap[q] = gp(b.bstart)[dest + 1] - b0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kS; ++u) {
            if (u >= nu) break;
            const uint32_t r = meta[u] >> 24;
            if (r >= 28u) continue;
            const float3 v = make_float3(vx[u], vy[u], vz[u]);
            uint32_t j = 0u;
            bool placed = false;
            if (r < 27u) {
                const uint32_t p = gpos[r] + (meta[u] & 0xffffffu);
                if (p < gcap[r]) {
                    j = gbeg[r] + p;
                    placed = true;
                }
            }
            if (!placed) {   // far (or full) destination: slow path
                const int3 nc = next_cell(b, px[u], py[u], pz[u], v, sh1);
                const int3 db = brick_of_cell(b, nc);
                if (r == 27u) placed = place_single(b, dst, (uint32_t)(db.x + nb0 * (db.y + nb1 * db.z)), &j);
                if (!placed) placed = place_overflow(b, dst, k, nc, pm[u], v, &j);
            }
            if (!placed) {
                d[5] += 1;
                continue;
            }
            // byte offset of destination slot j (64-bit for buffers of 2^30 slots or more)
            typedef typename std::conditional<kWide, unsigned long long, uint32_t>::type Off;
            const Off o = (Off)j * 4u;
            stg(ox, o, px[u]);
            stg(oy, o, py[u]);
            stg(oz, o, pz[u]);
            stg(ovx, o, v.x);
            stg(ovy, o, v.y);
            stg(ovz, o, v.z);
            if (has_id) stg(oid, o, id[u]);
            if (has_m) stg(gp(b.m[dst]), o, pm[u]);
        }
        if (ch + 1 < nch) __syncthreads();
    }
    step_flush<kT>(d, vacf, dacc + (size_t)uniform(tl.box) * kAccLanes * 3, blockIdx.x);
    if (threadIdx.x == 0) gp(b.bsize[src])[brick] = 0u;   // after every wave read it (step_flush's barrier)
}

// Particles of the overflow bucket of the current buffer (one workgroup per
// box, after the brick step): the same step, with the cell data the flagged
// bricks published.  Adds their diagnostics to d.
__device__ void overflow_step(const BoxDev& b, const BoxState& s, long long (&d)[kNumDiag])
{
    const int src = s.parity, dst = s.parity ^ 1;
    const uint32_t nbk = (uint32_t)b.nbrick;
    const uint32_t ob = gp(b.bstart)[nbk];
    const uint32_t cnt = min(gp(b.bsize[src])[nbk], gp(b.bstart)[nbk + 1] - ob);
    if (cnt == 0) return;
    const float3 sh = grid_shift(b, s.k), sh1 = grid_shift(b, s.k + 1);
    const bool has_m = b.m[src] != nullptr;
    const bool vacf = vacf_due(b, s);
    for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) {
        const uint32_t si = ob + i;
        const float vx = gp(b.p[src][3])[si], vy = gp(b.p[src][4])[si], vz = gp(b.p[src][5])[si];
        const float x = fold(fmaf(vx, b.dt, gp(b.p[src][0])[si]), b.len[0]);
        const float y = fold(fmaf(vy, b.dt, gp(b.p[src][1])[si]), b.len[1]);
        const float z = fold(fmaf(vz, b.dt, gp(b.p[src][2])[si]), b.len[2]);
        const float m = has_m ? gp(b.m[src])[si] : 1.0f;
        const uint32_t c = collision_cell(b, x, y, z, sh);
        float3 v;
        if (b.conserve_l && b.uam) {   // angular-momentum rule: cell data published as CellAm
            const CellAm& g = b.uam[c];
            double rl[3];
            am_local(b.a, x, y, z, sh, rl);
            v = am_velocity(vx, vy, vz, rl, g.u, g.rc, g.n, g.om, b.ca, b.sa);
        } else {
            v = apply_rotation(load_rot(gp(b.un) + c), vx, vy, vz);
        }
        diag_check(d, v);
        const int3 nc = next_cell(b, x, y, z, v, sh1);
        const int3 db = brick_of_cell(b, nc);
        uint32_t j = 0u;
        bool placed = place_single(b, dst, (uint32_t)(db.x + b.nb[0] * (db.y + b.nb[1] * db.z)), &j);
        if (!placed) placed = place_overflow(b, dst, s.k, nc, m, v, &j);
        if (!placed) {
            d[5] += 1;
            continue;
        }
        const int32_t id = b.pid[src] ? gp(b.pid[src])[si] : 0;
        if (vacf) vacf_term(b, id, v, d);
        put_particle(b, dst, j, x, y, z, v, id, m, has_m);
    }
}

// Re-bucketing step, first kernel: mark the holes of the current buffer
// (slots past the fill of their bucket) with pid -1, so that the counting
// sort can walk every slot.  Also used by the host before reading a brick
// box's state (all = 1: whatever the rebucket flag).
__global__ __launch_bounds__(kBlock) void k_mark_holes(const Tile* __restrict__ tiles,
                                                        const BoxDev* __restrict__ boxes,
                                                        const BoxState* __restrict__ st, int all, int box)
{
    const Tile tl = box >= 0 ? box_tile(boxes, box) : tiles[blockIdx.x];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (b.binning != 1) return;
    if (!all && (box_idle(s) || !s.rebucket)) return;
    const uint32_t* __restrict__ bs = b.bstart;
    const uint32_t* __restrict__ sz = b.bsize[s.parity];
    const int nbk = b.nbrick;
    for (int64_t i = tl.begin + threadIdx.x; i < tl.end; i += kBlock) {
        const int lo = bucket_of_slot(bs, nbk, i);
        const uint32_t fill = min(sz[lo], bs[lo + 1] - bs[lo]);
        if ((uint32_t)(i - bs[lo]) >= fill) mark_hole(b, s.parity, i);
    }
}

// Re-bucketing step: escape sums left for this step belong to particles the
// sort is about to put into their buckets; drop them.
__global__ __launch_bounds__(kBlock) void k_rebucket_clear(const Tile* __restrict__ tiles,
                                                            const BoxDev* __restrict__ boxes,
                                                            const BoxState* __restrict__ st)
{
    const Tile tl = tiles[blockIdx.x];
    const BoxState s = st[tl.box];
    const BoxDev& b = boxes[tl.box];
    if (b.binning != 1 || box_idle(s) || !s.rebucket) return;
    const int brick = (int)tl.begin;
    uint32_t* flag = b.eflag + (size_t)(s.k & 1) * b.nbrick + brick;
    if (*flag != (uint32_t)(s.k + 1)) return;
    const int nb0 = b.nb[0], nb1 = b.nb[1];
    const int bx = brick % nb0, by = (brick / nb0) % nb1, bz = brick / (nb0 * nb1);
    const int lox = brick_lo(bx, b.bshift[0]), loy = brick_lo(by, b.bshift[1]), loz = brick_lo(bz, b.bshift[2]);
    const int ex = min(1 << b.bshift[0], b.L[0] - lox);
    const int ey = min(1 << b.bshift[1], b.L[1] - loy);
    const int ez = min(1 << b.bshift[2], b.L[2] - loz);
    const uint32_t L0 = (uint32_t)b.L[0], L01 = (uint32_t)b.L[0] * (uint32_t)b.L[1];
    for (int c = threadIdx.x; c < ex * ey * ez; c += kBlock) {
        const int lx = c % ex, ly = (c / ex) % ey, lz = c / (ex * ey);
        const uint32_t gc = (uint32_t)(lox + lx) + L0 * (uint32_t)(loy + ly) + L01 * (uint32_t)(loz + lz);
        CellAcc z = {0ull, 0ull, 0ull, 0ull};
        store_acc(gp(b.esc[s.k & 1]) + gc, z);
        if (b.ecnt[0]) b.ecnt[s.k & 1][gc] = 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) *flag = 0u;
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

// Rank of every live slot among the slots with the same key (SORT: its
// collision cell, numbered in the blocked order of sort_key; re-bucketing:
// the brick of that cell), and the per-key
// counts in cstart.  The tile is taken in quarters of kCountPart slots; each
// quarter gathers its keys in an LDS hash table (open addressing, load factor
// at most 1/2), so a key takes one global atomic per quarter-tile, and the
// atomics of all distinct keys are issued together rather than one after
// another.  (Halves with a 32 KB table ran 29 % slower: fewer workgroups per
// CU.)
constexpr int kCountPart = kPartTile / 4;
constexpr int kCountPer = kCountPart / kBlock;    // slots per thread per quarter
constexpr int kHashSlots = 2 * kCountPart;
constexpr int kOwnSlots = kHashSlots / kBlock;   // hash slots each thread owns
constexpr uint32_t kHashEmpty = 0xffffffffu;

__device__ __forceinline__ uint32_t hash_slot(uint32_t key)
{
    return (key * 0x9E3779B1u) >> (32 - 11);   // Fibonacci hashing onto kHashSlots = 2048
}
static_assert(kHashSlots == 2048, "hash_slot maps onto 2048 slots");

__global__ __launch_bounds__(kBlock) void k_count(const Tile* __restrict__ tiles,
                                                   const BoxDev* __restrict__ boxes,
                                                   const BoxState* __restrict__ st)
{
    __shared__ uint32_t hkey[kHashSlots];
    __shared__ uint32_t hval[kHashSlots];   // count of the key in this quarter, then its global base
    __shared__ uint16_t slots[kHashSlots];  // per wave: the occupied slots its lanes own
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const BoxState s = st[uniform(tl.box)];
    const BoxDev& b = boxes[uniform(tl.box)];
    if (box_idle(s) || !sort_due(b, s)) return;
    const int par = uniform(s.parity);
    const MPCD_G float* __restrict__ x = gp(b.p[par][0]);
    const MPCD_G float* __restrict__ y = gp(b.p[par][1]);
    const MPCD_G float* __restrict__ z = gp(b.p[par][2]);
    const MPCD_G float* __restrict__ vx = gp(b.p[par][3]);
    const MPCD_G float* __restrict__ vy = gp(b.p[par][4]);
    const MPCD_G float* __restrict__ vz = gp(b.p[par][5]);
    const MPCD_G int32_t* __restrict__ pid = b.pid[par] ? gp(b.pid[par]) : nullptr;
    MPCD_G uint32_t* __restrict__ cell = gp(b.cell);
    MPCD_G uint32_t* __restrict__ rank = gp(b.rank);
    MPCD_G uint32_t* __restrict__ counts = gp(b.cstart);
    const bool by_brick = (b.binning == 1);
    const float3 sh = grid_shift(b, uniform(s.k));
    const float dt = b.dt;
    for (int64_t h0 = tl.begin; h0 < tl.end; h0 += kCountPart) {
        for (int q = threadIdx.x; q < kHashSlots; q += kBlock) {
            hkey[q] = kHashEmpty;
            hval[q] = 0u;
        }
        __syncthreads();
        uint32_t slot_rank[kCountPer];   // hash slot << 16 | rank inside the quarter; kHashEmpty: none
        float qx[kCountPer], qy[kCountPer], qz[kCountPer], ux[kCountPer], uy[kCountPer], uz[kCountPer];
        bool live[kCountPer];
#pragma unroll
        for (int u = 0; u < kCountPer; ++u) {   // issue every load first
            const int64_t i = h0 + (int64_t)u * kBlock + threadIdx.x;
            const int64_t j = i < tl.end ? i : tl.begin;
            qx[u] = x[j];
            qy[u] = y[j];
            qz[u] = z[j];
            ux[u] = vx[j];
            uy[u] = vy[j];
            uz[u] = vz[j];
            live[u] = i < tl.end && (pid ? pid[j] >= 0 : !(qx[u] < 0.0f));
        }
#pragma unroll
        for (int u = 0; u < kCountPer; ++u) {
            slot_rank[u] = kHashEmpty;
            if (!live[u]) continue;   // hole (or past the tile)
            const int64_t i = h0 + (int64_t)u * kBlock + threadIdx.x;
            const float px = fold(fmaf(ux[u], dt, qx[u]), b.len[0]);
            const float py = fold(fmaf(uy[u], dt, qy[u]), b.len[1]);
            const float pz = fold(fmaf(uz[u], dt, qz[u]), b.len[2]);
            uint32_t key;
            if (by_brick) {   // the brick holding the collision cell of this step
                const int3 c = make_int3(axis_cell(px, sh.x, b.inv_a, b.L[0]), axis_cell(py, sh.y, b.inv_a, b.L[1]),
                                         axis_cell(pz, sh.z, b.inv_a, b.L[2]));
                const int3 d = brick_of_cell(b, c);
                key = (uint32_t)(d.x + b.nb[0] * (d.y + b.nb[1] * d.z));
            } else {   // the position of its collision cell in the sort's cell order
                key = sort_cell(b, px, py, pz, sh);
            }
            cell[i] = key;
            uint32_t hs = hash_slot(key);
            while (true) {   // at most kCountPart keys in kHashSlots slots: a free slot exists
                const uint32_t old = atomicCAS(&hkey[hs], kHashEmpty, key);
                if (old == kHashEmpty || old == key) break;
                hs = (hs + 1u) & (kHashSlots - 1);
            }
            slot_rank[u] = (hs << 16) | atomicAdd(&hval[hs], 1u);
        }
        __syncthreads();
        // one global atomic per distinct key of the quarter: its base among all
        // tiles.  Each wave first lists the occupied slots among those its
        // lanes own (ballot and popcount), so its atomics go out together,
        // one per lane, rather than one round trip per owned slot.
        {
            const int lane = threadIdx.x & (kWave - 1);
            const unsigned long long below = (1ull << lane) - 1ull;
            uint16_t* const wl = slots + (threadIdx.x / kWave) * (kWave * kOwnSlots);
            uint32_t nl = 0u;   // wave-uniform
#pragma unroll
            for (int t = 0; t < kOwnSlots; ++t) {
                const int q = t * kBlock + threadIdx.x;
                const bool occ = hkey[q] != kHashEmpty;
                const unsigned long long m = __ballot(occ);
                if (occ) wl[nl + (uint32_t)__popcll(m & below)] = (uint16_t)q;
                nl += (uint32_t)__popcll(m);
            }
            __builtin_amdgcn_wave_barrier();
            for (uint32_t e = (uint32_t)lane; e < nl; e += kWave) {
                const int q = wl[e];
                hval[q] = gatomic_add(counts + hkey[q], hval[q]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kCountPer; ++u) {
            if (slot_rank[u] == kHashEmpty) continue;
            const int64_t i = h0 + (int64_t)u * kBlock + threadIdx.x;
            rank[i] = hval[slot_rank[u] >> 16] + (slot_rank[u] & 0xffffu);
        }
        __syncthreads();   // the table is reset for the next quarter
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
    for (int64_t c = tl.begin + threadIdx.x; c < tl.end; c += kBlock) v += key_capacity(b, c, b.cstart[c]);
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

// per cell tile: exclusive scan of the key capacities into starts.  For
// brick boxes the keys are bricks, and the starts become the bucket layout of
// the buffer the scatter fills (counts plus slack; overflow bucket last).
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
    uint32_t cnt[kPer], cap[kPer];
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        cnt[j] = (c0 + j < tl.end) ? b.cstart[c0 + j] : 0u;
        cap[j] = (c0 + j < tl.end) ? key_capacity(b, c0 + j, cnt[j]) : 0u;
        v += cap[j];
    }
    uint32_t total;
    const uint32_t start = tilesum[t] + block_exclusive_scan(v, &total);
    const bool brick = (b.binning == 1);
    const int64_t nbk = b.nbrick;
    uint32_t run = start;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t c = c0 + j;
        if (c < tl.end) {
            b.cstart[c] = run;
            if (brick && c < nbk) {
                b.bstart[c] = run;
                b.bsize[s.parity ^ 1][c] = cnt[j];
                b.bsize[s.parity][c] = 0u;   // the next step's destination
                if (c == nbk - 1) {         // overflow bucket: the rest of the buffer
                    b.bstart[nbk] = run + cap[j];
                    b.bstart[nbk + 1] = (uint32_t)b.nslot;
                    b.bsize[s.parity ^ 1][nbk] = 0u;
                    b.bsize[s.parity][nbk] = 0u;
                }
            }
        }
        run += cap[j];
    }
    if (tl.end == b.ncell && threadIdx.x == 0) b.cstart[b.ncell] = brick ? tilesum[t] + total : (uint32_t)b.n;
}

__global__ __launch_bounds__(kBlock) void k_scatter(const Tile* __restrict__ tiles,
                                                     const BoxDev* __restrict__ boxes,
                                                     const BoxState* __restrict__ st)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const BoxState s = st[uniform(tl.box)];
    const BoxDev& b = boxes[uniform(tl.box)];
    if (box_idle(s) || !sort_due(b, s)) return;
    const int src = uniform(s.parity), dst = src ^ 1;
    const bool stream = (b.binning == 2);
    const bool has_m = b.m[src] != nullptr;
    const float dt = b.dt;
    const MPCD_G float* __restrict__ ix = ugp(b.p[src][0]);
    const MPCD_G float* __restrict__ iy = ugp(b.p[src][1]);
    const MPCD_G float* __restrict__ iz = ugp(b.p[src][2]);
    const MPCD_G float* __restrict__ ivx = ugp(b.p[src][3]);
    const MPCD_G float* __restrict__ ivy = ugp(b.p[src][4]);
    const MPCD_G float* __restrict__ ivz = ugp(b.p[src][5]);
    const MPCD_G int32_t* __restrict__ iid = b.pid[src] ? gp(b.pid[src]) : nullptr;
    MPCD_G float* __restrict__ ox = gp(b.p[dst][0]);
    MPCD_G float* __restrict__ oy = gp(b.p[dst][1]);
    MPCD_G float* __restrict__ oz = gp(b.p[dst][2]);
    MPCD_G float* __restrict__ ovx = gp(b.p[dst][3]);
    MPCD_G float* __restrict__ ovy = gp(b.p[dst][4]);
    MPCD_G float* __restrict__ ovz = gp(b.p[dst][5]);
    MPCD_G int32_t* __restrict__ oid = b.pid[dst] ? gp(b.pid[dst]) : nullptr;
    const MPCD_G uint32_t* __restrict__ cell = gp(b.cell);
    const MPCD_G uint32_t* __restrict__ rank = gp(b.rank);
    const MPCD_G uint32_t* __restrict__ cstart = gp(b.cstart);
    if (b.perm) {
        // SORT binning with the plain rule: only the permutation moves here.
        // k_cell_rotate gathers each run of cells through it and writes the
        // particles to the next buffer with coalesced stores; scattering
        // 4-byte indices instead of 24-byte particles cuts the partial-line
        // writes, which neighbouring tiles fill at different times.  A SORT
        // box has no holes (nslot = n).
        MPCD_G uint32_t* __restrict__ perm = gp(b.perm);
        constexpr int kP = 16;
        for (int64_t i0 = tl.begin + threadIdx.x; i0 < tl.end; i0 += (int64_t)kBlock * kP) {
            uint32_t key[kP], rk[kP];
#pragma unroll
            for (int u = 0; u < kP; ++u) {
                const int64_t i = i0 + (int64_t)u * kBlock;
                const int64_t j = i < tl.end ? i : tl.begin;
                key[u] = cell[j];
                rk[u] = rank[j];
            }
#pragma unroll
            for (int u = 0; u < kP; ++u) {
                const int64_t i = i0 + (int64_t)u * kBlock;
                if (i < tl.end) perm[cstart[key[u]] + rk[u]] = (uint32_t)i;
            }
        }
        return;
    }
    constexpr int kU = 8;   // particles per thread in flight (the destination gathers wait on cstart)
    for (int64_t i0 = tl.begin + threadIdx.x; i0 < tl.end; i0 += (int64_t)kBlock * kU) {
        float qx[kU], qy[kU], qz[kU], ux[kU], uy[kU], uz[kU];
        int32_t id[kU];
        uint32_t key[kU], rk[kU];
        bool live[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {   // issue every load first
            const int64_t i = i0 + (int64_t)u * kBlock;
            const int64_t j = i < tl.end ? i : tl.begin;
            key[u] = cell[j];
            rk[u] = rank[j];
            qx[u] = ix[j];
            qy[u] = iy[j];
            qz[u] = iz[j];
            ux[u] = ivx[j];
            uy[u] = ivy[j];
            uz[u] = ivz[j];
            id[u] = iid ? iid[j] : 0;
            // the same predicate as k_count: a hole (or past the tile) is skipped
            live[u] = i < tl.end && (iid ? id[u] >= 0 : !(qx[u] < 0.0f));
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (!live[u]) continue;
            const int64_t i = i0 + (int64_t)u * kBlock;
            const int64_t j = (int64_t)cstart[key[u]] + rk[u];
            float px = qx[u], py = qy[u], pz = qz[u];
            if (stream) {
                px = fold(fmaf(ux[u], dt, px), b.len[0]);
                py = fold(fmaf(uy[u], dt, py), b.len[1]);
                pz = fold(fmaf(uz[u], dt, pz), b.len[2]);
            }
            ox[j] = px;
            oy[j] = py;
            oz[j] = pz;
            ovx[j] = ux[u];
            ovy[j] = uy[u];
            ovz[j] = uz[u];
            if (oid) oid[j] = id[u];
            if (has_m) gp(b.m[dst])[j] = gp(b.m[src])[i];
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
    if (due && boxes[bx].binning == 1) s.rebuckets += 1;
    s.rebucket = 0;
}

// Angular-momentum-conserving collision of one cell whose particles occupy
// [beg, end) of the current buffer (streamed, SORT binning): three passes of
// one thread over the cell (moments, angular-momentum change, new
// velocities) with the shared am_* functions.
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
    long long sm[kAmMoments] = {};
    if (end - beg >= kMaxCellCount) d[5] += 1;   // the cell's sums may have wrapped
    for (uint32_t j = beg; j < end; ++j) {
        double r[3];
        long long t[kAmMoments];
        am_local(a, px[j], py[j], pz[j], sh, r);
        am_moments(mass_of(mp, j), vx[j], vy[j], vz[j], r, t);
#pragma unroll
        for (int q = 0; q < kAmMoments; ++q) sm[q] += t[q];
    }
    double u[3], rc[3], Q[6], n[3], om[3];
    am_cell(b, k, c, sm, u, rc, Q, n);
    long long sl[3] = {0, 0, 0};
    for (uint32_t j = beg; j < end; ++j) {
        double r[3];
        long long t[3];
        am_local(a, px[j], py[j], pz[j], sh, r);
        if (!am_dl(mass_of(mp, j), vx[j], vy[j], vz[j], r, u, rc, n, ca, sa, t)) d[5] += 1;
        sl[0] += t[0];
        sl[1] += t[1];
        sl[2] += t[2];
    }
    am_omega(Q, sl, om);
    for (uint32_t j = beg; j < end; ++j) {
        double r[3];
        am_local(a, px[j], py[j], pz[j], sh, r);
        const float3 v = am_velocity(vx[j], vy[j], vz[j], r, u, rc, n, om, ca, sa);
        if (vacf) vacf_term(b, b.pid[par][j], v, d);
        vx[j] = v.x;
        vy[j] = v.y;
        vz[j] = v.z;
        diag_check(d, v);
    }
}

// Plain collision of one cell whose particles occupy [beg, end) of the
// current buffer, by one thread straight from global memory (SORT path, a
// cell too large for the staging area of k_cell_rotate).
__device__ void collide_cell_serial(const BoxDev& b, int par, long long k, uint32_t c, uint32_t beg, uint32_t end,
                                    long long (&d)[kNumDiag], bool vacf)
{
    float* __restrict__ vx = b.p[par][3];
    float* __restrict__ vy = b.p[par][4];
    float* __restrict__ vz = b.p[par][5];
    const float* __restrict__ mp = b.m[par];
    if (end - beg >= kMaxCellCount) d[5] += 1;   // the cell's sums may have wrapped
    unsigned long long sx = 0, sy = 0, sz = 0, sw = 0;
    for (uint32_t j = beg; j < end; ++j) {
        const float mj = mass_of(mp, j);
        sx += to_fixed(mj * vx[j]);
        sy += to_fixed(mj * vy[j]);
        sz += to_fixed(mj * vz[j]);
        sw += to_fixed(mj);
    }
    double uc[3];
    fixed_mean3(sx, sy, sz, sw, uc);
    const CellRot cr = cell_rotation(uc[0], uc[1], uc[2], cell_axis(b, k, c), b.ca, b.sa);
    for (uint32_t j = beg; j < end; ++j) {
        const float3 v = apply_rotation(cr, vx[j], vy[j], vz[j]);
        vx[j] = v.x;
        vy[j] = v.y;
        vz[j] = v.z;
        diag_check(d, v);
        if (vacf) vacf_term(b, b.pid[par][j], v, d);
    }
}

// SORT path: the particles of the cell with sort key c (sort_key) go to
// slots [cstart[c], cstart[c+1]) of the new buffer; perm names the slot of
// the old buffer each one comes from.  A workgroup takes its cell tile in
// runs of at most kRotCells cells holding at most kRotCap particles: it
// gathers the run's particles through perm, writes their streamed positions
// (and ids, masses) to the new buffer with coalesced stores and stages the
// velocities (and masses) in LDS; one thread per cell sums its particles from
// LDS (exact fixed point, the same terms as the brick step) and builds the
// cell's collision map, then every thread applies the maps to its particles
// and stores them coalesced.  The next run's gathers are in flight while a
// run is collided.  A cell larger than the staging area is moved into place
// and walked by one thread in global memory.  Under the angular-momentum rule
// k_scatter has already moved the particles, and one thread walks each cell
// (three passes).
constexpr int kRotCap = 1024;
constexpr int kRotCells = 128;

// held to 4 waves per SIMD: 128 VGPRs, no spills (unbounded it takes 147 and
// runs 6 % slower at 3 waves)
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_cell_rotate(const Tile* __restrict__ tiles, const BoxDev* __restrict__ boxes, const BoxState* __restrict__ st,
                   long long* __restrict__ dacc)
{
    __shared__ uint32_t cs[kCellTile + 1];     // cstart of the tile's cells
    __shared__ float sv[3][kRotCap];
    __shared__ float sm[kRotCap];
    __shared__ uint8_t seg[kRotCap];           // run-local cell of each staged particle
    __shared__ f32x4 rot[kRotCells][3];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const Tile tl = tiles[t];
    const BoxState s = st[uniform(tl.box)];
    const BoxDev& b = boxes[uniform(tl.box)];
    if (box_idle(s) || b.binning != 2) return;
    const int par = uniform(s.parity);
    const long long k = uniform(s.k);
    const bool vacf = vacf_due(b, s);
    long long d[kNumDiag] = {};
    if (b.conserve_l) {
        const float3 sh = grid_shift(b, k);
        for (int64_t c = tl.begin + threadIdx.x; c < tl.end; c += kBlock) {
            const uint32_t beg = b.cstart[c], end = b.cstart[c + 1];
            if (beg != end)
                collide_cell_am(b, par, k, cell_of_key(b.L, b.sshift, (uint32_t)c), beg, end, sh, b.ca, b.sa, d, vacf);
        }
        step_flush(d, vacf, dacc + (size_t)tl.box * kAccLanes * 3, blockIdx.x);
        return;
    }
    // the particles of the next buffer's slots come from the current buffer
    // through the counting sort's permutation
    const int src = par ^ 1;
    const MPCD_G uint32_t* const perm = ugp(b.perm);
    const MPCD_G float* const ix = ugp(b.p[src][0]);
    const MPCD_G float* const iy = ugp(b.p[src][1]);
    const MPCD_G float* const iz = ugp(b.p[src][2]);
    const MPCD_G float* const ivx = ugp(b.p[src][3]);
    const MPCD_G float* const ivy = ugp(b.p[src][4]);
    const MPCD_G float* const ivz = ugp(b.p[src][5]);
    const MPCD_G float* const im = b.m[src] ? ugp(b.m[src]) : nullptr;
    const MPCD_G int32_t* const iid = b.pid[src] ? ugp(b.pid[src]) : nullptr;
    MPCD_G float* const ox = ugp(b.p[par][0]);
    MPCD_G float* const oy = ugp(b.p[par][1]);
    MPCD_G float* const oz = ugp(b.p[par][2]);
    MPCD_G float* const vx = ugp(b.p[par][3]);
    MPCD_G float* const vy = ugp(b.p[par][4]);
    MPCD_G float* const vz = ugp(b.p[par][5]);
    MPCD_G float* const om = b.m[par] ? ugp(b.m[par]) : nullptr;
    MPCD_G int32_t* const pid = b.pid[par] ? ugp(b.pid[par]) : nullptr;
    const float dt = b.dt;
    const uint32_t last = (uint32_t)(b.n - 1);   // a slot index beyond it would be a broken permutation
    const int nc = (int)(tl.end - tl.begin);
    for (int i = threadIdx.x; i <= nc; i += kBlock) cs[i] = gp(b.cstart)[tl.begin + i];
    __syncthreads();
    // the run [c0, e): as many cells as fit (uniform binary search on cs)
    auto run_end = [&](int c0) -> int {
        int e1 = c0 + 1;
        const uint32_t b0 = cs[c0];
        if (cs[e1] - b0 <= (uint32_t)kRotCap) {
            int lo = e1, hi = min(nc, c0 + kRotCells);
            while (lo < hi) {
                const int m = (lo + hi + 1) >> 1;
                if (cs[m] - b0 <= (uint32_t)kRotCap) lo = m;
                else hi = m - 1;
            }
            e1 = lo;
        }
        return e1;
    };
    constexpr int kPer = kRotCap / kBlock;
    float gx[kPer], gy[kPer], gz[kPer], qx[kPer], qy[kPer], qz[kPer], qm[kPer];
    int32_t qi[kPer];
    uint32_t si[kPer];
    // A run's loads go in two stages, one run apart: its source slots (perm),
    // then, a run later, its particles through them; so a run's gathers never
    // wait on its own perm loads.
    auto load_perm = [&](uint32_t b0, uint32_t n0) {
#pragma unroll
        for (int m = 0; m < kPer; ++m) {
            const uint32_t j = (uint32_t)(m * kBlock) + threadIdx.x;
            si[m] = j < n0 ? perm[b0 + j] : 0u;
        }
    };
    auto gather = [&](uint32_t n0) {
#pragma unroll
        for (int m = 0; m < kPer; ++m) {
            const uint32_t j = (uint32_t)(m * kBlock) + threadIdx.x;
            if (j < n0) {
                const uint32_t i = min(si[m], last);
                gx[m] = ix[i];
                gy[m] = iy[i];
                gz[m] = iz[i];
                qx[m] = ivx[i];
                qy[m] = ivy[i];
                qz[m] = ivz[i];
                qm[m] = im ? im[i] : 1.0f;
                qi[m] = iid ? iid[i] : 0;
            }
        }
    };
    struct Run {
        int c, e;            // cells [c, e) of the tile
        uint32_t base, np;   // their slots [base, base + np)
    };
    auto run_at = [&](int c0) -> Run {
        if (c0 >= nc) return Run{c0, c0, 0u, 0u};
        const int e0 = run_end(c0);
        return Run{c0, e0, cs[c0], cs[e0] - cs[c0]};
    };
    auto fits = [&](const Run& r) { return r.c < nc && r.np <= (uint32_t)kRotCap; };
    // r: the run being collided (gathers in flight), r2: the next (perm in flight)
    Run r = run_at(0), r2 = run_at(r.e);
    if (fits(r)) {
        load_perm(r.base, r.np);
        gather(r.np);
    }
    if (fits(r2)) load_perm(r2.base, r2.np);
    while (r.c < nc) {
        const int c = r.c, e = r.e;
        const uint32_t base = r.base, np = r.np;
        if (np > (uint32_t)kRotCap) {   // one cell larger than the staging area
            // moved into place (streamed), then walked by one thread
            for (uint32_t j = threadIdx.x; j < np; j += kBlock) {
                const uint32_t i = min(perm[base + j], last);
                const float ux = ivx[i], uy = ivy[i], uz = ivz[i];
                ox[base + j] = fold(fmaf(ux, dt, ix[i]), b.len[0]);
                oy[base + j] = fold(fmaf(uy, dt, iy[i]), b.len[1]);
                oz[base + j] = fold(fmaf(uz, dt, iz[i]), b.len[2]);
                vx[base + j] = ux;
                vy[base + j] = uy;
                vz[base + j] = uz;
                if (pid) pid[base + j] = iid[i];
                if (om) om[base + j] = im[i];
            }
            __syncthreads();
            if (threadIdx.x == 0)
                collide_cell_serial(b, par, k, cell_of_key(b.L, b.sshift, (uint32_t)(tl.begin + c)), base, cs[e], d,
                                    vacf);
            r = r2;
            r2 = run_at(r.e);
            if (fits(r)) gather(r.np);
            if (fits(r2)) load_perm(r2.base, r2.np);
            continue;
        }
        // positions streamed (the arithmetic k_count chose the cell with),
        // ids and masses go straight to the next buffer; velocities to LDS
#pragma unroll
        for (int m = 0; m < kPer; ++m) {
            const uint32_t j = (uint32_t)(m * kBlock) + threadIdx.x;
            if (j < np) {
                ox[base + j] = fold(fmaf(qx[m], dt, gx[m]), b.len[0]);
                oy[base + j] = fold(fmaf(qy[m], dt, gy[m]), b.len[1]);
                oz[base + j] = fold(fmaf(qz[m], dt, gz[m]), b.len[2]);
                if (pid) pid[base + j] = qi[m];
                if (om) om[base + j] = qm[m];
                sv[0][j] = qx[m];
                sv[1][j] = qy[m];
                sv[2][j] = qz[m];
                sm[j] = qm[m];
            }
        }
        __syncthreads();
        // the next run's gathers and the one after's perm loads are in flight
        // while this run is collided
        const Run r3 = run_at(r2.e);
        if (fits(r2)) gather(r2.np);
        if (fits(r3)) load_perm(r3.base, r3.np);
        if (threadIdx.x < e - c) {
            const int q = threadIdx.x;
            const uint32_t rb = cs[c + q] - base, re = cs[c + q + 1] - base;
            if (rb != re) {
                if (re - rb >= kMaxCellCount) d[5] += 1;   // the cell's sums may have wrapped
                unsigned long long sx = 0, sy = 0, sz = 0, sw = 0;
                for (uint32_t j = rb; j < re; ++j) {
                    const float mj = sm[j];
                    sx += to_fixed(mj * sv[0][j]);
                    sy += to_fixed(mj * sv[1][j]);
                    sz += to_fixed(mj * sv[2][j]);
                    sw += to_fixed(mj);
                    seg[j] = (uint8_t)q;
                }
                double uc[3];
                fixed_mean3(sx, sy, sz, sw, uc);
                const uint32_t cell = cell_of_key(b.L, b.sshift, (uint32_t)(tl.begin + c + q));
                const CellRot cr = cell_rotation(uc[0], uc[1], uc[2], cell_axis(b, k, cell), b.ca, b.sa);
                f32x4 r0, r1, r2;
                r0.x = cr.m[0]; r0.y = cr.m[1]; r0.z = cr.m[2]; r0.w = cr.m[3];
                r1.x = cr.m[4]; r1.y = cr.m[5]; r1.z = cr.m[6]; r1.w = cr.m[7];
                r2.x = cr.m[8]; r2.y = cr.t[0]; r2.z = cr.t[1]; r2.w = cr.t[2];
                rot[q][0] = r0;
                rot[q][1] = r1;
                rot[q][2] = r2;
            }
        }
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < np; j += kBlock) {
            const int q = seg[j];
            const f32x4 r0 = rot[q][0], r1 = rot[q][1], r2 = rot[q][2];
            CellRot cr;
            cr.m[0] = r0.x; cr.m[1] = r0.y; cr.m[2] = r0.z; cr.m[3] = r0.w;
            cr.m[4] = r1.x; cr.m[5] = r1.y; cr.m[6] = r1.z; cr.m[7] = r1.w;
            cr.m[8] = r2.x; cr.t[0] = r2.y; cr.t[1] = r2.z; cr.t[2] = r2.w;
            const float3 v = apply_rotation(cr, sv[0][j], sv[1][j], sv[2][j]);
            vx[base + j] = v.x;
            vy[base + j] = v.y;
            vz[base + j] = v.z;
            diag_check(d, v);
            if (vacf) vacf_term(b, pid[base + j], v, d);
        }
        __syncthreads();   // the staging area is refilled by the next run
        r = r2;
        r2 = r3;
    }
    step_flush(d, vacf, dacc + (size_t)tl.box * kAccLanes * 3, blockIdx.x);
}

// --------------------------------------------------------------------------
// end of step: per box, the overflow bucket (brick boxes), the VACF sample
// and range check from the step's accumulators, k++

__global__ __launch_bounds__(kBlock) void k_box_finish(const int32_t* __restrict__ active,
                                                        const BoxDev* __restrict__ boxes,
                                                        BoxState* __restrict__ st,
                                                        long long* __restrict__ dacc,
                                                        int* __restrict__ host_flag)
{
    const int bx = active[blockIdx.x];
    BoxState* sp = &st[bx];
    if (box_idle(*sp)) return;
    const BoxDev& b = boxes[bx];
    const bool by_cell = (b.binning == 2);
    long long d[kNumDiag] = {};
    if (!by_cell) overflow_step(b, *sp, d);
    // this thread's share of the exact sums: its particles plus, for the
    // first kAccLanes threads, one accumulator lane (then cleared)
    long long hi = d[4] >> 32, lo = (long long)(unsigned long long)(unsigned)(d[4] & 0xffffffffll), viol = d[5];
    long long* a = dacc + (size_t)bx * kAccLanes * 3;
    if (threadIdx.x < kAccLanes) {
        long long* l = a + (size_t)threadIdx.x * 3;
        hi += l[0];
        lo += l[1];
        viol += l[2];
        l[0] = 0;
        l[1] = 0;
        l[2] = 0;
    }
    __shared__ long long red[3][kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    hi = wave_sum(hi);
    lo = wave_sum(lo);
    viol = wave_sum(viol);
    if (lane == 0) {
        red[0][w] = hi;
        red[1][w] = lo;
        red[2][w] = viol;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long th = 0, tl = 0, tv = 0;
        for (int i = 0; i < kBlock / kWave; ++i) {
            th += red[0][i];
            tl += red[1][i];
            tv += red[2][i];
        }
        const double vsum = (double)th + (double)tl * 2.3283064365386963e-10;   // (hi 2^32 + lo) 2^-32
        const bool vac = vacf_due(b, *sp);
        if (tv != 0) sp->status = -5;   // velocity out of range / not finite
        if (vac && sp->vacf_len < b.vacf_cap && b.n > 0)
            b.vacf[sp->vacf_len++] = vsum / (double)b.n;
        if (!by_cell) {
            const int src = sp->parity, nbk = b.nbrick;
            gp(b.bsize[src])[nbk] = 0u;   // overflow bucket drained
            // particles left in the overflow bucket: ask the host for a
            // re-bucketing (new capacities) at its next step call
            if (gp(b.bsize[src ^ 1])[nbk] != 0u) {
                sp->overflow_steps += 1;
                sp->rebucket = 1;
                if (host_flag) __hip_atomic_store(host_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            sp->parity ^= 1;   // the brick step wrote the other buffer
        }
        sp->k += 1;
        if (sp->remaining > 0) sp->remaining -= 1;
    }
}

// --------------------------------------------------------------------------
// initial state on the device (not part of the step)

__global__ __launch_bounds__(kBlock) void k_init_maxwell(const BoxDev* __restrict__ boxes,
                                                          const BoxState* __restrict__ st, int box,
                                                          float vscale, long long* __restrict__ partials)
{
    const int t = blockIdx.x;
    const Tile tl = box_tile(boxes, box);
    const BoxDev& b = boxes[tl.box];
    const int par = st[tl.box].parity;
    long long d[kNumDiag] = {};
    for (int64_t i = tl.begin + threadIdx.x; i < tl.end; i += kBlock) {
        if (i >= b.n) {   // spare slot of a brick box
            mark_hole(b, par, i);
            continue;
        }
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
        if (b.pid[par]) b.pid[par][i] = (int32_t)i;
        diag_particle(d, make_float3(vx, vy, vz), 1.0f);
    }
    block_diag(d, partials + (size_t)t * kNumDiag);
}

// v <- (v - V) * scale with (V, scale) = the box state's adj[]; partial
// sums of the adjusted velocities
__global__ __launch_bounds__(kBlock) void k_init_adjust(const BoxDev* __restrict__ boxes,
                                                         const BoxState* __restrict__ st, int box,
                                                         long long* __restrict__ partials)
{
    const int t = blockIdx.x;
    const Tile tl = box_tile(boxes, box);
    const BoxDev& b = boxes[tl.box];
    const int par = st[tl.box].parity;
    const float mx = st[tl.box].adj[0], my = st[tl.box].adj[1], mz = st[tl.box].adj[2];
    const float scale = st[tl.box].adj[3];
    long long d[kNumDiag] = {};
    for (int64_t i = tl.begin + threadIdx.x; i < tl.end; i += kBlock) {
        if (!slot_live(b, par, i)) continue;
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
__global__ __launch_bounds__(kBlock) void k_snapshot(const BoxDev* __restrict__ boxes,
                                                      const BoxState* __restrict__ st, int box,
                                                      int set_v0, long long* __restrict__ partials)
{
    const int t = blockIdx.x;
    const Tile tl = box_tile(boxes, box);
    const BoxDev& b = boxes[tl.box];
    const int par = st[tl.box].parity;
    const bool has_v0 = b.vacf_stride > 0;
    long long d[kNumDiag] = {};
    for (int64_t i = tl.begin + threadIdx.x; i < tl.end; i += kBlock) {
        if (!slot_live(b, par, i)) continue;
        const float vx = b.p[par][3][i], vy = b.p[par][4][i], vz = b.p[par][5][i];
        const int32_t id = b.pid[par] ? b.pid[par][i] : 0;
        if (has_v0 && set_v0) b.v0[id] = make_float4(vx, vy, vz, 0.0f);
        diag_particle(d, make_float3(vx, vy, vz), mass_of(b.m[par], i));
        if (has_v0) vacf_term(b, id, make_float3(vx, vy, vz), d);
    }
    block_diag(d, partials + (size_t)t * kNumDiag);
}

// Block sum of one int128 per thread and component; thread 0 gets the totals.
__device__ __forceinline__ void block_sum128(__int128 (&acc)[kNumDiag], __int128 (&tot)[kNumDiag])
{
    __shared__ __int128 red[kBlock][kNumDiag];
#pragma unroll
    for (int j = 0; j < kNumDiag; ++j) red[threadIdx.x][j] = acc[j];
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int j = 0; j < kNumDiag; ++j) {
        __int128 v = 0;
        for (int i = 0; i < kBlock; ++i) v += red[i][j];
        tot[j] = v;
    }
}

// What the exact box sums are used for (thread 0; see k_box_stats).
__device__ void box_stats_finish(const __int128 (&tot)[kNumDiag], const BoxDev* __restrict__ box,
                                 BoxState* __restrict__ st, int mode, double kT, double mass)
{
#pragma clang fp contract(off)
    double d[kNumDiag];
    for (int j = 0; j < kNumDiag; ++j)
        d[j] = (j == 5) ? (double)tot[j] : (double)tot[j] * 2.3283064365386963e-10;   // 2^-32
    d[3] = (double)((tot[3] << 32) + tot[6]) * 2.3283064365386963e-10;   // energy: high and low words
    const long long n = box->n;
    if (mode == kStatsCentre || mode == kStatsScale) {
        float a[4] = {0.0f, 0.0f, 0.0f, 1.0f};
        if (n > 1 && mode == kStatsCentre) {
            a[0] = (float)(d[0] / (double)n);
            a[1] = (float)(d[1] / (double)n);
            a[2] = (float)(d[2] / (double)n);
        } else if (n > 1) {
            const double P2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const double T = mass * (d[3] - P2 / (double)n) / (3.0 * (double)(n - 1));
            a[3] = (float)(T > 0.0 ? sqrt(kT / T) : 1.0);
        }
        for (int k = 0; k < 4; ++k) st->adj[k] = a[k];
        return;
    }
    for (int k = 0; k < 4; ++k) st->diag[k] = d[k];
    if (mode & kStatsOrigin) {
        st->vacf_len = 0;
        if (box->vacf_stride > 0 && n > 0) {
            box->vacf[0] = d[4] / (double)n;
            st->vacf_len = 1;
        }
    }
    // a new state (admission, mpcd_set_state) is judged on its own; a
    // snapshot on demand only adds flags, so a box marked by a step (or by
    // its initial state) stays marked
    const bool ok = d[5] == 0.0 && d[3] < 1e300;
    if (mode & kStatsOrigin) st->status = ok ? 0 : -5;
    else if (!ok) st->status = -5;
}

// Exact sums of one box's per-tile partials, rounded once to FP64, and the
// use made of them:
//   kStatsCentre   adj = (mean velocity, 1): centres the initial velocities
//   kStatsScale    adj = (0, sqrt(kT/T)): rescales them to temperature kT,
//                  T = m (sum v^2 - |sum v|^2 / n) / (3 (n - 1))
//   kStatsSnapshot diag = (sum m v, sum m v^2), status from the range marks;
//                  with kStatsOrigin also VACF sample 0 = sum v.v0 / n
// Boxes with fewer than two particles get the identity adjustment.  128-bit
// integer accumulation, so the order of the partials does not matter.  One
// workgroup over all tiles, or (many tiles) k_box_stats_tiles first folds
// runs of `per` tiles into one 128-bit partial each, kept in the first two
// tiles' slots of the run, and this kernel reads those (packed = 1).
__global__ __launch_bounds__(kBlock) void k_box_stats(const long long* __restrict__ partials, int nitems,
                                                       int per, int packed, const BoxDev* __restrict__ box,
                                                       BoxState* __restrict__ st, int mode, double kT,
                                                       double mass)
{
    __int128 acc[kNumDiag], tot[kNumDiag];
#pragma unroll
    for (int j = 0; j < kNumDiag; ++j) acc[j] = 0;
    for (int t = threadIdx.x; t < nitems; t += kBlock) {
        if (packed) {
            const __int128* q = reinterpret_cast<const __int128*>(partials + (size_t)t * per * kNumDiag);
#pragma unroll
            for (int j = 0; j < kNumDiag; ++j) acc[j] += q[j];
        } else {
#pragma unroll
            for (int j = 0; j < kNumDiag; ++j) acc[j] += partials[(size_t)t * kNumDiag + j];
        }
    }
    block_sum128(acc, tot);
    if (threadIdx.x == 0) box_stats_finish(tot, box, st, mode, kT, mass);
}

// First level of k_box_stats for boxes with many tiles: workgroup g sums the
// partials of tiles [g per, (g + 1) per) and stores the 128-bit totals over
// the first two tiles of its run (per >= 2; each workgroup reads and writes
// only its own run).
__global__ __launch_bounds__(kBlock) void k_box_stats_tiles(long long* __restrict__ partials, int ntiles, int per)
{
    const int t0 = blockIdx.x * per, t1 = min(ntiles, t0 + per);
    __int128 acc[kNumDiag], tot[kNumDiag];
#pragma unroll
    for (int j = 0; j < kNumDiag; ++j) acc[j] = 0;
    for (int t = t0 + threadIdx.x; t < t1; t += kBlock)
#pragma unroll
        for (int j = 0; j < kNumDiag; ++j) acc[j] += partials[(size_t)t * kNumDiag + j];
    block_sum128(acc, tot);
    __syncthreads();   // every thread has read its tiles before thread 0 overwrites the first two
    if (threadIdx.x == 0) {
        __int128* q = reinterpret_cast<__int128*>(partials + (size_t)t0 * kNumDiag);
        for (int j = 0; j < kNumDiag; ++j) q[j] = tot[j];
    }
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

// Over the slots i of a buffer: dst[i] = src[pid[i]] (gather by id) or
// dst[pid[i]] = src[i] (scatter by id); pid holds each id of [0, n) once and
// -1 in holes.
__global__ __launch_bounds__(kBlock) void k_permute_f32(float* __restrict__ dst, const float* __restrict__ src,
                                                         const int32_t* __restrict__ pid, int64_t nslot,
                                                         int64_t n, int scatter)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nslot; i += (int64_t)gridDim.x * kBlock) {
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

// Exact momentum and kinetic energy of n particles in caller arrays (the
// diagnostics of k_snapshot without a box): workgroup t sums particles
// [t kPartTile, (t + 1) kPartTile) into kNumDiag exact partials, then one
// workgroup adds the partials in 128-bit integers and writes
// out = (sum m v (3), sum m v^2, range violations), each rounded once.
__global__ __launch_bounds__(kBlock) void k_moments_tiles(const float* __restrict__ vx, const float* __restrict__ vy,
                                                           const float* __restrict__ vz, const float* __restrict__ m,
                                                           int64_t n, long long* __restrict__ partials)
{
    const int64_t begin = (int64_t)blockIdx.x * kPartTile, end = min(n, begin + (int64_t)kPartTile);
    long long d[kNumDiag] = {};
    for (int64_t i = begin + threadIdx.x; i < end; i += kBlock)
        diag_particle(d, make_float3(vx[i], vy[i], vz[i]), m ? m[i] : 1.0f);
    block_diag(d, partials + (size_t)blockIdx.x * kNumDiag);
}

__global__ __launch_bounds__(kBlock) void k_moments_finish(const long long* __restrict__ partials, int ntile,
                                                            double* __restrict__ out)
{
    __int128 acc[kNumDiag], tot[kNumDiag];
#pragma unroll
    for (int j = 0; j < kNumDiag; ++j) acc[j] = 0;
    for (int t = threadIdx.x; t < ntile; t += kBlock)
#pragma unroll
        for (int j = 0; j < kNumDiag; ++j) acc[j] += partials[(size_t)t * kNumDiag + j];
    block_sum128(acc, tot);
    if (threadIdx.x == 0) {
#pragma clang fp contract(off)
        for (int j = 0; j < 3; ++j) out[j] = (double)tot[j] * 2.3283064365386963e-10;   // 2^-32
        out[3] = (double)((tot[3] << 32) + tot[6]) * 2.3283064365386963e-10;
        out[4] = (double)tot[5];
    }
}

// Streaming copy of n16 16-byte words: workgroup g copies its own contiguous
// chunk, each thread moving kU words per trip with every load issued before
// the stores (the fastest of the copy forms measured on this GPU: grid-stride
// with and without non-temporal hints, one to eight words per trip, 1024 to
// 65536 workgroups).  It measures the practical HBM ceiling that the step
// kernels are compared with.
__global__ __launch_bounds__(kBlock) void k_hbm_copy(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                                      int64_t n16)
{
    constexpr int kU = 4;
    const int64_t per = (n16 + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(n16, b0 + per);
    int64_t i = b0 + threadIdx.x;
    for (; i + (kU - 1) * kBlock < b1; i += kU * kBlock) {
        f32x4 t[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) t[u] = src[i + u * kBlock];
#pragma unroll
        for (int u = 0; u < kU; ++u) dst[i + u * kBlock] = t[u];
    }
    for (; i < b1; i += kBlock) dst[i] = src[i];
}

// --------------------------------------------------------------------------
// host launchers

#define MPCD_LAUNCH(kern, grid, block, stream, ...)                              \
    do {                                                                          \
        if ((grid) > 0) hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, stream, __VA_ARGS__); \
    } while (0)

template <int kT, int kS, bool kMass, bool kAM, bool kWide, bool kIds>
static void brick_step_run(const Tables& T, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {   // the largest brick record (kMaxBrickCells or kMaxAmBrickCells cells)
        (void)hipFuncSetAttribute((const void*)k_brick_step<kT, kS, kMass, kAM, kWide, kIds>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL((k_brick_step<kT, kS, kMass, kAM, kWide, kIds>), dim3(T.nbtiles), dim3(kT), T.brick_lds + 16,
                       s, T.btiles, T.brick_box, T.boxes, T.state, T.dacc);
}
// Instances: plain without particle ids, plain and per-particle masses with
// 32-bit store offsets (every brick buffer below 2^30 slots), masses with
// 64-bit offsets, and the angular-momentum rule (64-bit offsets; compute
// bound).  The masses instances also serve boxes without masses, and every
// instance but the first serves boxes with and without ids.
template <int kT, int kS>
static void brick_step_at(const Tables& T, hipStream_t s)
{
    if (T.brick_am) brick_step_run<kT, kS, true, true, true, true>(T, s);
    else if (T.brick_wide) brick_step_run<kT, kS, true, false, true, true>(T, s);
    else if (T.brick_mass) brick_step_run<kT, kS, true, false, false, true>(T, s);
    else if (T.brick_ids) brick_step_run<kT, kS, false, false, false, true>(T, s);
    else brick_step_run<kT, kS, false, false, false, false>(T, s);
}

// Launch shapes of the brick step (workgroup size, particles per thread),
// smallest first: one workgroup holds threads x slots particles in
// registers.  Small workgroups let many bricks per CU overlap their phases.
static const struct {
    int threads, slots;
    void (*run)(const Tables&, hipStream_t);
} kBrickShapes[] = {
    {128, 8, brick_step_at<128, 8>},
    {256, 6, brick_step_at<256, 6>},   // fits 4 waves per SIMD
    {256, 8, brick_step_at<256, 8>},
    {512, 8, brick_step_at<512, 8>},
};
constexpr int kNumBrickShapes = (int)(sizeof(kBrickShapes) / sizeof(kBrickShapes[0]));

int brick_shape_for(int64_t bucket)
{
    for (int i = 0; i < kNumBrickShapes; ++i)
        if ((int64_t)kBrickShapes[i].threads * kBrickShapes[i].slots >= bucket) return i;
    return kNumBrickShapes - 1;   // larger buckets run in several chunks
}
int brick_shape_threads(int shape) { return kBrickShapes[shape].threads; }
int brick_shape_slots(int shape) { return kBrickShapes[shape].slots; }

void launch_brick_step(const Tables& T, hipStream_t s)
{
    if (T.nbtiles <= 0) return;
    kBrickShapes[T.brick_shape].run(T, s);
}
void launch_mark_holes(const Tile* tiles, int ntiles, const Tables& T, int all, hipStream_t s)
{
    MPCD_LAUNCH(k_mark_holes, ntiles, kBlock, s, tiles, T.boxes, T.state, all, -1);
}
void launch_rebucket_clear(const Tables& T, hipStream_t s)
{
    MPCD_LAUNCH(k_rebucket_clear, T.nbtiles, kBlock, s, T.btiles, T.boxes, T.state);
}
void launch_box_finish(const Tables& T, hipStream_t s)
{
    MPCD_LAUNCH(k_box_finish, T.nactive, kBlock, s, T.active, T.boxes, T.state, T.dacc, T.host_flag);
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
    MPCD_LAUNCH(k_cell_rotate, T.nctiles, kBlock, s, T.ctiles, T.boxes, T.state, T.dacc);
}

// Per-box launchers: one workgroup per particle tile of box `box` (ntile =
// ceil(nslot / kPartTile)); `part` holds ntile x kNumDiag partials.
void launch_init_maxwell(const Tables& T, int32_t box, int ntile, float vscale, long long* part, hipStream_t s)
{
    MPCD_LAUNCH(k_init_maxwell, ntile, kBlock, s, T.boxes, T.state, box, vscale, part);
}
void launch_init_adjust(const Tables& T, int32_t box, int ntile, long long* part, hipStream_t s)
{
    MPCD_LAUNCH(k_init_adjust, ntile, kBlock, s, T.boxes, T.state, box, part);
}
void launch_snapshot(const Tables& T, int32_t box, int ntile, int set_v0, long long* part, hipStream_t s)
{
    MPCD_LAUNCH(k_snapshot, ntile, kBlock, s, T.boxes, T.state, box, set_v0, part);
}
void launch_box_stats(const Tables& T, int32_t box, int ntile, long long* part, int mode, double kT,
                      double mass, hipStream_t s)
{
    if (ntile <= 4 * kBlock) {
        hipLaunchKernelGGL(k_box_stats, dim3(1), dim3(kBlock), 0, s, part, ntile, 1, 0, T.boxes + box,
                           T.state + box, mode, kT, mass);
        return;
    }
    const int per = (ntile + kBlock - 1) / kBlock;   // >= 5, so each run holds two tiles' slots
    const int groups = (ntile + per - 1) / per;
    hipLaunchKernelGGL(k_box_stats_tiles, dim3(groups), dim3(kBlock), 0, s, part, ntile, per);
    hipLaunchKernelGGL(k_box_stats, dim3(1), dim3(kBlock), 0, s, part, groups, per, 1, T.boxes + box,
                       T.state + box, mode, kT, mass);
}
void launch_mark_holes_box(const Tables& T, int32_t box, int ntile, hipStream_t s)
{
    MPCD_LAUNCH(k_mark_holes, ntile, kBlock, s, nullptr, T.boxes, T.state, 1, box);
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
void launch_permute_f32(float* dst, const float* src, const int32_t* pid, int64_t nslot, int64_t n, int scatter,
                        hipStream_t s)
{
    const int64_t g = (nslot + kBlock - 1) / kBlock;
    MPCD_LAUNCH(k_permute_f32, (int)(g < 65536 ? g : 65536), kBlock, s, dst, src, pid, nslot, n, scatter);
}
void launch_moments(const float* vx, const float* vy, const float* vz, const float* m, int64_t n,
                    long long* partials, double* out, hipStream_t s)
{
    const int ntile = (int)((n + kPartTile - 1) / kPartTile);
    MPCD_LAUNCH(k_moments_tiles, ntile, kBlock, s, vx, vy, vz, m, n, partials);
    hipLaunchKernelGGL(k_moments_finish, dim3(1), dim3(kBlock), 0, s, partials, ntile, out);
}
void launch_hbm_copy(const void* src, void* dst, int64_t n16, int blocks, hipStream_t s)
{
    MPCD_LAUNCH(k_hbm_copy, blocks, kBlock, s, (const f32x4*)src, (f32x4*)dst, n16);
}
void launch_fill_zero_u32(uint32_t* p, int64_t n, hipStream_t s)
{
    const int64_t g = (n + kBlock - 1) / kBlock;
    MPCD_LAUNCH(k_fill_zero_u32, (int)(g < 65536 ? g : 65536), kBlock, s, p, n);
}

}  // namespace mpcd
