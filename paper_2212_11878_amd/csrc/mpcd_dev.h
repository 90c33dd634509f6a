// mpcd_dev.h -- records shared by the HIP kernels and the host engine of
// libmpcd.so, plus the device-side helpers of the SRD step (Philox, cell
// index, fixed-point sums, rotation).  Internal: not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace mpcd {

// Pointers into device memory are read from the box table, so the compiler
// cannot infer their address space and would emit flat (generic) memory
// instructions; casting them to the global address space gives global_*
// loads, stores and atomics (flat ones also occupy the LDS counter).
#define MPCD_G __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ MPCD_G T* gp(T* p)
{
    return (MPCD_G T*)p;
}
template <class T>
__device__ __forceinline__ const MPCD_G T* gp(const T* p)
{
    return (const MPCD_G T*)p;
}
template <class T>
__device__ __forceinline__ T gatomic_add(MPCD_G T* p, T v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads per workgroup of the particle kernels
constexpr int kPartTile = 4096;      // particles per particle tile (16 per thread)
constexpr int kCellTile = 2048;      // cells per cell tile
constexpr int kMaxBrickCells = 1024; // cells of one brick (LDS of its workgroup)
constexpr int kSortBlockShift = 4;    // the counting sort orders cells in blocks of 16^3
constexpr int kAccWords = 5;         // 64-bit words per brick cell's sums record (4 used)
constexpr int kUnWords = 12;         // 32-bit words per brick cell's data record (7 used)
constexpr int kBrickCellBytes = 8 * kAccWords + 4 * kUnWords;   // LDS per brick cell
// Angular-momentum-conserving collision on bricks: per cell 18 64-bit LDS
// words (first the 13 moment sums, then u, r_c, n, Q / omega in FP64 and the
// 3 angular-momentum sums), and at most kMaxAmBrickCells cells per brick.
constexpr int kAmWords = 18;
constexpr int kAmCellBytes = 8 * kAmWords;
constexpr int kMaxAmBrickCells = 512;
constexpr int kAccLanes = 64;        // step accumulator lanes per box (spread the atomics)
constexpr int kNumDiag = 7;          // per-tile exact partials: sum v (3), sum v^2 (high words), sum v.v0,
                                     // range violations, sum v^2 (low words)

// Per-cell accumulator: exact 64-bit fixed-point sums (quantum 2^-32) of the
// momentum m v and of the mass m (equal masses count as m = 1, so w is
// 2^32 times the particle count).  32 bytes, one sector.
struct alignas(32) CellAcc {
    unsigned long long sx, sy, sz;
    unsigned long long w;
};

// Per-cell collision as an affine map of the velocity: v' = M v + t with
// M = R(n, alpha) (Rodrigues: cos(a) I + sin(a) [n]x + (1 - cos(a)) n n^T,
// n the cell's unit axis) and t = u - M u (u the cell's mass-weighted mean
// velocity), so that v' = u + R (v - u).  Built per cell in FP64 and stored
// in FP32 (48 bytes, three 16-byte pieces).
struct alignas(16) CellRot {
    float m[9];   // row-major M
    float t[3];
};

// Per-cell data of the angular-momentum-conserving collision (FP64): mean
// velocity u, centre of mass r_c (inside the shifted cell), unit axis n and
// the rigid-rotation correction omega; v' = u + R(n, alpha)(v - u) +
// omega x (r - r_c).
struct CellAm {
    double u[3], rc[3], n[3], om[3];
};
// Read-only description of one box, resident in device memory.  Particle
// arrays come in two buffers (ping-pong) of `nslot` slots; the buffer in use
// is BoxState::parity.  Slots that hold no particle carry pid -1 once the
// holes have been marked (the step kernels never read them).
//
// Brick binning (MPCD_BIN_ATOMIC): the L0 x L1 x L2 cells are split into
// nb0 x nb1 x nb2 bricks of 2^bshift cells per dimension (the last brick of
// a dimension may be shorter).  A buffer is cut into
// nbrick + 1 buckets: bucket d = [bstart[d], bstart[d+1]) holds, in its first
// bsize[parity][d] slots, the particles whose collision cell of the coming
// step (position streamed with the current velocity, grid shifted by that
// step's shift) lies in brick d; the last bucket (index nbrick) takes the
// particles that found their bucket full.  The capacities are set by a
// counting sort (re-bucketing) with slack, so one workgroup per brick sees
// every particle of its cells and nothing else.
struct BoxDev {
    float* p[2][6];        // x, y, z, vx, vy, vz
    float4* v0;            // VACF reference velocity of each particle id (x, y, z, unused); null if untracked
    int32_t* pid[2];       // particle identity (admission order); -1 in holes.  Null for boxes
                           // without particle ids (MPCD_UNORDERED): their holes carry x = -1
    float* m[2];           // per-particle masses (null: all particles equal)
    uint32_t* cell;        // sort key of each slot
    uint32_t* rank;        // rank of each slot inside its key (sort)
    uint32_t* perm;        // SORT binning, plain rule: slot of the current buffer whose particle
                           // goes to each slot of the next (null otherwise)
    uint32_t* cstart;      // counts, then exclusive starts, per key (C + 1)
    CellRot* un;           // brick mode: collision map of the cells of flagged bricks
    CellAm* uam;           // brick mode with conserve_l: the same for the angular-momentum rule
    CellAcc* esc[2];       // brick mode: per cell, sums of overflow particles (step parity)
    uint32_t* ecnt[2];     // brick mode with per-particle masses: per cell, overflow particles counted
    uint32_t* eflag;       // brick mode: per brick, k+1 when esc[k & 1] holds data for it
    uint32_t* bstart;      // brick mode: bucket starts (nbrick + 2)
    uint32_t* bsize[2];    // brick mode: particles in each bucket of each buffer (nbrick + 1)
    double* vacf;          // VACF samples
    int64_t n;             // particles
    int64_t nslot;         // slots per buffer (n for SORT boxes)
    int64_t ncell;
    int32_t L[3];
    int32_t nb[3];         // bricks per dimension
    int32_t bshift[3];     // brick edge 2^bshift cells per dimension
    int32_t bmax[3];       // largest brick extent per dimension
    int32_t sshift[3];     // block edge 2^sshift cells of the counting sort's cell order
    int32_t nbrick;
    int32_t vacf_stride;   // 0 = untracked
    int32_t vacf_cap;
    int32_t binning;       // MPCD_BIN_ATOMIC (bricks) or MPCD_BIN_SORT
    int32_t conserve_l;    // 1: angular-momentum-conserving rule
    int32_t ptile0, ptile1;   // slot tiles [ptile0, ptile1)
    int32_t ctile0, ctile1;   // cell tiles [ctile0, ctile1)
    int32_t btile0, btile1;   // brick tiles [btile0, btile1)
    float len[3];          // L_d * a
    float a, inv_a, dt;
    double ca, sa;         // cos(alpha), sin(alpha)
    float mass;
    uint32_t key0, key1;   // Philox key = seed
};

// Mutable per-box state, resident in device memory and advanced by the last
// kernel of every step, so a captured step replays unchanged.
struct BoxState {
    long long k;           // steps completed
    long long remaining;   // steps left; < 0 = unbounded
    long long vacf_origin; // step at which v0 was taken
    int parity;            // particle buffer in use
    int vacf_len;
    int status;            // 0 or MPCD_ESTATE
    int rebucket;          // brick mode: buckets to be rebuilt by the counting sort
    long long overflow_steps;   // brick mode: steps in which a bucket was full
    long long rebuckets;        // brick mode: re-bucketings done
    double diag[4];        // sum m v (3), sum m v^2 of the last snapshot (exact sums, rounded once)
    float adj[4];          // initial-state adjustment v <- (v - adj[0..2]) * adj[3]
};

// Record copies to and from global memory as native vectors (struct
// assignment is not defined across address spaces).
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store_acc(MPCD_G CellAcc* p, const CellAcc& a)
{
    MPCD_G u64x2* q = (MPCD_G u64x2*)p;
    u64x2 lo, hi;
    lo.x = a.sx; lo.y = a.sy; hi.x = a.sz; hi.y = a.w;
    q[0] = lo;
    q[1] = hi;
}

__device__ __forceinline__ CellAcc load_acc(const MPCD_G CellAcc* p)
{
    const MPCD_G u64x2* q = (const MPCD_G u64x2*)p;
    const u64x2 lo = q[0], hi = q[1];
    CellAcc a;
    a.sx = lo.x; a.sy = lo.y; a.sz = hi.x; a.w = hi.y;
    return a;
}

__device__ __forceinline__ void store_rot(MPCD_G CellRot* p, const CellRot& r)
{
    MPCD_G f32x4* q = (MPCD_G f32x4*)p;
    f32x4 a, b, c;
    a.x = r.m[0]; a.y = r.m[1]; a.z = r.m[2]; a.w = r.m[3];
    b.x = r.m[4]; b.y = r.m[5]; b.z = r.m[6]; b.w = r.m[7];
    c.x = r.m[8]; c.y = r.t[0]; c.z = r.t[1]; c.w = r.t[2];
    q[0] = a;
    q[1] = b;
    q[2] = c;
}

__device__ __forceinline__ CellRot load_rot(const MPCD_G CellRot* p)
{
    const MPCD_G f32x4* q = (const MPCD_G f32x4*)p;
    const f32x4 a = q[0], b = q[1], c = q[2];
    CellRot r;
    r.m[0] = a.x; r.m[1] = a.y; r.m[2] = a.z; r.m[3] = a.w;
    r.m[4] = b.x; r.m[5] = b.y; r.m[6] = b.z; r.m[7] = b.w;
    r.m[8] = c.x; r.t[0] = c.y; r.t[1] = c.z; r.t[2] = c.w;
    return r;
}

// A contiguous range of one box's particles or cells.
struct Tile {
    int32_t box;
    int32_t pad;
    int64_t begin, end;
};

// ----------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products whose halves are exchanged with the odd words and the round key;
// the key advances by the Weyl increments after every round.
__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b)
{
    return (uint32_t)(((uint64_t)a * b) >> 32);
}

__host__ __device__ __forceinline__ uint4 philox4x32_10(uint4 ctr, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a = ctr.x, b = ctr.z;
        const uint32_t lo_a = a * 0xD2511F53u, hi_a = mulhi32(a, 0xD2511F53u);
        const uint32_t lo_b = b * 0xCD9E8D57u, hi_b = mulhi32(b, 0xCD9E8D57u);
        ctr = make_uint4(hi_b ^ ctr.y ^ k0, lo_b, hi_a ^ ctr.w ^ k1, lo_a);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return ctr;
}

// top 24 bits as a float in [0, 1); exact
__host__ __device__ __forceinline__ float unit24(uint32_t r)
{
    return (float)(r >> 8) * 5.9604644775390625e-8f;   // 2^-24
}

// Grid shift of step k: s_d = a (u_d - 1/2), stream 0.
__host__ __device__ __forceinline__ float3 grid_shift(const BoxDev& b, long long k)
{
    const uint4 r = philox4x32_10(
        make_uint4((uint32_t)k, 0u, (uint32_t)((unsigned long long)k >> 32), 0u), b.key0, b.key1);
    return make_float3(b.a * (unit24(r.x) - 0.5f), b.a * (unit24(r.y) - 0.5f),
                       b.a * (unit24(r.z) - 0.5f));
}

// Rotation axis of canonical cell c at step k, uniform on the sphere
// (z uniform in [-1, 1), azimuth uniform), stream 1.
__device__ __forceinline__ float3 cell_axis(const BoxDev& b, long long k, uint32_t c)
{
    const uint4 q = philox4x32_10(
        make_uint4((uint32_t)k, c, (uint32_t)((unsigned long long)k >> 32), 1u), b.key0, b.key1);
    const float z = 2.0f * unit24(q.x) - 1.0f;
    const float phi = 6.2831853071795864769f * unit24(q.y);
    float sp, cp;
    sincosf(phi, &sp, &cp);
    const float rho = sqrtf(fmaxf(0.0f, 1.0f - z * z));
    float3 n = make_float3(rho * cp, rho * sp, z);
    // renormalise (one Newton step on rsqrt) so |n| = 1 to rounding, unbiased
    const float nn = n.x * n.x + n.y * n.y + n.z * n.z;
    float r = rsqrtf(nn);
    r = r * (1.5f - 0.5f * nn * r * r);
    return make_float3(n.x * r, n.y * r, n.z * r);
}

// Periodic fold of a streamed coordinate into [0, len).  A coordinate less
// than one box length outside needs one add or subtract (x + len of a
// negative x rounds at most up to len, which the subtract maps to 0); farther
// ones (and non-finite values) take the floor division and a final guard.
__host__ __device__ __forceinline__ float fold(float x, float len)
{
    if (!(x >= -len && x < 2.0f * len)) {
        x -= len * floorf(x / len);
        x = (x < 0.0f) ? x + len : x;
        x = (x >= len) ? x - len : x;
        return (x < 0.0f || x >= len) ? 0.0f : x;   // rounding landed on an edge
    }
    x = (x < 0.0f) ? x + len : x;
    return (x >= len) ? x - len : x;
}

// Cell index along one axis of the grid displaced by s (floor((x - s)/a)),
// folded periodically: for x in [0, L a) and |s| <= a/2 the floor lies in
// [-1, L], so one add or subtract wraps it.  axis_cell_raw may return values
// outside [0, L) for non-finite x (callers range-check it); axis_cell clamps.
__host__ __device__ __forceinline__ int axis_cell_raw(float x, float s, float inv_a, int L)
{
    unsigned i = (unsigned)(int)floorf((x - s) * inv_a);
    const unsigned up = i + (unsigned)L;
    i = up < i ? up : i;   // -1 -> L - 1
    const unsigned dn = i - (unsigned)L;
    return (int)(dn < i ? dn : i);   // L -> 0
}
__host__ __device__ __forceinline__ int axis_cell(float x, float s, float inv_a, int L)
{
    const int c = axis_cell_raw(x, s, inv_a, L);
    return c < 0 ? 0 : (c > L - 1 ? L - 1 : c);
}

__device__ __forceinline__ uint32_t collision_cell(const BoxDev& b, float x, float y, float z,
                                                   float3 s)
{
    const int ix = axis_cell(x, s.x, b.inv_a, b.L[0]);
    const int iy = axis_cell(y, s.y, b.inv_a, b.L[1]);
    const int iz = axis_cell(z, s.z, b.inv_a, b.L[2]);
    return (uint32_t)ix + (uint32_t)b.L[0] * ((uint32_t)iy + (uint32_t)b.L[1] * (uint32_t)iz);
}

// Brick geometry along one dimension: brick i covers cells
// [i 2^shift, min((i+1) 2^shift, L)).
__host__ __device__ __forceinline__ int brick_lo(int i, int shift) { return i << shift; }
__host__ __device__ __forceinline__ int brick_of(int c, int shift) { return c >> shift; }

// Cell order of the counting sort (SORT binning): cells are numbered block by
// block, in blocks of 2^sh[d] cells per dimension (blocks in x-fastest order,
// cells x-fastest inside a block; the last block of a dimension may be
// shorter, and the numbering stays dense over [0, L0 L1 L2)).  A particle
// moves at most one cell per step, so in this order its new place in the
// sorted buffer lies close to its old one and the scatter's writes stay
// local.  sort_key maps cell (ix, iy, iz) to its position; cell_of_key maps
// a position back to the cell index ix + L0 (iy + L1 iz).
__host__ __device__ __forceinline__ uint32_t sort_key(const int32_t L[3], const int32_t sh[3], int ix, int iy, int iz)
{
    const uint64_t Lx = (uint64_t)L[0], Ly = (uint64_t)L[1], Lz = (uint64_t)L[2];
    const uint64_t lox = (uint64_t)((ix >> sh[0]) << sh[0]), loy = (uint64_t)((iy >> sh[1]) << sh[1]),
                   loz = (uint64_t)((iz >> sh[2]) << sh[2]);
    const uint64_t bx = (uint64_t)1 << sh[0], by = (uint64_t)1 << sh[1], bz = (uint64_t)1 << sh[2];
    const uint64_t ex = Lx - lox < bx ? Lx - lox : bx;
    const uint64_t ey = Ly - loy < by ? Ly - loy : by;
    const uint64_t ez = Lz - loz < bz ? Lz - loz : bz;
    const uint64_t base = loz * Lx * Ly + ez * (loy * Lx + ey * lox);
    return (uint32_t)(base + ((uint64_t)ix - lox) + ex * (((uint64_t)iy - loy) + ey * ((uint64_t)iz - loz)));
}

__host__ __device__ __forceinline__ uint32_t cell_of_key(const int32_t L[3], const int32_t sh[3], uint32_t key)
{
    // 32-bit arithmetic: with block edges clipped to the box, every product
    // below is at most the number of cells (< 2^32)
    const uint32_t Lx = (uint32_t)L[0], Ly = (uint32_t)L[1], Lz = (uint32_t)L[2];
    const uint32_t bx = (1u << sh[0]) < Lx ? (1u << sh[0]) : Lx;
    const uint32_t by = (1u << sh[1]) < Ly ? (1u << sh[1]) : Ly;
    const uint32_t bz = (1u << sh[2]) < Lz ? (1u << sh[2]) : Lz;
    uint32_t r = key;
    // block layer along z (the last one may be thinner)
    const uint32_t nz = (Lz + bz - 1) / bz;
    uint32_t iz = r / (Lx * Ly * bz);
    iz = iz < nz - 1 ? iz : nz - 1;
    const uint32_t loz = iz * bz, ez = Lz - loz < bz ? Lz - loz : bz;
    r -= loz * Lx * Ly;
    // block row along y inside the layer
    const uint32_t ny = (Ly + by - 1) / by;
    uint32_t iy = r / (Lx * ez * by);
    iy = iy < ny - 1 ? iy : ny - 1;
    const uint32_t loy = iy * by, ey = Ly - loy < by ? Ly - loy : by;
    r -= loy * Lx * ez;
    // block along x inside the row
    const uint32_t nx = (Lx + bx - 1) / bx;
    uint32_t ix = r / (ey * ez * bx);
    ix = ix < nx - 1 ? ix : nx - 1;
    const uint32_t lox = ix * bx, ex = Lx - lox < bx ? Lx - lox : bx;
    r -= lox * ey * ez;
    const uint32_t cx = lox + r % ex, cy = loy + (r / ex) % ey, cz = loz + r / (ex * ey);
    return cx + Lx * (cy + Ly * cz);
}

// Sort key of the collision cell of streamed position (x, y, z) under shift s.
__device__ __forceinline__ uint32_t sort_cell(const BoxDev& b, float x, float y, float z, float3 s)
{
    return sort_key(b.L, b.sshift, axis_cell(x, s.x, b.inv_a, b.L[0]), axis_cell(y, s.y, b.inv_a, b.L[1]),
                    axis_cell(z, s.z, b.inv_a, b.L[2]));
}

// Neighbour of brick b at offset r (-1, 0, 1) along a dimension with nb
// bricks (periodic), or -1 when there is none (nb <= 2 and b + r outside).
__host__ __device__ __forceinline__ int brick_nbr(int b, int r, int nb)
{
    int t = b + r;
    if (nb >= 3) {
        t += (t < 0) ? nb : 0;
        t -= (t >= nb) ? nb : 0;
        return t;
    }
    return (t >= 0 && t < nb) ? t : -1;
}

// Offset (-1, 0, 1) of brick `to` from brick `from` along a dimension with nb
// bricks (periodic); 2 when it is farther.
__host__ __device__ __forceinline__ int brick_rel(int from, int to, int nb)
{
    int r = to - from;
    if (nb >= 3) {
        if (r == nb - 1) r = -1;
        else if (r == 1 - nb) r = 1;
    }
    return (r >= -1 && r <= 1) ? r : 2;
}

// Brick decomposition of one box: bricks of `want` cells per dimension (a
// power of two; 8 when 0), at most the box.
struct BrickGeom {
    int L[3], shift[3], nb[3], bmax[3], nbrick, bvol;
};

inline bool brick_edge_ok(int e) { return e == 0 || (e >= 2 && e <= 64 && (e & (e - 1)) == 0); }

inline BrickGeom brick_geometry(const int32_t L[3], const int32_t want[3])
{
    BrickGeom g{};
    g.nbrick = 1;
    g.bvol = 1;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = L[d];
        const int B = want[d] > 0 ? want[d] : 8;
        int sh = 0;
        while ((2 << sh) <= B) ++sh;   // floor(log2 B)
        g.shift[d] = sh;
        g.nb[d] = (L[d] + (1 << sh) - 1) >> sh;
        g.bmax[d] = L[d] < (1 << sh) ? L[d] : (1 << sh);
        g.nbrick *= g.nb[d];
        g.bvol *= g.bmax[d];
    }
    return g;
}

// Bucket holding slot i: the last d in [0, nbk] with start[d] <= i (empty
// buckets share their start with the next one); start[0] = 0.
__host__ __device__ __forceinline__ int bucket_of_slot(const uint32_t* start, int nbk, int64_t i)
{
    int lo = 0, hi = nbk;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)start[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ceil(sqrt(n)), exactly, for n < 2^32.
__host__ __device__ __forceinline__ uint32_t isqrt_ceil(uint32_t n)
{
    uint32_t r = (uint32_t)sqrtf((float)n);
    while ((unsigned long long)r * r > n) --r;
    while ((unsigned long long)r * r < n) ++r;
    return r;
}

// Spare slots given to a bucket that re-bucketing found holding n
// particles: the bucket's size wanders like a Poisson count, so the margin
// is about 4 standard deviations plus 1/8 and a constant.
__host__ __device__ __forceinline__ uint32_t bucket_slack(uint32_t n) { return (n >> 3) + 4u * isqrt_ceil(n) + 32u; }

// Slots per buffer of a brick box: the buckets with their slack (the sum of
// sqrt(n_d) over nb buckets is at most sqrt(nb n)), plus an overflow bucket
// that can take every particle.
inline int64_t brick_slots(int64_t n, int64_t nbrick)
{
    const int64_t root = (int64_t)ceil(sqrt((double)n * (double)nbrick)) + 1;
    return 2 * n + (n >> 3) + 4 * (root + nbrick) + 32 * nbrick;
}

// Velocity in 64-bit fixed point with quantum 2^-32: v 2^32 truncated toward
// zero, as a two's-complement integer, taken from the bits of v (exact for
// |v| >= 2^-9; smaller magnitudes lose less than one quantum).  With the
// 24-bit significand m (implicit bit set) and biased exponent e,
// |v| 2^32 = m 2^(e - 118) = (m 2^39) >> (157 - e); exponents of 2^-33 and
// below shift everything out (the shift is capped at 63), and so do
// |v| >= 2^31, zero, subnormal and non-finite values (the range check of the
// steps flags every velocity from kVelocityLimit up).
__host__ __device__ __forceinline__ unsigned long long to_fixed(float v)
{
    const uint32_t u = __builtin_bit_cast(uint32_t, v);
    const uint32_t e = (u >> 23) & 0xffu;
    const uint32_t sh = (e == 0u || e > 157u) ? 63u : (157u - e < 63u ? 157u - e : 63u);
    const unsigned long long mag = ((unsigned long long)((u & 0x7fffffu) | 0x800000u) << 39) >> sh;
    return (u >> 31) ? 0ull - mag : mag;
}

// Range of the exact sums.  Every velocity component stays below
// kVelocityLimit and every mass in [kMassMin, kMassMax], so a term m v 2^32
// of a cell sum is below 2^48; a cell of fewer than kMaxCellCount particles
// then sums to less than 2^60, and a box tile of kPartTile particles too, so
// no 64-bit sum can wrap.  The steps count a violation (the box's status
// becomes MPCD_ESTATE) for every velocity beyond the limit and every cell
// holding kMaxCellCount particles or more.
constexpr float kVelocityLimit = 256.0f;    // 2^8
constexpr float kMassMin = 0.00390625f;     // 2^-8
constexpr float kMassMax = 256.0f;          // 2^8
constexpr uint32_t kMaxCellCount = 4096u;   // 2^12

// Exact value of a two's-complement 64-bit fixed-point sum as FP64 (hi and
// lo 32-bit halves are exact; their combination rounds once).
__host__ __device__ __forceinline__ double fixed_to_double(unsigned long long s)
{
#pragma clang fp contract(off)
    const double hi = (double)(int)(unsigned)(s >> 32);
    const double lo = (double)(unsigned)(s & 0xffffffffu);
    return hi * 4294967296.0 + lo;
}

// Mass-weighted mean velocity of a cell, sum(m v) / sum(m), from the exact
// fixed-point sums, in FP64: one reciprocal of the mass sum, three products.
__host__ __device__ __forceinline__ void fixed_mean3(unsigned long long sx, unsigned long long sy, unsigned long long sz,
                                            unsigned long long w, double u[3])
{
#pragma clang fp contract(off)
    const double inv = 1.0 / fixed_to_double(w);
    u[0] = fixed_to_double(sx) * inv;
    u[1] = fixed_to_double(sy) * inv;
    u[2] = fixed_to_double(sz) * inv;
}

// Slot i of buffer par holds a particle: holes carry pid -1, or x = -1 in
// boxes without particle ids (a non-finite position still counts as a
// particle; valid positions are never negative).
__device__ __forceinline__ bool slot_live(const BoxDev& b, int par, int64_t i)
{
    return b.pid[par] ? b.pid[par][i] >= 0 : !(b.p[par][0][i] < 0.0f);
}
__device__ __forceinline__ void mark_hole(const BoxDev& b, int par, int64_t i)
{
    if (b.pid[par]) b.pid[par][i] = -1;
    else b.p[par][0][i] = -1.0f;
}

// mass of particle i (1 when the box has equal masses)
__device__ __forceinline__ float mass_of(const float* __restrict__ m, int64_t i)
{
    return m ? m[i] : 1.0f;
}

// The collision map of a cell with mean velocity u (FP64) and axis n (FP32,
// normalised here in FP64).  M is rounded to FP32 entry by entry; t is
// formed from the rounded M, so that sum(m v') = M P + M_tot (u - M u) = P
// holds to the rounding of the result.  The entry roundings are independent
// from cell to cell, so they add no systematic change of the kinetic energy
// (a rotation evaluated in FP32 with one cos(a), sin(a) pair for every cell
// does: cos^2 + sin^2 != 1 by a fixed amount).
__host__ __device__ __forceinline__ CellRot cell_rotation(double ux, double uy, double uz, float3 axis, double ca,
                                                 double sa)
{
    double nx = axis.x, ny = axis.y, nz = axis.z;
    const double inv = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
    nx *= inv;
    ny *= inv;
    nz *= inv;
    const double oc = 1.0 - ca;
    CellRot r;
    r.m[0] = (float)(ca + oc * nx * nx);
    r.m[1] = (float)(oc * nx * ny - sa * nz);
    r.m[2] = (float)(oc * nx * nz + sa * ny);
    r.m[3] = (float)(oc * ny * nx + sa * nz);
    r.m[4] = (float)(ca + oc * ny * ny);
    r.m[5] = (float)(oc * ny * nz - sa * nx);
    r.m[6] = (float)(oc * nz * nx - sa * ny);
    r.m[7] = (float)(oc * nz * ny + sa * nx);
    r.m[8] = (float)(ca + oc * nz * nz);
    r.t[0] = (float)(ux - ((double)r.m[0] * ux + (double)r.m[1] * uy + (double)r.m[2] * uz));
    r.t[1] = (float)(uy - ((double)r.m[3] * ux + (double)r.m[4] * uy + (double)r.m[5] * uz));
    r.t[2] = (float)(uz - ((double)r.m[6] * ux + (double)r.m[7] * uy + (double)r.m[8] * uz));
    return r;
}

// v' = M v + t (three fused multiply-adds per component, fixed order)
__host__ __device__ __forceinline__ float3 apply_rotation(const CellRot& r, float vx, float vy, float vz)
{
    return make_float3(fmaf(r.m[0], vx, fmaf(r.m[1], vy, fmaf(r.m[2], vz, r.t[0]))),
                       fmaf(r.m[3], vx, fmaf(r.m[4], vy, fmaf(r.m[5], vz, r.t[1]))),
                       fmaf(r.m[6], vx, fmaf(r.m[7], vy, fmaf(r.m[8], vz, r.t[2]))));
}

// Rotated relative velocity R w in FP64 (Rodrigues, as cell_rotation).
__device__ __forceinline__ void rotate_w(double nx, double ny, double nz, double ca, double sa,
                                         const double w[3], double out[3])
{
#pragma clang fp contract(off)
    const double d = nx * w[0] + ny * w[1] + nz * w[2];
    const double px = d * nx, py = d * ny, pz = d * nz;
    out[0] = px + ca * (w[0] - px) + sa * (ny * w[2] - nz * w[1]);
    out[1] = py + ca * (w[1] - py) + sa * (nz * w[0] - nx * w[2]);
    out[2] = pz + ca * (w[2] - pz) + sa * (nx * w[1] - ny * w[0]);
}

// Moore-Penrose pseudo-inverse of a symmetric 3x3 matrix a[3][3] by cyclic
// Jacobi rotations (eigenvalues below tol times the largest count as zero).
__device__ __forceinline__ void sym3_pinv(double a[3][3], double tol, double out[3][3])
{
#pragma clang fp contract(off)
    double v[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 12; ++sweep) {
        if (fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]) < 1e-300) break;
#pragma unroll
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            if (fabs(a[p][q]) < 1e-300) continue;
            const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
            const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double akp = a[k][p], akq = a[k][q];
                a[k][p] = c * akp - sn * akq;
                a[k][q] = sn * akp + c * akq;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double apk = a[p][k], aqk = a[q][k];
                a[p][k] = c * apk - sn * aqk;
                a[q][k] = sn * apk + c * aqk;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double vkp = v[k][p], vkq = v[k][q];
                v[k][p] = c * vkp - sn * vkq;
                v[k][q] = sn * vkp + c * vkq;
            }
        }
    }
    const double e0 = a[0][0], e1 = a[1][1], e2 = a[2][2];
    const double emax = fmax(fabs(e0), fmax(fabs(e1), fabs(e2)));
    const double i0 = (emax > 0 && fabs(e0) > tol * emax) ? 1.0 / e0 : 0.0;
    const double i1 = (emax > 0 && fabs(e1) > tol * emax) ? 1.0 / e1 : 0.0;
    const double i2 = (emax > 0 && fabs(e2) > tol * emax) ? 1.0 / e2 : 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            out[i][j] = v[i][0] * i0 * v[j][0] + v[i][1] * i1 * v[j][1] + v[i][2] * i2 * v[j][2];
}

// Every component finite and below kVelocityLimit in magnitude (written with
// comparisons only: a maximum would drop a NaN component).
__host__ __device__ __forceinline__ bool in_range(float3 v)
{
    return fabsf(v.x) < kVelocityLimit && fabsf(v.y) < kVelocityLimit && fabsf(v.z) < kVelocityLimit;
}

// Exact diagnostics: per-particle terms in 64-bit fixed point (quantum 2^-32)
// so block and box sums do not depend on summation order.
__device__ __forceinline__ long long fixed_term(double t)
{
#pragma clang fp contract(off)
    t = fmin(fmax(t * 4294967296.0, -4.0e18), 4.0e18);
    return (long long)rint(t);
}

// Momentum m v and twice the kinetic energy m v^2 of one particle (the energy
// term, below 2^60, is summed as high and low 32-bit words so that a tile of
// kPartTile particles cannot wrap), and the range check of its velocity and
// mass.
__device__ __forceinline__ void diag_particle(long long (&d)[kNumDiag], float3 v, float m)
{
    d[0] += fixed_term((double)m * v.x);
    d[1] += fixed_term((double)m * v.y);
    d[2] += fixed_term((double)m * v.z);
    const long long e = fixed_term((double)m * ((double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z));
    d[3] += e >> 32;
    d[6] += e & 0xffffffffll;
    if (!in_range(v) || !(m >= kMassMin && m <= kMassMax)) d[5] += 1;
}

// range check of a new velocity (non-finite or beyond the exact-sum range)
__host__ __device__ __forceinline__ void diag_check(long long (&d)[kNumDiag], float3 v)
{
    if (!in_range(v)) d[5] += 1;
}

// VACF term v . v0, below 3 2^48 in fixed point, so a workgroup's sum of at
// most 4096 terms stays below 2^62
__device__ __forceinline__ void diag_vacf(long long (&d)[kNumDiag], float3 v, float w0x, float w0y,
                                          float w0z)
{
    d[4] += fixed_term((double)v.x * w0x + (double)v.y * w0y + (double)v.z * w0z);
}

// --------------------------------------------------------------------------
// Angular-momentum-conserving collision (the plain rotation followed by the
// rigid-body velocity omega x r' that restores the cell's angular momentum
// about its centre of mass, omega = -I^+ dL).  The same functions serve the
// counting-sort path (one thread walks a cell) and the brick path (LDS sums
// over a brick), so both give the same bits: every cell sum is an exact
// fixed-point integer and the per-cell algebra is FP64.

constexpr int kAmMoments = 13;   // m, m v (3), m r (3), m r r^T (6)

// Position of a streamed particle inside its shifted cell (shift sh, edge a),
// each component in [0, a).
__device__ __forceinline__ void am_local(double a, float x, float y, float z, float3 sh, double r[3])
{
#pragma clang fp contract(off)
    const double q[3] = {(double)x - sh.x, (double)y - sh.y, (double)z - sh.z};
    if (a == 1.0) {   // unit cells: the same value without the divisions
#pragma unroll
        for (int e = 0; e < 3; ++e) r[e] = q[e] - floor(q[e]);
        return;
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) r[e] = q[e] - a * floor(q[e] / a);
}

// One particle's exact terms of the first pass: mass, momentum, first and
// second position moments.
__device__ __forceinline__ void am_moments(double mj, float vx, float vy, float vz, const double r[3],
                                           long long t[kAmMoments])
{
#pragma clang fp contract(off)
    t[0] = fixed_term(mj);
    t[1] = fixed_term(mj * vx);
    t[2] = fixed_term(mj * vy);
    t[3] = fixed_term(mj * vz);
#pragma unroll
    for (int e = 0; e < 3; ++e) t[4 + e] = fixed_term(mj * r[e]);
    t[7] = fixed_term(mj * r[0] * r[0]);
    t[8] = fixed_term(mj * r[0] * r[1]);
    t[9] = fixed_term(mj * r[0] * r[2]);
    t[10] = fixed_term(mj * r[1] * r[1]);
    t[11] = fixed_term(mj * r[1] * r[2]);
    t[12] = fixed_term(mj * r[2] * r[2]);
}

// Cell data from the first-pass sums: mean velocity u, centre of mass rc,
// second moment Q (xx, xy, xz, yy, yz, zz) about rc, and the unit axis n of
// canonical cell c at step k.
__device__ __forceinline__ void am_cell(const BoxDev& b, long long k, uint32_t c, const long long s[kAmMoments],
                                        double u[3], double rc[3], double Q[6], double n[3])
{
#pragma clang fp contract(off)
    const double M = fixed_to_double((unsigned long long)s[0]);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        u[e] = fixed_to_double((unsigned long long)s[1 + e]) / M;
        rc[e] = fixed_to_double((unsigned long long)s[4 + e]) / M;
    }
    // sums are in units of 2^-32: Mt is the true mass; u and rc are ratios
    const double k2 = 2.3283064365386963e-10;
    const double Mt = M * k2;
    Q[0] = fixed_to_double((unsigned long long)s[7]) * k2 - Mt * rc[0] * rc[0];
    Q[1] = fixed_to_double((unsigned long long)s[8]) * k2 - Mt * rc[0] * rc[1];
    Q[2] = fixed_to_double((unsigned long long)s[9]) * k2 - Mt * rc[0] * rc[2];
    Q[3] = fixed_to_double((unsigned long long)s[10]) * k2 - Mt * rc[1] * rc[1];
    Q[4] = fixed_to_double((unsigned long long)s[11]) * k2 - Mt * rc[1] * rc[2];
    Q[5] = fixed_to_double((unsigned long long)s[12]) * k2 - Mt * rc[2] * rc[2];
    const float3 ax = cell_axis(b, k, c);
    const double nx = ax.x, ny = ax.y, nz = ax.z;
    const double inv = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
    n[0] = nx * inv;
    n[1] = ny * inv;
    n[2] = nz * inv;
}

// One particle's exact second-pass terms: the change of its angular momentum
// about rc under the plain rotation, m r' x (R w - w), w = v - u.  Returns
// false when a term reaches 2^48 in fixed point (a cell of fewer than
// kMaxCellCount such terms cannot wrap its 64-bit sum).
__device__ __forceinline__ bool am_dl(double mj, float vx, float vy, float vz, const double r[3],
                                      const double u[3], const double rc[3], const double n[3], double ca,
                                      double sa, long long t[3])
{
#pragma clang fp contract(off)
    double w[3], rw[3];
    w[0] = (double)vx - u[0];
    w[1] = (double)vy - u[1];
    w[2] = (double)vz - u[2];
    rotate_w(n[0], n[1], n[2], ca, sa, w, rw);
    const double rp[3] = {r[0] - rc[0], r[1] - rc[1], r[2] - rc[2]};
    const double dw[3] = {rw[0] - w[0], rw[1] - w[1], rw[2] - w[2]};
    t[0] = fixed_term(mj * (rp[1] * dw[2] - rp[2] * dw[1]));
    t[1] = fixed_term(mj * (rp[2] * dw[0] - rp[0] * dw[2]));
    t[2] = fixed_term(mj * (rp[0] * dw[1] - rp[1] * dw[0]));
    constexpr long long kLim = 1ll << 48;
    return t[0] > -kLim && t[0] < kLim && t[1] > -kLim && t[1] < kLim && t[2] > -kLim && t[2] < kLim;
}

// omega = -I^+ dL with I = tr(Q) 1 - Q (pseudo-inverse: rank-deficient cells,
// e.g. one or two particles, get no correction along the null directions).
__device__ __forceinline__ void am_omega(const double Q6[6], const long long sl[3], double om[3])
{
#pragma clang fp contract(off)
    const double k2 = 2.3283064365386963e-10;
    const double dL[3] = {fixed_to_double((unsigned long long)sl[0]) * k2,
                          fixed_to_double((unsigned long long)sl[1]) * k2,
                          fixed_to_double((unsigned long long)sl[2]) * k2};
    const double Q[3][3] = {{Q6[0], Q6[1], Q6[2]}, {Q6[1], Q6[3], Q6[4]}, {Q6[2], Q6[4], Q6[5]}};
    double I[3][3], Ip[3][3];
    const double tr = Q[0][0] + Q[1][1] + Q[2][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) I[i][j] = (i == j ? tr : 0.0) - Q[i][j];
    sym3_pinv(I, 1e-10, Ip);
#pragma unroll
    for (int i = 0; i < 3; ++i) om[i] = -(Ip[i][0] * dL[0] + Ip[i][1] * dL[1] + Ip[i][2] * dL[2]);
}

// New velocity: u + R (v - u) + omega x (r - rc), rounded once to FP32.
__device__ __forceinline__ float3 am_velocity(float vx, float vy, float vz, const double r[3], const double u[3],
                                              const double rc[3], const double n[3], const double om[3],
                                              double ca, double sa)
{
#pragma clang fp contract(off)
    double w[3], rw[3];
    w[0] = (double)vx - u[0];
    w[1] = (double)vy - u[1];
    w[2] = (double)vz - u[2];
    rotate_w(n[0], n[1], n[2], ca, sa, w, rw);
    const double rp[3] = {r[0] - rc[0], r[1] - rc[1], r[2] - rc[2]};
    return make_float3((float)(u[0] + rw[0] + (om[1] * rp[2] - om[2] * rp[1])),
                       (float)(u[1] + rw[1] + (om[2] * rp[0] - om[0] * rp[2])),
                       (float)(u[2] + rw[2] + (om[0] * rp[1] - om[1] * rp[0])));
}

// Blocks are dealt round-robin to the 8 XCDs; renumber so that each XCD
// works on one contiguous run of tiles (neighbouring bricks exchange
// particles, whose bucket lines then meet in one L2).
__device__ __forceinline__ int xcd_tile(int bid, int nblocks)
{
    const int q = nblocks >> 3, r = nblocks & 7;
    const int x = bid & 7, i = bid >> 3;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace mpcd
