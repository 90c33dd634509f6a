/*
 * mpcd.h -- C ABI of the MI355X Stochastic Rotation Dynamics (SRD/MPCD)
 * library libmpcd.so.
 *
 * The library advances periodic boxes of point particles with the SRD step
 * of Halver, Junghans, Sutmann, "Kokkos-Based Implementation of MPCD on
 * Heterogeneous Nodes" (arXiv 2212.11878), Sec. 2: every step it
 *   1. streams every particle, x <- x + v dt, folded into the periodic box
 *      (the paper's benchmark boundary conditions, Sec. 4);
 *   2. draws a random grid shift s in [-a/2, a/2)^3 (Sec. 2, Fig. 1) and puts
 *      each particle into the cell floor((x - s)/a) of the displaced grid
 *      (Sec. 3.1, Listing 1);
 *   3. reduces each cell's centre-of-mass velocity u_c = sum(m v)/sum(m)
 *      (Sec. 3.3, Listing 4);
 *   4. rotates each relative velocity v - u_c by the fixed angle alpha about
 *      a random unit axis drawn per cell (Sec. 2, parts (ii)-(iii)).
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the box seed;
 * the shift of step k uses counter (k_lo, 0, k_hi, 0), the axis of canonical
 * cell c = ix + Lx (iy + Ly iz) uses counter (k_lo, c, k_hi, 1).  Results
 * therefore depend only on (seed, step, state), never on storage order or on
 * which other boxes share the device.
 *
 * Precision: positions and velocities are FP32.  Per-cell momentum sums are
 * exact two's-complement 64-bit fixed point (velocity quantum 2^-32, each
 * term truncated toward zero, exact for |v| >= 2^-9), so the sum is
 * independent of summation order; global momentum / energy diagnostics are
 * exact fixed-point sums rounded once to FP64.
 *
 * Range of the exact sums: every velocity component must stay below 256 in
 * magnitude (units of a per unit time: choose units with kT/m of order 1, as
 * the method's reduced units do), every per-particle mass in [2^-8, 2^8],
 * and every collision cell below 4096 particles.  A step that meets a
 * velocity or a cell outside this range, or a non-finite velocity, marks the
 * box MPCD_ESTATE (mpcd_observe); no sum ever wraps silently.
 *
 * General conventions
 *   - Every call returns an mpcd_status; a failing call leaves the context
 *     unchanged (admission is all-or-nothing).
 *   - A context is not thread safe: use it from one host thread.
 *   - Device work is queued on the context's HIP stream; only mpcd_observe,
 *     mpcd_get_state, mpcd_set_state, mpcd_set_mass, mpcd_get_mass,
 *     mpcd_get_vacf, mpcd_set_vacf and mpcd_kernel_stats synchronise with
 *     it, and mpcd_admit when it times autotuner trials
 *     (MPCD_BIN_AUTO, a box of at least 2^21 cells of a shape class new to
 *     the context).
 *   - Pointers marked "host" are ordinary host memory owned by the caller
 *     and only read or written during the call.
 */
#ifndef MPCD_H
#define MPCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPCD_ABI_VERSION 4

typedef enum {
    MPCD_OK = 0,
    MPCD_EINVAL = -1,   /* invalid argument or descriptor                  */
    MPCD_ENOMEM = -2,   /* over the context's device-memory budget, or the
                           allocator refused                                */
    MPCD_EDEVICE = -3,  /* a HIP runtime call failed                        */
    MPCD_EBUSY = -4,    /* no free slot                                     */
    MPCD_ESTATE = -5,   /* NaN/Inf detected in a box's diagnostics          */
    MPCD_ENOTFOUND = -6 /* slot not live                                    */
} mpcd_status;

/* mpcd_box_desc.flags */
#define MPCD_INIT_MAXWELL 0x1u   /* draw uniform positions and Maxwellian
                                    velocities on the device (zero momentum,
                                    temperature exactly kT)                 */
#define MPCD_INIT_EXTERNAL 0x2u  /* caller supplies the state with
                                    mpcd_set_state before the first step    */
#define MPCD_TRACK_VACF 0x4u     /* record the velocity autocorrelation     */
#define MPCD_CONSERVE_L 0x10u    /* angular-momentum-conserving collision
                                    (the "+a" variant of Sec. 2): after the
                                    rotation each cell gets the rigid-body
                                    velocity w x r' that restores its angular
                                    momentum about its centre of mass,
                                    w = -I^+ dL; kinetic energy is then not
                                    conserved.  Brick binning and counting-
                                    sort binning give the same bits; bricks
                                    of such a box hold at most 512 cells.  */
#define MPCD_PARTICLE_MASS 0x8u  /* every particle carries its own mass
                                    (initially desc.mass; mpcd_set_mass);
                                    cell velocities are mass weighted
                                    (Sec. 3.3, Listing 4)                   */
#define MPCD_UNORDERED 0x20u     /* particle identity is not kept: the steps
                                    move x and v only (48 instead of 56 bytes
                                    per particle-step on bricks), and
                                    mpcd_get_state returns the particles in
                                    storage order.  The SRD result is the
                                    same set of particles (the collision
                                    never depends on storage order).  Not
                                    with MPCD_TRACK_VACF or
                                    MPCD_PARTICLE_MASS (EINVAL)             */

/* mpcd_options.binning */
#define MPCD_BIN_AUTO 0    /* autotuner chooses per box-shape class         */
#define MPCD_BIN_ATOMIC 1  /* particles kept in buckets by the brick of cells
                              holding their next collision cell; one pass
                              per brick: LDS-atomic cell sums, rotation, and
                              the store into the next step's bucket.  A box
                              whose two buffers would need 2^32 slots or more
                              (about 1.9e9 particles) uses MPCD_BIN_SORT   */
#define MPCD_BIN_SORT 2    /* counting-sort particles by collision cell every
                              step, then reduce each cell's contiguous run   */

/* One periodic box (a "slot" once admitted). */
typedef struct {
    int32_t L[3];          /* cells per edge, each in [1, 4096]; L0*L1*L2 < 2^31 */
    double a;              /* cell edge, > 0 (at most 16 with MPCD_CONSERVE_L) */
    int64_t n_particles;   /* >= 0                                           */
    double dt;             /* streaming time step, > 0                       */
    double alpha;          /* rotation angle in radians, finite              */
    double kT;             /* initial temperature (MPCD_INIT_MAXWELL), > 0,
                              with kT / mass <= 256 (thermal speed <= 16)   */
    double mass;           /* particle mass, > 0 (all particles), or the
                              initial one with MPCD_PARTICLE_MASS, then in
                              [2^-8, 2^8]                                   */
    uint64_t seed;         /* Philox key                                     */
    int64_t n_steps;       /* steps this box runs, then idles; 0 = unbounded */
    uint32_t flags;        /* one MPCD_INIT_* | MPCD_TRACK_VACF |
                              MPCD_PARTICLE_MASS | MPCD_CONSERVE_L |
                              MPCD_UNORDERED                                 */
    int32_t vacf_stride;   /* steps between VACF samples, >= 1 when tracked  */
    int32_t vacf_capacity; /* max VACF samples kept; 0 = n_steps/stride + 1
                              (1024 if n_steps == 0)                        */
} mpcd_box_desc;

/* Device allocator supplied by the caller (e.g. backed by PyTorch).  Must
 * return device memory aligned to >= 256 bytes, or NULL, and be ordered on
 * the context stream: memory given back by the free callback may be handed
 * out again only to work queued after it on that stream (PyTorch's caching
 * allocator on the same stream is). */
typedef void* (*mpcd_alloc_fn)(size_t bytes, void* user);
typedef void (*mpcd_free_fn)(void* ptr, void* user);

typedef struct {
    int32_t binning;        /* MPCD_BIN_*                                    */
    int32_t brick[3];       /* ATOMIC: brick edge in cells per dimension,
                               each 0 (auto) or a power of two in [2, 64];
                               a box whose brick (edges clipped to its own
                               edges) exceeds 1024 cells is refused by
                               mpcd_admit with MPCD_EINVAL                   */
    int32_t block;          /* reserved, must be 0                           */
    int32_t use_graph;      /* 1: replay steps from a captured hipGraph      */
    int64_t hbm_budget;     /* bytes all boxes may occupy; 0 = unlimited     */
    void* stream;           /* hipStream_t; NULL = the library creates one   */
    mpcd_alloc_fn alloc;    /* NULL = hipMalloc                              */
    mpcd_free_fn free;      /* NULL = hipFree                                */
    void* user;             /* passed to alloc/free                          */
    int32_t device;         /* HIP device ordinal                            */
    int32_t max_slots;      /* 0 = 4096                                      */
} mpcd_options;

typedef struct {
    int64_t step;           /* steps completed                               */
    double P[3];            /* total momentum (FP64 sum of FP32 data)        */
    double E_kin;           /* kinetic energy                                */
    double T;               /* sum m |v - V|^2 / (3 (N - 1)), k_B = 1        */
    double mass_total;
    int32_t status;         /* MPCD_OK or MPCD_ESTATE                        */
    int32_t vacf_len;       /* number of VACF samples                        */
    const double* vacf;     /* host; valid until the next call on the ctx;
                               sample j = (1/N) sum_i v_i(j stride) . v_i(0) */
    int64_t n_particles;
    int32_t binning;        /* binning mode in use for this box              */
    int32_t brick[3];       /* ATOMIC: brick edges in use (largest brick)    */
    int64_t overflow_steps; /* ATOMIC: steps in which a bucket was full (its
                               particles took the slow overflow path)      */
    int64_t rebuckets;      /* ATOMIC: re-bucketings since admission or the
                               last mpcd_set_state                          */
} mpcd_observables;

/* Per-kernel timing collected while profiling is on. */
typedef struct {
    const char* name;       /* static string                                 */
    int64_t launches;
    double total_ms;        /* sum of HIP-event durations on the ctx stream  */
} mpcd_kernel_stat;

typedef struct mpcd_ctx mpcd_ctx;   /* opaque, owned by the library */

/* Create a context on options->device (options may be NULL: defaults): the
 * device tables that let one launch sequence advance many independent boxes
 * (the paper's small systems under-fill a GPU, Sec. 4; batching them is this
 * library's answer).  *out receives the handle.  EINVAL for bad options,
 * EDEVICE if the device cannot be used, ENOMEM if the tables cannot be
 * allocated. */
int mpcd_create(const mpcd_options* options, mpcd_ctx** out);

/* Admit one box (Sec. 4 workload: cubic periodic box of unit cells holding
 * on average n_particles / (L0 L1 L2) particles).  Allocates its device
 * state through the context allocator and, with MPCD_INIT_MAXWELL, draws the
 * initial state on the device (Philox counter (i_lo, i_hi, 0, 2) for
 * positions, (i_lo, i_hi, 0, 3) for Box-Muller velocities; mean removed,
 * rescaled to temperature kT).  The initial state is queued on the stream
 * behind the steps already queued, and the box joins the next mpcd_step.
 * The box starts at step 0.  *slot receives its index.
 * ENOMEM over budget, EBUSY no free slot, EINVAL bad descriptor. */
int mpcd_admit(mpcd_ctx* ctx, const mpcd_box_desc* desc, int32_t* slot);

/* Queue n_steps SRD steps (Sec. 2: streaming, random grid shift, cell
 * velocity, rotation about a random axis) for every live box whose step
 * budget is not exhausted; boxes that reach desc.n_steps stop advancing.
 * Asynchronous on the context stream.  EINVAL for n_steps < 0. */
int mpcd_step(mpcd_ctx* ctx, int32_t n_steps);

/* Synchronise and read a box's diagnostics: total momentum and kinetic
 * energy, which the collision conserves (Sec. 2), and the temperature, each
 * summed exactly over the current state by one pass on the device (the
 * steps themselves only check the range and, on sampled steps, accumulate
 * the VACF).  out (host) is filled; out->vacf stays valid until the next
 * call on ctx.  Returns MPCD_ESTATE (and fills *out) if a velocity became
 * non-finite or left the range of the exact sums; ENOTFOUND for a slot not
 * live. */
int mpcd_observe(mpcd_ctx* ctx, int32_t slot, mpcd_observables* out);

/* Copy a box's state -- the particle positions and velocities that the
 * method advances (Sec. 2) -- to host memory xyzv (6 N floats, SoA: x[N],
 * y[N], z[N], vx[N], vy[N], vz[N]) in the particle order given at admission
 * / the last mpcd_set_state (MPCD_UNORDERED boxes: storage order); *step
 * (host, may be NULL) receives the steps completed.  Synchronises.
 * ESTATE if the device copy is inconsistent; ENOTFOUND for a slot not
 * live. */
int mpcd_get_state(mpcd_ctx* ctx, int32_t slot, float* xyzv, int64_t* step);

/* Replace a box's state (Sec. 2: positions and velocities) with host xyzv
 * (layout as mpcd_get_state; positions must lie in [0, L_d a)) and set its
 * step counter, which keys the random shift and axes of the following
 * steps; the velocities become the VACF reference v(0), starting a new
 * series (mpcd_set_vacf restores an old one).  EINVAL if a position is out
 * of range or not finite (state unchanged).  Synchronises. */
int mpcd_set_state(mpcd_ctx* ctx, int32_t slot, const float* xyzv, int64_t step);

/* Per-particle masses (box admitted with MPCD_PARTICLE_MASS): host mass[N],
 * indexed like mpcd_set_state's particles, each in [2^-8, 2^8].  The cell
 * velocity becomes sum(m v) / sum(m) (Sec. 3.3, Listing 4) and the
 * diagnostics are mass weighted.  Masses travel with their particles and
 * survive mpcd_set_state.  EINVAL for a box without per-particle masses or a
 * bad value (state unchanged).  Synchronises. */
int mpcd_set_mass(mpcd_ctx* ctx, int32_t slot, const float* mass);

/* Copy a box's per-particle masses (Sec. 3.3, Listing 4) to host mass[N] in
 * particle order, as mpcd_set_mass takes them.  EINVAL for a box without
 * per-particle masses.  Synchronises. */
int mpcd_get_mass(mpcd_ctx* ctx, int32_t slot, float* mass);

/* Read a box's VACF record (MPCD_TRACK_VACF): host v0 (3 N floats SoA,
 * particle order; may be NULL) receives the reference velocities, *origin
 * (may be NULL) the step at which they were taken, samples (host) up to max
 * of the samples so far (sample j = (1/N) sum_i v_i(origin + j stride) .
 * v0_i), *len (may be NULL) their number.  With mpcd_get_state,
 * mpcd_get_mass and mpcd_set_vacf it checkpoints a box so that a resumed run
 * continues bit for bit.  EINVAL for a box without VACF.  Synchronises. */
int mpcd_get_vacf(mpcd_ctx* ctx, int32_t slot, float* v0, int64_t* origin, double* samples, int32_t max,
                  int32_t* len);

/* Restore a VACF record after mpcd_set_state: host v0 (3 N floats SoA,
 * particle order, finite), the origin step and the len samples taken so
 * far, which must be exactly those of steps origin, origin + stride, ... up
 * to the box's current step (EINVAL otherwise, or if len exceeds the
 * capacity).  Synchronises. */
int mpcd_set_vacf(mpcd_ctx* ctx, int32_t slot, const float* v0, int64_t origin, const double* samples,
                  int32_t len);

/* Free a box's device state; the slot number may be reused.  Does not wait
 * for queued steps: the memory goes back through the context's allocator,
 * which must be stream-ordered (work already queued on the context stream
 * may still read it; hipFree, the default, waits for the device).  The box
 * tables are rebuilt before the next step.  ENOTFOUND for a slot not live.
 * This is also how a request is cancelled in flight: released with steps of
 * it still queued, the box stops there and the other boxes go on unchanged.
 * (Slots are this library's unit of batching; the paper has none.) */
int mpcd_release(mpcd_ctx* ctx, int32_t slot);

/* Turn per-kernel HIP-event timing on (1) or off (0); turning it on clears
 * the statistics.  While it is on, steps are launched eagerly (not from the
 * captured graph) with an event pair around every kernel. */
int mpcd_profile(mpcd_ctx* ctx, int32_t enable);

/* Synchronise and copy up to max entries of per-kernel timing into out
 * (host); *count receives the number of kernels with statistics. */
int mpcd_kernel_stats(mpcd_ctx* ctx, mpcd_kernel_stat* out, int32_t max, int32_t* count);

/* Release every box and the context itself (waits for the stream).  NULL is
 * ignored. */
void mpcd_destroy(mpcd_ctx* ctx);

/* Static description of a status code. */
const char* mpcd_strerror(int status);

/* MPCD_ABI_VERSION of the loaded library. */
int mpcd_abi_version(void);

/* Exact total momentum and twice the kinetic energy of n particles held in
 * caller device arrays -- the quantities the collision conserves (Sec. 2),
 * summed as mpcd_observe sums them (exact 64-bit fixed-point terms, 128-bit
 * totals, each result rounded once to FP64): vx, vy, vz (device, n floats
 * each), mass (device, n floats, or NULL for unit masses).  out (device, 5
 * doubles) receives sum m v (3), sum m v^2 and the number of particles
 * outside the range of the exact sums (velocity component >= 256 or not
 * finite, mass outside [2^-8, 2^8]).  Works on HIP stream `stream` (NULL =
 * the null stream) with a workspace of ceil(n / 4096) x 56 bytes that it
 * allocates, and waits for the stream before it frees it.  EINVAL for bad
 * arguments, EDEVICE if the allocation or a launch fails. */
int mpcd_moments(const float* vx, const float* vy, const float* vz, const float* mass, int64_t n, double* out,
                 void* stream);

/* mpcd_moments for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, the same results bit for bit, but the workspace is a
 * static device array of the library (3.5 MiB per GPU, kept until the process
 * ends), so n may be at most 2^28 particles (EINVAL beyond), nothing is
 * allocated or freed, and the call returns without waiting (out is written
 * in stream order).  Every call on a GPU shares that GPU's workspace: calls
 * whose work overlaps on one GPU (different streams, or host threads) race;
 * calls ordered on one stream do not. */
int mpcd_moments_noalloc(const float* vx, const float* vy, const float* vz, const float* mass, int64_t n,
                         double* out, void* stream);

/* The CPU leg of hybrid CPU+GPU execution (Sec. 3.2 and Sec. 4, Fig. 2f: part
 * of a run's work on the host's cores next to the GPU).  Advances one box
 * held in host memory by n_steps SRD steps, steps step .. step + n_steps - 1,
 * on `threads` host threads (0 = every core), with the GPU path's method and
 * random streams: streaming with the periodic fold (Sec. 2), the grid shift
 * of Sec. 3.1 and the per-cell axes drawn from Philox4x32-10 keyed by
 * desc->seed, exact fixed-point cell sums (the mass-weighted mean of Sec. 3.3
 * with MPCD_PARTICLE_MASS), the cell's collision map built in FP64 and
 * applied in FP32; binning is a counting sort by collision cell every step.
 * Results match the GPU's within the parity tolerance (the host's sinf/cosf
 * can move an axis by one unit in the last place).
 *   xyzv: host, 6 n floats SoA (x, y, z, vx, vy, vz), positions in [0, L a),
 *         updated in place; on return the particles are in the cell order of
 *         the last step;
 *   mass: host, n floats in [2^-8, 2^8] with MPCD_PARTICLE_MASS, else NULL;
 *   pid:  host, n int32 or NULL, any values (e.g. particle ids);
 * mass and pid travel with their particles.  The caller owns every buffer;
 * the call allocates host memory of about 40 bytes per particle and 8 per
 * cell for its duration, and returns when the steps are done.  EINVAL for a
 * descriptor mpcd_admit refuses, MPCD_CONSERVE_L or MPCD_TRACK_VACF (kept by
 * contexts only), a position outside the box or a non-finite velocity (the
 * state is then untouched); ESTATE when a velocity leaves the range of the
 * exact sums or a cell holds 4096 particles or more (the state then holds
 * the steps' results); ENOMEM when the work buffers cannot be allocated and
 * EDEVICE when a host thread cannot start (in both cases before any step:
 * the state is untouched). */
int mpcd_host_step(const mpcd_box_desc* desc, float* xyzv, float* mass, int32_t* pid, int64_t step,
                   int32_t n_steps, int32_t threads);

/* Measurement only (not part of the method): copy `bytes` bytes from device
 * src to device dst with the library's streaming copy kernel (16-byte loads
 * and stores, `blocks` workgroups of 256 threads each copying a contiguous
 * chunk, 0 = 8192) on HIP stream
 * `stream` (NULL = the null stream), asynchronously.  Its rate is the
 * practical HBM ceiling the SRD kernels are compared with.  EINVAL unless
 * both pointers are 16-byte aligned and bytes is a multiple of 16. */
int mpcd_hbm_copy(const void* src, void* dst, size_t bytes, int32_t blocks, void* stream);

#ifdef __cplusplus
}
#endif
#endif
