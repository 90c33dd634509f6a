/*
 * mpcd_oracle.h -- plain, slow FP64 CPU oracle for one Stochastic Rotation
 * Dynamics (SRD / MPCD) time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no source, header, table or constant
 * generator with the HIP library.
 *
 * What it computes (Halver, Junghans, Sutmann, "Kokkos-Based Implementation
 * of MPCD on Heterogeneous Nodes", arXiv 2212.11878):
 *   Sec. 2: particles are sorted into a randomly shifted grid of cubic cells;
 *     in every cell the velocity relative to the cell's centre-of-mass
 *     velocity is split into the components parallel and perpendicular to a
 *     random axis, and the perpendicular one is turned about the axis by a
 *     fixed angle.  This conserves linear momentum and kinetic energy.
 *   Sec. 3.1, Listing 1: the collision grid origin is displaced by the
 *     random offset, i.e. a particle at x sits in cell floor((x - s)/a).
 *   Sec. 3.3, Listing 4: the cell velocity is mass weighted:
 *     u_c = sum(m v) / sum(m).
 *   Sec. 4: benchmark boxes are cubic and periodic, a = 1, 10 particles per
 *     cell on average.
 * What the paper leaves open is filled from the SRD literature it cites
 * (Gompper, Ihle, Kroll, Winkler, Adv. Polym. Sci. 221 (2009)):
 *   streaming x <- x + v dt before every collision, periodic wrap; shift
 *   uniform in [-a/2, a/2)^3; axis uniform on the unit sphere; rotation by
 *   +alpha, right handed (Rodrigues); temperature with 3(N-1) degrees of
 *   freedom.  The random draws come from Philox4x32-10 (Salmon, Moraes,
 *   Dror, Shaw, SC'11), written here from that paper's definition:
 *     shift : key = seed, counter = (k_lo, 0, k_hi, 0)
 *     axis  : key = seed, counter = (k_lo, cell, k_hi, 1)
 *   where k is the step number (0 for the first step) and cell the canonical
 *   index ix + Lx*(iy + Ly*iz) of the shifted collision cell.
 */
#ifndef MPCD_ORACLE_H
#define MPCD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t  L[3];     /* cells per edge */
    double   a;        /* cell edge */
    double   dt;       /* time step */
    double   alpha;    /* rotation angle in radians */
    uint64_t seed;     /* Philox key */
} oracle_box;

/* Philox4x32 with 10 rounds: out = Philox(ctr, key). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Top 24 bits of a 32-bit word scaled to [0, 1): exact in FP32 and FP64. */
double oracle_u24(uint32_t r);

/* Random grid shift of step k, s_d in [-a/2, a/2). */
void oracle_shift(uint64_t seed, uint64_t k, double a, double s[3]);

/* Random unit axis of canonical cell c at step k. */
void oracle_axis(uint64_t seed, uint64_t k, uint32_t c, double n[3]);

/* Rotate w about the unit axis n by the angle whose cosine and sine are
 * (ca, sa):  w' = w ca + (n x w) sa + n (n.w)(1 - ca). */
void oracle_rotate(const double n[3], double ca, double sa, const double w[3], double out[3]);

/* Streaming with periodic wrap into [0, L_d a). */
void oracle_stream(const oracle_box* b, int64_t N, double* x, double* y, double* z,
                   const double* vx, const double* vy, const double* vz);

/* Canonical shifted-cell index of a position inside the box. */
int64_t oracle_cell_of(const oracle_box* b, const double s[3], double x, double y, double z);

/* oracle_cell_of for every particle: out[i] = cell of particle i. */
void oracle_cells(const oracle_box* b, const double s[3], int64_t N,
                  const double* x, const double* y, const double* z, int64_t* out);

/* Per-cell sums for shift s: count[c], P[3c+d] = sum m v_d, M[c] = sum m
 * (m == NULL means unit masses).  Arrays have L0*L1*L2 entries; they are
 * overwritten. */
void oracle_cell_sums(const oracle_box* b, const double s[3], int64_t N,
                      const double* x, const double* y, const double* z,
                      const double* vx, const double* vy, const double* vz, const double* m,
                      int64_t* count, double* P, double* M);

/* Collision of step k (no streaming): bin with the step-k shift, form the
 * mass-weighted cell velocities, rotate every relative velocity.  If
 * cell_out != NULL it receives each particle's canonical cell.
 * Returns 0, or -1 if memory could not be allocated. */
int oracle_collide(const oracle_box* b, uint64_t k, int64_t N,
                   const double* x, const double* y, const double* z,
                   double* vx, double* vy, double* vz, const double* m, int64_t* cell_out);

/* Collision with an axis supplied by the caller for every cell (axes[3c+d])
 * and the shift supplied explicitly.  Used to pin the rotation step against
 * hand-worked examples. */
int oracle_collide_given(const oracle_box* b, const double s[3], const double* axes, int64_t N,
                         const double* x, const double* y, const double* z,
                         double* vx, double* vy, double* vz, const double* m);

/* Angular-momentum-conserving collision of step k (the "+a" variants the
 * paper mentions in Sec. 2; rule of Noguchi and Gompper, as reviewed in
 * Gompper et al. 2009): after the stochastic rotation every particle of a
 * cell gets the rigid-body velocity w x r'_i, r'_i its position relative to
 * the cell's centre of mass, with w = -I^+ dL, I the cell's moment of inertia
 * tensor about that centre (pseudo-inverse for collinear cells) and dL the
 * change of the cell's angular momentum caused by the rotation.  Linear and
 * angular momentum of every cell are conserved; kinetic energy is not.
 * Returns 0, or -1 if memory could not be allocated. */
int oracle_collide_am(const oracle_box* b, uint64_t k, int64_t N,
                      const double* x, const double* y, const double* z,
                      double* vx, double* vy, double* vz, const double* m);

/* oracle_collide_am with a caller-supplied shift and per-cell axes. */
int oracle_collide_am_given(const oracle_box* b, const double s[3], const double* axes, int64_t N,
                            const double* x, const double* y, const double* z,
                            double* vx, double* vy, double* vz, const double* m);

/* Position of a particle relative to the lower corner of its shifted cell,
 * each component in [0, a). */
void oracle_cell_local(const oracle_box* b, const double s[3], double x, double y, double z,
                       double r[3]);

/* Moore-Penrose pseudo-inverse of a symmetric 3x3 matrix (row major) from
 * an analytic eigen-decomposition: eigenvalues in closed form (Smith 1961),
 * the isolated eigenvalue's eigenvector from a cross product of two rows of
 * A - l I, the other two from the 2x2 block in the orthogonal plane;
 * eigenvalues of magnitude at most tol * (largest) count as 0. */
void oracle_sym3_pinv(const double A[9], double tol, double out[9]);

/* One full step k: streaming, then collision. */
int oracle_step(const oracle_box* b, uint64_t k, int64_t N,
                double* x, double* y, double* z, double* vx, double* vy, double* vz,
                const double* m, int64_t* cell_out);

/* nsteps steps starting at step k0. */
int oracle_run(const oracle_box* b, uint64_t k0, int64_t nsteps, int64_t N,
               double* x, double* y, double* z, double* vx, double* vy, double* vz,
               const double* m);

/* Global diagnostics: out[0..2] = total momentum, out[3] = kinetic energy,
 * out[4] = temperature with 3(N-1) degrees of freedom (k_B = 1),
 * out[5] = total mass. */
void oracle_diagnostics(int64_t N, const double* vx, const double* vy, const double* vz,
                        const double* m, double out[6]);

#ifdef __cplusplus
}
#endif
#endif
