/*
 * mpcd_oracle.c -- plain FP64 CPU oracle of the SRD step (test infrastructure
 * only; see mpcd_oracle.h for what is computed and which passage each part
 * follows).  Single threaded, no SIMD intrinsics, no fast-math: every step is
 * written the way the method states it, so it can be checked by eye.
 */
#include "mpcd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 4).  One round multiplies the
 * even counter words by two fixed odd constants, swaps the 32-bit halves of
 * the products with the odd words and mixes in the key; between rounds the
 * key is advanced by two Weyl constants (the golden ratio and sqrt(3) - 1 in
 * 32-bit fixed point). */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double oracle_u24(uint32_t r)
{
    return (double)(r >> 8) * (1.0 / 16777216.0);
}

static void seed_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32);
}

/* Sec. 2 / Fig. 1: the collision grid is displaced by a random vector each
 * step; uniform in [-a/2, a/2)^3 (SRD literature).  Stream 0 of Philox. */
void oracle_shift(uint64_t seed, uint64_t k, double a, double s[3])
{
    uint32_t key[2], ctr[4], r[4];
    seed_key(seed, key);
    ctr[0] = (uint32_t)(k & 0xffffffffu);
    ctr[1] = 0u;
    ctr[2] = (uint32_t)(k >> 32);
    ctr[3] = 0u;
    oracle_philox4x32_10(ctr, key, r);
    for (int d = 0; d < 3; ++d)
        s[d] = a * (oracle_u24(r[d]) - 0.5);
}

/* Sec. 2: one randomly oriented axis per cell.  Uniform on the sphere by
 * Archimedes' hat-box theorem: z uniform in [-1, 1), azimuth uniform in
 * [0, 2 pi).  Stream 1 of Philox, counter word 1 = canonical cell. */
void oracle_axis(uint64_t seed, uint64_t k, uint32_t c, double n[3])
{
    uint32_t key[2], ctr[4], q[4];
    seed_key(seed, key);
    ctr[0] = (uint32_t)(k & 0xffffffffu);
    ctr[1] = c;
    ctr[2] = (uint32_t)(k >> 32);
    ctr[3] = 1u;
    oracle_philox4x32_10(ctr, key, q);
    double zc = 2.0 * oracle_u24(q[0]) - 1.0;
    double phi = 2.0 * M_PI * oracle_u24(q[1]);
    double rho = sqrt(1.0 - zc * zc);
    n[0] = rho * cos(phi);
    n[1] = rho * sin(phi);
    n[2] = zc;
}

/* Sec. 2: the component of w along n is kept, the perpendicular component
 * is turned by the fixed angle about n (Rodrigues' rotation formula). */
void oracle_rotate(const double n[3], double ca, double sa, const double w[3], double out[3])
{
    double cross[3] = {
        n[1] * w[2] - n[2] * w[1],
        n[2] * w[0] - n[0] * w[2],
        n[0] * w[1] - n[1] * w[0],
    };
    double ndotw = n[0] * w[0] + n[1] * w[1] + n[2] * w[2];
    for (int d = 0; d < 3; ++d)
        out[d] = w[d] * ca + cross[d] * sa + n[d] * ndotw * (1.0 - ca);
}

static double wrap_position(double x, double len)
{
    x = x - len * floor(x / len);
    if (x >= len) x -= len;
    if (x < 0.0) x += len;
    if (x >= len) x = 0.0;
    return x;
}

/* Streaming between collisions (not stated in the paper; standard SRD):
 * ballistic move by v dt, then the periodic boundary of Sec. 4. */
void oracle_stream(const oracle_box* b, int64_t N, double* x, double* y, double* z,
                   const double* vx, const double* vy, const double* vz)
{
    double len[3] = { b->L[0] * b->a, b->L[1] * b->a, b->L[2] * b->a };
    for (int64_t i = 0; i < N; ++i) {
        x[i] = wrap_position(x[i] + vx[i] * b->dt, len[0]);
        y[i] = wrap_position(y[i] + vy[i] * b->dt, len[1]);
        z[i] = wrap_position(z[i] + vz[i] * b->dt, len[2]);
    }
}

/* Listing 1: the grid origin moves by +s, so x lies in cell floor((x-s)/a);
 * indices are folded back periodically (the grey image cells of Fig. 1). */
int64_t oracle_cell_of(const oracle_box* b, const double s[3], double x, double y, double z)
{
    double p[3] = { x, y, z };
    int64_t idx[3];
    for (int d = 0; d < 3; ++d) {
        int64_t i = (int64_t)floor((p[d] - s[d]) / b->a);
        while (i < 0) i += b->L[d];
        while (i >= b->L[d]) i -= b->L[d];
        idx[d] = i;
    }
    return idx[0] + (int64_t)b->L[0] * (idx[1] + (int64_t)b->L[1] * idx[2]);
}

void oracle_cells(const oracle_box* b, const double s[3], int64_t N,
                  const double* x, const double* y, const double* z, int64_t* out)
{
    for (int64_t i = 0; i < N; ++i)
        out[i] = oracle_cell_of(b, s, x[i], y[i], z[i]);
}

static int64_t n_cells(const oracle_box* b)
{
    return (int64_t)b->L[0] * b->L[1] * b->L[2];
}

/* Listing 4: per cell, the mass-weighted momentum and the total mass. */
void oracle_cell_sums(const oracle_box* b, const double s[3], int64_t N,
                      const double* x, const double* y, const double* z,
                      const double* vx, const double* vy, const double* vz, const double* m,
                      int64_t* count, double* P, double* M)
{
    int64_t C = n_cells(b);
    memset(count, 0, sizeof(int64_t) * (size_t)C);
    memset(P, 0, sizeof(double) * 3 * (size_t)C);
    memset(M, 0, sizeof(double) * (size_t)C);
    for (int64_t i = 0; i < N; ++i) {
        int64_t c = oracle_cell_of(b, s, x[i], y[i], z[i]);
        double mi = m ? m[i] : 1.0;
        count[c] += 1;
        P[3 * c + 0] += mi * vx[i];
        P[3 * c + 1] += mi * vy[i];
        P[3 * c + 2] += mi * vz[i];
        M[c] += mi;
    }
}

/* Shared by oracle_collide and oracle_collide_given: sums, cell velocity,
 * rotation of every relative velocity (Sec. 2 parts (i)-(iii)). */
static int collide_with_axes(const oracle_box* b, const double s[3],
                             const double* axes, uint64_t seed, uint64_t k, int draw_axes,
                             int64_t N, const double* x, const double* y, const double* z,
                             double* vx, double* vy, double* vz, const double* m,
                             int64_t* cell_out)
{
    int64_t C = n_cells(b);
    int64_t* count = (int64_t*)malloc(sizeof(int64_t) * (size_t)C);
    double* P = (double*)malloc(sizeof(double) * 3 * (size_t)C);
    double* M = (double*)malloc(sizeof(double) * (size_t)C);
    double* ax = draw_axes ? (double*)malloc(sizeof(double) * 3 * (size_t)C) : NULL;
    if (!count || !P || !M || (draw_axes && !ax)) {
        free(count); free(P); free(M); free(ax);
        return -1;
    }
    oracle_cell_sums(b, s, N, x, y, z, vx, vy, vz, m, count, P, M);

    if (draw_axes) {
        for (int64_t c = 0; c < C; ++c) {
            if (count[c] > 0)
                oracle_axis(seed, k, (uint32_t)c, &ax[3 * c]);
        }
        axes = ax;
    }

    double ca = cos(b->alpha), sa = sin(b->alpha);
    for (int64_t i = 0; i < N; ++i) {
        int64_t c = oracle_cell_of(b, s, x[i], y[i], z[i]);
        if (cell_out) cell_out[i] = c;
        double u[3] = { P[3 * c] / M[c], P[3 * c + 1] / M[c], P[3 * c + 2] / M[c] };
        double w[3] = { vx[i] - u[0], vy[i] - u[1], vz[i] - u[2] };
        double r[3];
        oracle_rotate(&axes[3 * c], ca, sa, w, r);
        vx[i] = u[0] + r[0];
        vy[i] = u[1] + r[1];
        vz[i] = u[2] + r[2];
    }
    free(count); free(P); free(M); free(ax);
    return 0;
}

int oracle_collide(const oracle_box* b, uint64_t k, int64_t N,
                   const double* x, const double* y, const double* z,
                   double* vx, double* vy, double* vz, const double* m, int64_t* cell_out)
{
    double s[3];
    oracle_shift(b->seed, k, b->a, s);
    return collide_with_axes(b, s, NULL, b->seed, k, 1, N, x, y, z, vx, vy, vz, m, cell_out);
}

int oracle_collide_given(const oracle_box* b, const double s[3], const double* axes, int64_t N,
                         const double* x, const double* y, const double* z,
                         double* vx, double* vy, double* vz, const double* m)
{
    return collide_with_axes(b, s, axes, 0, 0, 0, N, x, y, z, vx, vy, vz, m, NULL);
}

/* ---------------------------------------------------------------------- */
/* Angular-momentum-conserving collision (SRD+a). */

void oracle_cell_local(const oracle_box* b, const double s[3], double x, double y, double z,
                       double r[3])
{
    double p[3] = { x, y, z };
    for (int d = 0; d < 3; ++d) {
        double q = p[d] - s[d];
        r[d] = q - b->a * floor(q / b->a);
        if (r[d] >= b->a) r[d] -= b->a;
        if (r[d] < 0.0) r[d] = 0.0;
    }
}

/* Determinant of a 3x3 matrix (row major), cofactor expansion on row 0. */
static double det3(const double A[9])
{
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* Eigenvalues of a symmetric 3x3 matrix in closed form, largest first
 * (O. K. Smith, "Eigenvalues of a symmetric 3 x 3 matrix", Comm. ACM 4
 * (1961) 168): with q = tr(A)/3 and p = sqrt(|A - q I|_F^2 / 6), the matrix
 * B = (A - q I)/p has the eigenvalues 2 cos(phi + 2 pi j/3), j = 0, 1, 2,
 * where cos(3 phi) = det(B)/2.  A degenerate pair comes out to about
 * sqrt(machine epsilon) only, but the isolated eigenvalue and the sum of
 * the pair stay accurate, which is all the pseudo-inverse below uses. */
static void sym3_eigenvalues(const double A[9], double e[3])
{
    const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    if (off == 0.0) {   /* diagonal */
        double d[3] = { A[0], A[4], A[8] };
        for (int i = 0; i < 3; ++i)
            for (int j = i + 1; j < 3; ++j)
                if (d[j] > d[i]) { double t = d[i]; d[i] = d[j]; d[j] = t; }
        e[0] = d[0]; e[1] = d[1]; e[2] = d[2];
        return;
    }
    const double q = (A[0] + A[4] + A[8]) / 3.0;
    const double f = (A[0] - q) * (A[0] - q) + (A[4] - q) * (A[4] - q) + (A[8] - q) * (A[8] - q) + 2.0 * off;
    const double p = sqrt(f / 6.0);
    double B[9];
    for (int i = 0; i < 9; ++i) B[i] = (A[i] - ((i % 4) == 0 ? q : 0.0)) / p;
    double r = det3(B) / 2.0;
    if (r < -1.0) r = -1.0;
    if (r > 1.0) r = 1.0;
    const double phi = acos(r) / 3.0;
    const double two_pi_3 = 2.0943951023931954923;   /* 2 pi / 3 */
    e[0] = q + 2.0 * p * cos(phi);
    e[2] = q + 2.0 * p * cos(phi + two_pi_3);
    e[1] = 3.0 * q - e[0] - e[2];
}

static void cross3(const double a[3], const double b[3], double out[3]);

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* y = A x for a 3x3 row-major A */
static void matvec3(const double A[9], const double x[3], double y[3])
{
    for (int i = 0; i < 3; ++i) y[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}

/* Moore-Penrose pseudo-inverse of a symmetric 3x3 matrix from an analytic
 * eigen-decomposition (no iteration):
 *   1. eigenvalues in closed form (sym3_eigenvalues);
 *   2. the isolated eigenvalue (the one farther from the middle eigenvalue,
 *      which the closed form gives to full accuracy) and its eigenvector as
 *      the longest cross product of two rows of A - l I (those rows span the
 *      plane orthogonal to the eigenvector);
 *   3. the other two eigenpairs from the 2x2 matrix A takes in that plane,
 *      diagonalised by the rotation angle t with tan(2t) = 2 b / (a - c);
 *   4. A^+ = sum of e e^T / l over the eigenpairs (l, e) with |l| > tol
 *      times the largest |l|; the others count as zero.
 * (Eigenvalues: O. K. Smith, Comm. ACM 4 (1961) 168; eigenvectors by cross
 * products as in J. Kopp, Int. J. Mod. Phys. C 19 (2008) 523.) */
void oracle_sym3_pinv(const double A[9], double tol, double out[9])
{
    double e[3];
    sym3_eigenvalues(A, e);
    for (int i = 0; i < 9; ++i) out[i] = 0.0;
    /* eigenvector of the isolated eigenvalue */
    const int iso = (e[0] - e[1] >= e[1] - e[2]) ? 0 : 2;
    double r[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r[i][j] = A[3 * i + j] - (i == j ? e[iso] : 0.0);
    double v[3] = { 1.0, 0.0, 0.0 }, best = 0.0;
    const int pairs[3][2] = { { 0, 1 }, { 0, 2 }, { 1, 2 } };
    for (int k = 0; k < 3; ++k) {
        double c[3];
        cross3(r[pairs[k][0]], r[pairs[k][1]], c);
        const double nn = dot3(c, c);
        if (nn > best) {
            best = nn;
            for (int d = 0; d < 3; ++d) v[d] = c[d];
        }
    }
    if (best > 0.0) {   /* otherwise A = l I: any unit vector will do */
        const double inv = 1.0 / sqrt(best);
        for (int d = 0; d < 3; ++d) v[d] *= inv;
    }
    /* orthonormal basis (u, w) of the plane orthogonal to v */
    int ax = 0;
    for (int d = 1; d < 3; ++d)
        if (fabs(v[d]) < fabs(v[ax])) ax = d;
    double ek[3] = { 0.0, 0.0, 0.0 }, u[3], w[3];
    ek[ax] = 1.0;
    cross3(v, ek, u);
    const double un = 1.0 / sqrt(dot3(u, u));
    for (int d = 0; d < 3; ++d) u[d] *= un;
    cross3(v, u, w);
    /* the 2x2 block [[a, b], [b, c]] of A in the plane, and its eigenpairs */
    double Au[3], Aw[3], Av[3];
    matvec3(A, u, Au);
    matvec3(A, w, Aw);
    matvec3(A, v, Av);
    const double a = dot3(u, Au), b = dot3(u, Aw), c = dot3(w, Aw);
    const double t = 0.5 * atan2(2.0 * b, a - c);
    const double ct = cos(t), st = sin(t);
    double vec[3][3], lam[3];
    for (int d = 0; d < 3; ++d) {
        vec[0][d] = v[d];
        vec[1][d] = ct * u[d] + st * w[d];
        vec[2][d] = -st * u[d] + ct * w[d];
    }
    lam[0] = dot3(v, Av);
    lam[1] = a * ct * ct + 2.0 * b * ct * st + c * st * st;
    lam[2] = a * st * st - 2.0 * b * ct * st + c * ct * ct;
    const double lmax = fmax(fabs(lam[0]), fmax(fabs(lam[1]), fabs(lam[2])));
    for (int k = 0; k < 3; ++k) {
        if (!(lmax > 0.0) || !(fabs(lam[k]) > tol * lmax)) continue;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) out[3 * i + j] += vec[k][i] * vec[k][j] / lam[k];
    }
}

static void cross3(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

static int collide_am_with_axes(const oracle_box* b, const double s[3], const double* axes,
                                uint64_t seed, uint64_t k, int draw_axes, int64_t N,
                                const double* x, const double* y, const double* z,
                                double* vx, double* vy, double* vz, const double* m)
{
    int64_t C = n_cells(b);
    double* M = (double*)calloc((size_t)C, sizeof(double));
    double* P = (double*)calloc(3 * (size_t)C, sizeof(double));     /* sum m v */
    double* R1 = (double*)calloc(3 * (size_t)C, sizeof(double));    /* sum m r */
    double* R2 = (double*)calloc(9 * (size_t)C, sizeof(double));    /* sum m r r^T */
    double* dL = (double*)calloc(3 * (size_t)C, sizeof(double));
    double* ax = draw_axes ? (double*)malloc(sizeof(double) * 3 * (size_t)C) : NULL;
    if (!M || !P || !R1 || !R2 || !dL || (draw_axes && !ax)) {
        free(M); free(P); free(R1); free(R2); free(dL); free(ax);
        return -1;
    }
    /* pass 1: mass, momentum, first and second moments of position */
    for (int64_t i = 0; i < N; ++i) {
        int64_t c = oracle_cell_of(b, s, x[i], y[i], z[i]);
        double mi = m ? m[i] : 1.0, r[3];
        oracle_cell_local(b, s, x[i], y[i], z[i], r);
        M[c] += mi;
        P[3 * c + 0] += mi * vx[i];
        P[3 * c + 1] += mi * vy[i];
        P[3 * c + 2] += mi * vz[i];
        for (int d = 0; d < 3; ++d) {
            R1[3 * c + d] += mi * r[d];
            for (int e = 0; e < 3; ++e) R2[9 * c + 3 * d + e] += mi * r[d] * r[e];
        }
    }
    if (draw_axes) {
        for (int64_t c = 0; c < C; ++c)
            if (M[c] > 0) oracle_axis(seed, k, (uint32_t)c, &ax[3 * c]);
        axes = ax;
    }
    double ca = cos(b->alpha), sa = sin(b->alpha);
    /* pass 2: angular momentum change of the plain rotation, per cell */
    for (int64_t i = 0; i < N; ++i) {
        int64_t c = oracle_cell_of(b, s, x[i], y[i], z[i]);
        double mi = m ? m[i] : 1.0, r[3], rc[3], w[3], rw[3], dw[3], l[3];
        oracle_cell_local(b, s, x[i], y[i], z[i], r);
        double v[3] = { vx[i], vy[i], vz[i] };
        for (int d = 0; d < 3; ++d) {
            rc[d] = r[d] - R1[3 * c + d] / M[c];
            w[d] = v[d] - P[3 * c + d] / M[c];
        }
        oracle_rotate(&axes[3 * c], ca, sa, w, rw);
        for (int d = 0; d < 3; ++d) dw[d] = rw[d] - w[d];
        cross3(rc, dw, l);
        for (int d = 0; d < 3; ++d) dL[3 * c + d] += mi * l[d];
    }
    /* per cell: omega = -I^+ dL, I about the centre of mass */
    for (int64_t c = 0; c < C; ++c) {
        if (M[c] <= 0) continue;
        double rcm[3] = { R1[3 * c] / M[c], R1[3 * c + 1] / M[c], R1[3 * c + 2] / M[c] };
        double Q[9], I[9], Ip[9];
        for (int d = 0; d < 3; ++d)
            for (int e = 0; e < 3; ++e) Q[3 * d + e] = R2[9 * c + 3 * d + e] - M[c] * rcm[d] * rcm[e];
        double tr = Q[0] + Q[4] + Q[8];
        for (int d = 0; d < 3; ++d)
            for (int e = 0; e < 3; ++e) I[3 * d + e] = (d == e ? tr : 0.0) - Q[3 * d + e];
        oracle_sym3_pinv(I, 1e-10, Ip);
        double om[3];
        for (int d = 0; d < 3; ++d)
            om[d] = -(Ip[3 * d] * dL[3 * c] + Ip[3 * d + 1] * dL[3 * c + 1] + Ip[3 * d + 2] * dL[3 * c + 2]);
        for (int d = 0; d < 3; ++d) dL[3 * c + d] = om[d];   /* reuse for omega */
    }
    /* pass 3: rotated relative velocity plus the rigid-body correction */
    for (int64_t i = 0; i < N; ++i) {
        int64_t c = oracle_cell_of(b, s, x[i], y[i], z[i]);
        double r[3], rc[3], w[3], rw[3], corr[3];
        oracle_cell_local(b, s, x[i], y[i], z[i], r);
        double v[3] = { vx[i], vy[i], vz[i] }, u[3];
        for (int d = 0; d < 3; ++d) {
            u[d] = P[3 * c + d] / M[c];
            rc[d] = r[d] - R1[3 * c + d] / M[c];
            w[d] = v[d] - u[d];
        }
        oracle_rotate(&axes[3 * c], ca, sa, w, rw);
        cross3(&dL[3 * c], rc, corr);
        vx[i] = u[0] + rw[0] + corr[0];
        vy[i] = u[1] + rw[1] + corr[1];
        vz[i] = u[2] + rw[2] + corr[2];
    }
    free(M); free(P); free(R1); free(R2); free(dL); free(ax);
    return 0;
}

int oracle_collide_am(const oracle_box* b, uint64_t k, int64_t N,
                      const double* x, const double* y, const double* z,
                      double* vx, double* vy, double* vz, const double* m)
{
    double s[3];
    oracle_shift(b->seed, k, b->a, s);
    return collide_am_with_axes(b, s, NULL, b->seed, k, 1, N, x, y, z, vx, vy, vz, m);
}

int oracle_collide_am_given(const oracle_box* b, const double s[3], const double* axes, int64_t N,
                            const double* x, const double* y, const double* z,
                            double* vx, double* vy, double* vz, const double* m)
{
    return collide_am_with_axes(b, s, axes, 0, 0, 0, N, x, y, z, vx, vy, vz, m);
}

int oracle_step(const oracle_box* b, uint64_t k, int64_t N,
                double* x, double* y, double* z, double* vx, double* vy, double* vz,
                const double* m, int64_t* cell_out)
{
    oracle_stream(b, N, x, y, z, vx, vy, vz);
    return oracle_collide(b, k, N, x, y, z, vx, vy, vz, m, cell_out);
}

int oracle_run(const oracle_box* b, uint64_t k0, int64_t nsteps, int64_t N,
               double* x, double* y, double* z, double* vx, double* vy, double* vz,
               const double* m)
{
    for (int64_t t = 0; t < nsteps; ++t) {
        int rc = oracle_step(b, k0 + (uint64_t)t, N, x, y, z, vx, vy, vz, m, NULL);
        if (rc) return rc;
    }
    return 0;
}

/* Conserved quantities of Sec. 2 (momentum, kinetic energy) and the kinetic
 * temperature of the momentum-conserving system. */
void oracle_diagnostics(int64_t N, const double* vx, const double* vy, const double* vz,
                        const double* m, double out[6])
{
    double P[3] = { 0, 0, 0 }, E = 0, Mt = 0;
    for (int64_t i = 0; i < N; ++i) {
        double mi = m ? m[i] : 1.0;
        P[0] += mi * vx[i];
        P[1] += mi * vy[i];
        P[2] += mi * vz[i];
        E += 0.5 * mi * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
        Mt += mi;
    }
    double V[3] = { P[0] / Mt, P[1] / Mt, P[2] / Mt };
    double th = 0;
    for (int64_t i = 0; i < N; ++i) {
        double mi = m ? m[i] : 1.0;
        double wx = vx[i] - V[0], wy = vy[i] - V[1], wz = vz[i] - V[2];
        th += mi * (wx * wx + wy * wy + wz * wz);
    }
    out[0] = P[0];
    out[1] = P[1];
    out[2] = P[2];
    out[3] = E;
    out[4] = N > 1 ? th / (3.0 * (double)(N - 1)) : 0.0;
    out[5] = Mt;
}
