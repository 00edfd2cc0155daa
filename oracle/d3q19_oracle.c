/*
 * D3Q19 central-moment lattice Boltzmann method -- plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU path.
 *
 * Source: A. De Rosis & C. Coreixas, "Multiphysics flow simulations using
 * D3Q19 lattice Boltzmann methods based on central moments" (arXiv
 * 2010.01628).  Every function names the section/equation it follows.
 *
 * Readings of the paper taken here:
 *   R1  Last row of the CM basis T (eq. "matrix") and of M (App. C) is printed
 *       as cy^2 cy^2; it is cy^2 cz^2 (the printed numeric M row is non-zero
 *       exactly at the four populations with cy,cz both non-zero).
 *   R2  The velocity used in the shift, the equilibrium and the output is the
 *       force-shifted u = (sum_i f_i c_i + F/2)/rho (App. E macroscopic
 *       variables; required for k1* = Fx/2 of eq. "posColl0").
 *   R3  App. C raw moments r16*, r17* miss cs^2 on the k5* term and r18*
 *       misses cs^2 on the k6* term (eq. "rawQ19"); cs^2 is inserted.
 *   R4  App. C populations f3* ("r4-r5-2-r6") and f12* ("r4-r5-r6") both read
 *       (r4 - r5 - 2 r6) cs^2/2 (eq. "pdfQ19").
 *   R5  K = diag(1,1,1,1, w_b, w,w,w,w,w, w_hi(9)); the paper sets w_b = 1 and
 *       w_hi = 1 (Sec. II.B).  w_b and w_hi are kept as free inputs so that the
 *       learned-rate variant and the bulk-rate tests can use them.
 *   R6  F is a force density (eq. "lbe" and the Rayleigh-Taylor body force).
 *   R9  Raw-moment variant (App. C, N = I): its printed post-collision list
 *       carries only the forcing terms of the CM scheme (F/2 on rows 1-3,
 *       cs^2 F/2 on rows 10-15).  The relaxation eq. (posColl0) with T = M
 *       needs the raw moments of the same forcing term, which App. B prints
 *       (eq. RMQ19, with velocity terms on rows 4-18); those are used.  Both
 *       agree when F = 0, and at K = I the variant equals the CM scheme.
 *
 * Layout: populations are structure-of-arrays, f[i*N + n] with
 * n = x + nx*(y + ny*z); forces F[d*N + n].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* Sec. II.A: discrete velocities, in the paper's "swap trick" order. */
static const int CX[Q] = {0, -1, 0, 0, -1, -1, -1, -1, 0, 0, 1, 0, 0, 1, 1, 1, 1, 0, 0};
static const int CY[Q] = {0, 0, -1, 0, -1, 1, 0, 0, -1, -1, 0, 1, 0, 1, -1, 0, 0, 1, 1};
static const int CZ[Q] = {0, 0, 0, -1, 0, 0, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1};

/* Sec. II.A: weights w0 = 1/3, ws = 1/18 (axis), wl = 1/36 (face diagonal). */
static double weight(int i)
{
    const double w0 = 1.0 / 3.0, ws = 1.0 / 18.0, wl = 1.0 / 36.0;
    if (i == 0) return w0;
    if ((i >= 1 && i <= 3) || (i >= 10 && i <= 12)) return ws;
    return wl;
}

static const double CS2 = 1.0 / 3.0; /* lattice sound speed squared, Sec. II.A */

/* Opposite direction: the swap-trick ordering pairs i with i+9. */
static int opposite(int i)
{
    if (i == 0) return 0;
    return i <= 9 ? i + 9 : i - 9;
}

void orc19_tables(int *c, double *w, int *opp)
{
    for (int i = 0; i < Q; ++i) {
        c[3 * i + 0] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}

/* Sec. II.A, eq. (EqQ19RM): extended D3Q19 equilibrium, written out term by
 * term exactly as printed (no factorisation). */
void orc19_feq(double rho, double ux, double uy, double uz, double *feq)
{
    const double x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
    feq[0] = rho / 3.0 * (1.0 - (x2 + y2 + z2) + 3.0 * (x2 * y2 + x2 * z2 + y2 * z2));
    feq[1] = rho / 18.0 * (1.0 - 3.0 * ux + 3.0 * (x2 - y2 - z2) + 9.0 * (ux * y2 + ux * z2) - 9.0 * (x2 * y2 + x2 * z2));
    feq[2] = rho / 18.0 * (1.0 - 3.0 * uy + 3.0 * (-x2 + y2 - z2) + 9.0 * (x2 * uy + uy * z2) - 9.0 * (x2 * y2 + y2 * z2));
    feq[3] = rho / 18.0 * (1.0 - 3.0 * uz + 3.0 * (-x2 - y2 + z2) + 9.0 * (x2 * uz + y2 * uz) - 9.0 * (x2 * z2 + y2 * z2));
    feq[4] = rho / 36.0 * (1.0 - 3.0 * (ux + uy) + 3.0 * (x2 + y2) + 9.0 * ux * uy - 9.0 * (x2 * uy + ux * y2) + 9.0 * x2 * y2);
    feq[5] = rho / 36.0 * (1.0 + 3.0 * (-ux + uy) + 3.0 * (x2 + y2) - 9.0 * ux * uy + 9.0 * (x2 * uy - ux * y2) + 9.0 * x2 * y2);
    feq[6] = rho / 36.0 * (1.0 - 3.0 * (ux + uz) + 3.0 * (x2 + z2) + 9.0 * ux * uz - 9.0 * (x2 * uz + ux * z2) + 9.0 * x2 * z2);
    feq[7] = rho / 36.0 * (1.0 + 3.0 * (-ux + uz) + 3.0 * (x2 + z2) - 9.0 * ux * uz + 9.0 * (x2 * uz - ux * z2) + 9.0 * x2 * z2);
    feq[8] = rho / 36.0 * (1.0 - 3.0 * (uy + uz) + 3.0 * (y2 + z2) + 9.0 * uy * uz - 9.0 * (y2 * uz + uy * z2) + 9.0 * y2 * z2);
    feq[9] = rho / 36.0 * (1.0 + 3.0 * (-uy + uz) + 3.0 * (y2 + z2) - 9.0 * uy * uz + 9.0 * (y2 * uz - uy * z2) + 9.0 * y2 * z2);
    feq[10] = rho / 18.0 * (1.0 + 3.0 * ux + 3.0 * (x2 - y2 - z2) - 9.0 * (ux * y2 + ux * z2) - 9.0 * (x2 * y2 + x2 * z2));
    feq[11] = rho / 18.0 * (1.0 + 3.0 * uy + 3.0 * (-x2 + y2 - z2) - 9.0 * (x2 * uy + uy * z2) - 9.0 * (x2 * y2 + y2 * z2));
    feq[12] = rho / 18.0 * (1.0 + 3.0 * uz + 3.0 * (-x2 - y2 + z2) - 9.0 * (x2 * uz + y2 * uz) - 9.0 * (x2 * z2 + y2 * z2));
    feq[13] = rho / 36.0 * (1.0 + 3.0 * (ux + uy) + 3.0 * (x2 + y2) + 9.0 * ux * uy + 9.0 * (x2 * uy + ux * y2) + 9.0 * x2 * y2);
    feq[14] = rho / 36.0 * (1.0 + 3.0 * (ux - uy) + 3.0 * (x2 + y2) - 9.0 * ux * uy + 9.0 * (-x2 * uy + ux * y2) + 9.0 * x2 * y2);
    feq[15] = rho / 36.0 * (1.0 + 3.0 * (ux + uz) + 3.0 * (x2 + z2) + 9.0 * ux * uz + 9.0 * (x2 * uz + ux * z2) + 9.0 * x2 * z2);
    feq[16] = rho / 36.0 * (1.0 + 3.0 * (ux - uz) + 3.0 * (x2 + z2) - 9.0 * ux * uz + 9.0 * (-x2 * uz + ux * z2) + 9.0 * x2 * z2);
    feq[17] = rho / 36.0 * (1.0 + 3.0 * (uy + uz) + 3.0 * (y2 + z2) + 9.0 * uy * uz + 9.0 * (y2 * uz + uy * z2) + 9.0 * y2 * z2);
    feq[18] = rho / 36.0 * (1.0 + 3.0 * (uy - uz) + 3.0 * (y2 + z2) - 9.0 * uy * uz + 9.0 * (-y2 * uz + uy * z2) + 9.0 * y2 * z2);
}

/* Sec. II.B, eq. (matrix): row r of the transformation matrix T evaluated on
 * the shifted velocity (bx, by, bz) = c_i - u.  Row 18 per reading R1. */
static double t_row(int r, double bx, double by, double bz)
{
    switch (r) {
    case 0: return 1.0;
    case 1: return bx;
    case 2: return by;
    case 3: return bz;
    case 4: return bx * bx + by * by + bz * bz;
    case 5: return bx * bx - by * by;
    case 6: return by * by - bz * bz;
    case 7: return bx * by;
    case 8: return bx * bz;
    case 9: return by * bz;
    case 10: return bx * bx * by;
    case 11: return bx * by * by;
    case 12: return bx * bx * bz;
    case 13: return bx * bz * bz;
    case 14: return by * by * bz;
    case 15: return by * bz * bz;
    case 16: return bx * bx * by * by;
    case 17: return bx * bx * bz * bz;
    default: return by * by * bz * bz;
    }
}

/* T(u), row-major 19x19: T[r*19+i] = monomial r of (c_i - u). */
void orc19_T(double ux, double uy, double uz, double *T)
{
    for (int r = 0; r < Q; ++r)
        for (int i = 0; i < Q; ++i)
            T[r * Q + i] = t_row(r, CX[i] - ux, CY[i] - uy, CZ[i] - uz);
}

/* Sec. II.B: Galilean-invariant equilibrium CMs (k0 = rho, k4 = 3 rho cs^2,
 * k16..18 = rho cs^4, all others zero). */
void orc19_keq(double rho, double *keq)
{
    for (int r = 0; r < Q; ++r) keq[r] = 0.0;
    keq[0] = rho;
    keq[4] = 3.0 * rho * CS2;
    keq[16] = rho * CS2 * CS2;
    keq[17] = rho * CS2 * CS2;
    keq[18] = rho * CS2 * CS2;
}

/* App. B, eq. (CMQ19): central moments of the forcing term, placed in the row
 * order of T.  R_100,010,001 = F; R_210 = cs^2 Fy, R_120 = cs^2 Fx,
 * R_201 = cs^2 Fz, R_102 = cs^2 Fx, R_021 = cs^2 Fz, R_012 = cs^2 Fy; the
 * second-order and fourth-order ones vanish, so do rows 4..9 and 16..18. */
void orc19_Rcm(double Fx, double Fy, double Fz, double *R)
{
    for (int r = 0; r < Q; ++r) R[r] = 0.0;
    R[1] = Fx;
    R[2] = Fy;
    R[3] = Fz;
    R[10] = CS2 * Fy; /* cx^2 cy */
    R[11] = CS2 * Fx; /* cx cy^2 */
    R[12] = CS2 * Fz; /* cx^2 cz */
    R[13] = CS2 * Fx; /* cx cz^2 */
    R[14] = CS2 * Fz; /* cy^2 cz */
    R[15] = CS2 * Fy; /* cy cz^2 */
}

/* App. C: raw-moment matrix M = T(0), the un-shifted basis (N = I). */
void orc19_M(double *M) { orc19_T(0.0, 0.0, 0.0, M); }

/* App. C: equilibrium raw moments of the RM formulation, as printed there
 * (rows in the order of M). */
void orc19_keq_rm(double rho, double ux, double uy, double uz, double *k)
{
    const double x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
    k[0] = rho;
    k[1] = rho * ux;
    k[2] = rho * uy;
    k[3] = rho * uz;
    k[4] = rho * (3.0 * CS2 + x2 + y2 + z2);
    k[5] = rho * (x2 - y2);
    k[6] = rho * (y2 - z2);
    k[7] = rho * ux * uy;
    k[8] = rho * ux * uz;
    k[9] = rho * uy * uz;
    k[10] = rho * uy * (x2 + CS2);
    k[11] = rho * ux * (y2 + CS2);
    k[12] = rho * uz * (x2 + CS2);
    k[13] = rho * ux * (z2 + CS2);
    k[14] = rho * uz * (y2 + CS2);
    k[15] = rho * uy * (z2 + CS2);
    k[16] = rho * (x2 + CS2) * (y2 + CS2);
    k[17] = rho * (x2 + CS2) * (z2 + CS2);
    k[18] = rho * (y2 + CS2) * (z2 + CS2);
}

/* App. B, eq. (RMQ19): raw moments R_pqr of the forcing term, placed in the
 * row order of M (rows 4..6 are the trace and the two differences of the
 * second-order ones).  Reading R9. */
void orc19_Rrm(double ux, double uy, double uz, double Fx, double Fy, double Fz, double *R)
{
    const double r200 = 2.0 * ux * Fx, r020 = 2.0 * uy * Fy, r002 = 2.0 * uz * Fz;
    R[0] = 0.0;
    R[1] = Fx;
    R[2] = Fy;
    R[3] = Fz;
    R[4] = r200 + r020 + r002;
    R[5] = r200 - r020;
    R[6] = r020 - r002;
    R[7] = ux * Fy + uy * Fx;
    R[8] = ux * Fz + uz * Fx;
    R[9] = uy * Fz + uz * Fy;
    R[10] = CS2 * Fy + ux * (ux * Fy + 2.0 * uy * Fx); /* 210 */
    R[11] = CS2 * Fx + uy * (uy * Fx + 2.0 * ux * Fy); /* 120 */
    R[12] = CS2 * Fz + ux * (ux * Fz + 2.0 * uz * Fx); /* 201 */
    R[13] = CS2 * Fx + uz * (uz * Fx + 2.0 * ux * Fz); /* 102 */
    R[14] = CS2 * Fz + uy * (uy * Fz + 2.0 * uz * Fy); /* 021 */
    R[15] = CS2 * Fy + uz * (uz * Fy + 2.0 * uy * Fz); /* 012 */
    R[16] = 2.0 * (ux * uy * (ux * Fy + uy * Fx) + CS2 * (ux * Fx + uy * Fy));
    R[17] = 2.0 * (ux * uz * (ux * Fz + uz * Fx) + CS2 * (ux * Fx + uz * Fz));
    R[18] = 2.0 * (uy * uz * (uy * Fz + uz * Fy) + CS2 * (uy * Fy + uz * Fz));
}

/* Macroscopic moments, Sec. II.A eq. (macro) with the F/2 shift (reading R2). */
static void macro(const double *f, const double *F, double *rho, double *u)
{
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        jx += f[i] * CX[i];
        jy += f[i] * CY[i];
        jz += f[i] * CZ[i];
    }
    *rho = r;
    u[0] = (jx + 0.5 * F[0]) / r;
    u[1] = (jy + 0.5 * F[1]) / r;
    u[2] = (jz + 0.5 * F[2]) / r;
}

/* App. C, eq. (rawQ19): post-collision raw moments r* = N^-1 k*, with the
 * missing cs^2 factors restored (reading R3). */
void orc19_rstar(double rho, double ux, double uy, double uz, const double *k, double *r)
{
    const double x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
    r[0] = rho;
    r[1] = rho * ux + k[1];
    r[2] = rho * uy + k[2];
    r[3] = rho * uz + k[3];
    r[4] = rho * (x2 + y2 + z2) + 2.0 * ux * k[1] + 2.0 * uy * k[2] + 2.0 * uz * k[3] + k[4];
    r[5] = rho * (x2 - y2) + 2.0 * ux * k[1] - 2.0 * uy * k[2] + k[5];
    r[6] = rho * (y2 - z2) + 2.0 * uy * k[2] - 2.0 * uz * k[3] + k[6];
    r[7] = rho * ux * uy + uy * k[1] + ux * k[2] + k[7];
    r[8] = rho * ux * uz + uz * k[1] + ux * k[3] + k[8];
    r[9] = rho * uy * uz + uz * k[2] + uy * k[3] + k[9];
    r[10] = rho * x2 * uy + 2.0 * ux * uy * k[1] + x2 * k[2] + uy * k[4] * CS2 + 2.0 * uy * k[5] * CS2 +
            uy * k[6] * CS2 + 2.0 * ux * k[7] + k[10];
    r[11] = rho * ux * y2 + y2 * k[1] + 2.0 * ux * uy * k[2] + ux * k[4] * CS2 - ux * k[5] * CS2 +
            ux * k[6] * CS2 + 2.0 * uy * k[7] + k[11];
    r[12] = rho * x2 * uz + 2.0 * ux * uz * k[1] + x2 * k[3] + uz * k[4] * CS2 + 2.0 * uz * k[5] * CS2 +
            uz * k[6] * CS2 + 2.0 * ux * k[8] + k[12];
    r[13] = rho * ux * z2 + z2 * k[1] + 2.0 * ux * uz * k[3] + ux * k[4] * CS2 - ux * k[5] * CS2 -
            2.0 * ux * k[6] * CS2 + 2.0 * uz * k[8] + k[13];
    r[14] = rho * y2 * uz + 2.0 * uy * uz * k[2] + y2 * k[3] + uz * k[4] * CS2 - uz * k[5] * CS2 +
            uz * k[6] * CS2 + 2.0 * uy * k[9] + k[14];
    r[15] = rho * uy * z2 + z2 * k[2] + 2.0 * uy * uz * k[3] + uy * k[4] * CS2 - uy * k[5] * CS2 -
            2.0 * uy * k[6] * CS2 + 2.0 * uz * k[9] + k[15];
    r[16] = rho * x2 * y2 + 2.0 * ux * y2 * k[1] + 2.0 * x2 * uy * k[2] + (x2 + y2) * k[4] * CS2 +
            (2.0 * y2 - x2) * k[5] * CS2 + (x2 + y2) * k[6] * CS2 + 4.0 * ux * uy * k[7] +
            2.0 * uy * k[10] + 2.0 * ux * k[11] + k[16];
    r[17] = rho * x2 * z2 + 2.0 * ux * z2 * k[1] + 2.0 * x2 * uz * k[3] + (x2 + z2) * k[4] * CS2 +
            (2.0 * z2 - x2) * k[5] * CS2 + (z2 - 2.0 * x2) * k[6] * CS2 + 4.0 * ux * uz * k[8] +
            2.0 * uz * k[12] + 2.0 * ux * k[13] + k[17];
    r[18] = rho * y2 * z2 + 2.0 * uy * z2 * k[2] + 2.0 * y2 * uz * k[3] + (y2 + z2) * k[4] * CS2 +
            (-y2 - z2) * k[5] * CS2 + (z2 - 2.0 * y2) * k[6] * CS2 + 4.0 * uy * uz * k[9] +
            2.0 * uz * k[14] + 2.0 * uy * k[15] + k[18];
}

/* App. C, eq. (pdfQ19): populations f* = M^-1 r*, with reading R4 on f3, f12. */
void orc19_fstar(const double *r, double *f)
{
    f[0] = r[0] - r[4] + r[16] + r[17] + r[18];
    f[1] = (r[11] + r[13] - r[1] - r[16] - r[17]) / 2.0 + (r[4] + 2.0 * r[5] + r[6]) * CS2 / 2.0;
    f[2] = (r[10] + r[15] - r[2] - r[16] - r[18]) / 2.0 + (r[4] + r[6] - r[5]) * CS2 / 2.0;
    f[3] = (r[12] + r[14] - r[3] - r[17] - r[18]) / 2.0 + (r[4] - r[5] - 2.0 * r[6]) * CS2 / 2.0;
    f[4] = (r[7] + r[16] - r[10] - r[11]) / 4.0;
    f[5] = (r[10] + r[16] - r[7] - r[11]) / 4.0;
    f[6] = (r[8] + r[17] - r[12] - r[13]) / 4.0;
    f[7] = (r[12] + r[17] - r[8] - r[13]) / 4.0;
    f[8] = (r[9] + r[18] - r[14] - r[15]) / 4.0;
    f[9] = (r[14] + r[18] - r[9] - r[15]) / 4.0;
    f[10] = (r[1] - r[11] - r[13] - r[16] - r[17]) / 2.0 + (r[4] + 2.0 * r[5] + r[6]) * CS2 / 2.0;
    f[11] = (r[2] - r[10] - r[15] - r[16] - r[18]) / 2.0 + (r[4] + r[6] - r[5]) * CS2 / 2.0;
    f[12] = (r[3] - r[12] - r[14] - r[17] - r[18]) / 2.0 + (r[4] - r[5] - 2.0 * r[6]) * CS2 / 2.0;
    f[13] = (r[7] + r[10] + r[11] + r[16]) / 4.0;
    f[14] = (r[11] + r[16] - r[7] - r[10]) / 4.0;
    f[15] = (r[8] + r[12] + r[13] + r[17]) / 4.0;
    f[16] = (r[13] + r[17] - r[8] - r[12]) / 4.0;
    f[17] = (r[9] + r[14] + r[15] + r[18]) / 4.0;
    f[18] = (r[15] + r[18] - r[9] - r[14]) / 4.0;
}

/* Dense solve A x = b (19x19) by Gaussian elimination with partial pivoting.
 * A and b are overwritten.  Returns 0 on success, -1 if A is singular. */
static int solve19(double *A, double *b, double *x)
{
    for (int col = 0; col < Q; ++col) {
        int piv = col;
        double best = fabs(A[col * Q + col]);
        for (int r = col + 1; r < Q; ++r) {
            double v = fabs(A[r * Q + col]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return -1;
        if (piv != col) {
            for (int c = 0; c < Q; ++c) {
                double t = A[col * Q + c];
                A[col * Q + c] = A[piv * Q + c];
                A[piv * Q + c] = t;
            }
            double t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        for (int r = col + 1; r < Q; ++r) {
            double m = A[r * Q + col] / A[col * Q + col];
            if (m == 0.0) continue;
            for (int c = col; c < Q; ++c) A[r * Q + c] -= m * A[col * Q + c];
            b[r] -= m * b[col];
        }
    }
    for (int r = Q - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < Q; ++c) s -= A[r * Q + c] * x[c];
        x[r] = s / A[r * Q + r];
    }
    return 0;
}

/* The same elimination for the other oracle files (n <= 19; A, b overwritten). */
int orc_solve19(double *A, double *b, double *x) { return solve19(A, b, x); }

enum { ORC_DEFINITION = 0, ORC_CLOSED_FORM = 1, ORC_RM_DEFINITION = 2, ORC_RM_CLOSED_FORM = 3 };

/*
 * One collision at one node, Sec. II.B eqs. (posColl0) and (system):
 *   rho, u from f (reading R2); k = T(u) f; k_eq; R = CMs of the force;
 *   k* = (I - K) k + K k_eq + (I - K/2) R;
 *   f* = T(u)^-1 k*   (mode ORC_DEFINITION: dense solve)
 *      = M^-1 N^-1 k* (mode ORC_CLOSED_FORM: App. C two-step closed forms).
 * Modes ORC_RM_*: the raw-moment variant of App. C (N = I, T = M): k = M f,
 * the raw equilibrium and forcing moments (reading R9), the same relaxation,
 * f* = M^-1 k* by a dense solve (ORC_RM_DEFINITION) or by the closed forms
 * of eq. (pdfQ19) with r* = k* (ORC_RM_CLOSED_FORM).
 * K holds the 19 diagonal entries of the relaxation matrix.  If kout/uout are
 * given they receive k (pre-collision moments) and the shifted velocity.
 */
int orc19_collide(const double *f, const double *F, const double *K, int mode, double *fstar,
                  double *kout, double *rho_out, double *uout)
{
    double rho, u[3];
    macro(f, F, &rho, u);
    const int raw = (mode == ORC_RM_DEFINITION || mode == ORC_RM_CLOSED_FORM);
    double T[Q * Q], k[Q], keq[Q], R[Q], ks[Q];
    if (raw)
        orc19_M(T);
    else
        orc19_T(u[0], u[1], u[2], T);
    for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += T[r * Q + i] * f[i];
        k[r] = s;
    }
    if (raw) {
        orc19_keq_rm(rho, u[0], u[1], u[2], keq);
        orc19_Rrm(u[0], u[1], u[2], F[0], F[1], F[2], R);
    } else {
        orc19_keq(rho, keq);
        orc19_Rcm(F[0], F[1], F[2], R);
    }
    for (int r = 0; r < Q; ++r) ks[r] = (1.0 - K[r]) * k[r] + K[r] * keq[r] + (1.0 - 0.5 * K[r]) * R[r];
    if (kout) memcpy(kout, k, sizeof k);
    if (rho_out) *rho_out = rho;
    if (uout) memcpy(uout, u, sizeof u);
    if (mode == ORC_DEFINITION || mode == ORC_RM_DEFINITION) {
        double b[Q];
        memcpy(b, ks, sizeof ks);
        return solve19(T, b, fstar);
    }
    if (mode == ORC_RM_CLOSED_FORM) {
        orc19_fstar(ks, fstar);
        return 0;
    }
    double rs[Q];
    /* The closed forms of App. C take k0* = rho. */
    orc19_rstar(ks[0], u[0], u[1], u[2], ks, rs);
    orc19_fstar(rs, fstar);
    return 0;
}

/* Standard K of Sec. II.B: diag(1,1,1,1, w_b, w x5, w_hi[0..8]). */
void orc19_K(double omega, double omega_bulk, const double *omega_hi, double *K)
{
    for (int r = 0; r < 4; ++r) K[r] = 1.0;
    K[4] = omega_bulk;
    for (int r = 5; r < 10; ++r) K[r] = omega;
    for (int r = 10; r < Q; ++r) K[r] = omega_hi ? omega_hi[r - 10] : 1.0;
}

static inline int64_t node(int x, int y, int z, int nx, int ny) { return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z); }
static inline int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

/*
 * One full time step on an nx*ny*nz lattice: collision at every node (the
 * function above), then streaming f_i(x + c_i, t+1) = f_i*(x, t) (eq.
 * "streaming_f") with periodic wrap in x and z; y is periodic too unless
 * walls_y != 0, in which case walls sit half a link outside y = 0 and
 * y = ny-1 and a population that would cross one returns to its node in the
 * opposite direction (halfway bounce-back, stationary walls).
 *
 * F: 3*N force density or NULL (no force).  Krates: 19 entries (same K at
 * every node) or, if per_node_K != 0, 19*N entries Krates[r*N + n].
 * Returns 0, or -1 if a collision system was singular.
 */
int orc19_step(int nx, int ny, int nz, int walls_y, const double *f, double *fnew, const double *F,
               const double *Krates, int per_node_K, int mode)
{
    const int64_t N = (int64_t)nx * ny * nz;
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int64_t n = 0; n < N; ++n) {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        double fl[Q], fs[Q], Fl[3] = {0.0, 0.0, 0.0}, Kl[Q];
        for (int i = 0; i < Q; ++i) fl[i] = f[(int64_t)i * N + n];
        if (F)
            for (int d = 0; d < 3; ++d) Fl[d] = F[(int64_t)d * N + n];
        for (int r = 0; r < Q; ++r) Kl[r] = per_node_K ? Krates[(int64_t)r * N + n] : Krates[r];
        if (orc19_collide(fl, Fl, Kl, mode, fs, NULL, NULL, NULL) != 0) err |= 1;
        for (int i = 0; i < Q; ++i) {
            int yd = y + CY[i];
            if (walls_y && (yd < 0 || yd >= ny)) {
                fnew[(int64_t)opposite(i) * N + n] = fs[i];
                continue;
            }
            const int xd = wrap(x + CX[i], nx), zd = wrap(z + CZ[i], nz);
            yd = wrap(yd, ny);
            fnew[(int64_t)i * N + node(xd, yd, zd, nx, ny)] = fs[i];
        }
    }
    return err ? -1 : 0;
}

/* Initialisation at equilibrium from the macroscopic fields (Sec. III:
 * populations start at the equilibrium of the initial fields). */
void orc19_init(int nx, int ny, int nz, const double *rho, const double *u, double *f)
{
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double fe[Q];
        orc19_feq(rho[n], u[n], u[N + n], u[2 * N + n], fe);
        for (int i = 0; i < Q; ++i) f[(int64_t)i * N + n] = fe[i];
    }
}

/* Density and force-shifted velocity at every node (eq. "macro", reading R2). */
void orc19_moments(int nx, int ny, int nz, const double *f, const double *F, double *rho, double *u)
{
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double fl[Q], Fl[3] = {0.0, 0.0, 0.0}, r, ul[3];
        for (int i = 0; i < Q; ++i) fl[i] = f[(int64_t)i * N + n];
        if (F)
            for (int d = 0; d < 3; ++d) Fl[d] = F[(int64_t)d * N + n];
        macro(fl, Fl, &r, ul);
        rho[n] = r;
        for (int d = 0; d < 3; ++d) u[(int64_t)d * N + n] = ul[d];
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * f_i(x, t+1) at selected nodes only, from the full state f at time t: by the
 * streaming rule f_i(x, t+1) = f*_i(x - c_i, t), or f*_opp(i)(x, t) when
 * x - c_i lies beyond a y wall; each f* from one collision (the function
 * above) at the node it comes from.  out[s*19 + i] for sample s.  Lets a test
 * check single outputs of a lattice too large for a full oracle step.
 */
int orc19_step_at(int nx, int ny, int nz, int walls_y, const double *f, const double *F, const double *Krates,
                  int per_node_K, int mode, const int64_t *nodes, int nsample, double *out)
{
    const int64_t N = (int64_t)nx * ny * nz;
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int s = 0; s < nsample; ++s) {
        const int64_t n = nodes[s];
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        for (int i = 0; i < Q; ++i) {
            int src_x = x, src_y = y, src_z = z, comp = i;
            const int ys = y - CY[i];
            if (walls_y && (ys < 0 || ys >= ny)) {
                comp = opposite(i);
            } else {
                src_x = wrap(x - CX[i], nx);
                src_y = wrap(ys, ny);
                src_z = wrap(z - CZ[i], nz);
            }
            const int64_t m = node(src_x, src_y, src_z, nx, ny);
            double fl[Q], fs[Q], Fl[3] = {0.0, 0.0, 0.0}, Kl[Q];
            for (int j = 0; j < Q; ++j) fl[j] = f[(int64_t)j * N + m];
            if (F)
                for (int d = 0; d < 3; ++d) Fl[d] = F[(int64_t)d * N + m];
            for (int r = 0; r < Q; ++r) Kl[r] = per_node_K ? Krates[(int64_t)r * N + m] : Krates[r];
            if (orc19_collide(fl, Fl, Kl, mode, fs, NULL, NULL, NULL) != 0) err |= 1;
            out[(int64_t)s * Q + i] = fs[comp];
        }
    }
    return err ? -1 : 0;
}
