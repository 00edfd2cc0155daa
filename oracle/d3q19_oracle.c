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
 *   R3  App. C prints the back-transform as closed forms (raw moments
 *       r* = N^-1 k*, eq. "rawQ19"; populations f* = M^-1 r*, eq. "pdfQ19"),
 *       three of whose rows lack a cs^2 factor and two of whose population
 *       formulas are misprinted.  This oracle uses none of the printed closed
 *       forms: it solves T(u) f* = k* with T(u) built from its definition,
 *       so those misprints cannot reach it.
 *   R5  K = diag(1,1,1,1, w_b, w,w,w,w,w, w_hi(9)); the paper sets w_b = 1 and
 *       w_hi = 1 (Sec. II.B).  w_b and w_hi are kept as free inputs so that the
 *       learned-rate variant and the bulk-rate tests can use them.
 *   R6  F is a force density (eq. "lbe" and the Rayleigh-Taylor body force).
 *   R9  Raw-moment variant (App. C, N = I): its printed post-collision list
 *       carries only the forcing terms of the CM scheme (F/2 on rows 1-3,
 *       cs^2 F/2 on rows 10-15).  The relaxation eq. (posColl0) with T = M
 *       needs the raw moments of the same equilibrium and forcing term, which
 *       are computed here from their definition, M f_eq and M T(u)^-1 R^CM
 *       (App. B prints the latter as eq. RMQ19).  With F = 0 both readings
 *       agree, and at K = I the variant equals the CM scheme.
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

/* Sec. II.B, eq. (matrix): the 19 rows of the transformation matrix T
 * evaluated on one shifted velocity (bx, by, bz) = c_i - u, i.e. column i of
 * T(u).  Row 18 per reading R1. */
static void t_column(double bx, double by, double bz, double *t)
{
    t[0] = 1.0;
    t[1] = bx;
    t[2] = by;
    t[3] = bz;
    t[4] = bx * bx + by * by + bz * bz;
    t[5] = bx * bx - by * by;
    t[6] = by * by - bz * bz;
    t[7] = bx * by;
    t[8] = bx * bz;
    t[9] = by * bz;
    t[10] = bx * bx * by;
    t[11] = bx * by * by;
    t[12] = bx * bx * bz;
    t[13] = bx * bz * bz;
    t[14] = by * by * bz;
    t[15] = by * bz * bz;
    t[16] = bx * bx * by * by;
    t[17] = bx * bx * bz * bz;
    t[18] = by * by * bz * bz;
}

/* T(u), row-major 19x19: T[r*19+i] = monomial r of (c_i - u). */
void orc19_T(double ux, double uy, double uz, double *T)
{
    for (int i = 0; i < Q; ++i) {
        double t[Q];
        t_column(CX[i] - ux, CY[i] - uy, CZ[i] - uz, t);
        for (int r = 0; r < Q; ++r) T[r * Q + i] = t[r];
    }
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
        const double inv_pivot = 1.0 / A[col * Q + col];
        for (int r = col + 1; r < Q; ++r) {
            double m = A[r * Q + col] * inv_pivot;
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

/* Sec. II.A-B: the extended D3Q19 equilibrium (eq. EqQ19RM) is the
 * population set whose central moments are the Galilean-invariant k_eq:
 * f_eq = T(u)^-1 k_eq (the paper states both forms; the CM one is used). */
void orc19_feq(double rho, double ux, double uy, double uz, double *feq)
{
    double T[Q * Q], k[Q];
    orc19_T(ux, uy, uz, T);
    orc19_keq(rho, k);
    solve19(T, k, feq);
}

/* App. C: raw moments (rows of M) of the same equilibrium, M f_eq, the
 * equilibrium of the raw-moment variant. */
void orc19_keq_rm(double rho, double ux, double uy, double uz, double *k)
{
    double M[Q * Q], fe[Q];
    orc19_M(M);
    orc19_feq(rho, ux, uy, uz, fe);
    for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += M[r * Q + i] * fe[i];
        k[r] = s;
    }
}

/* App. B (eq. RMQ19 prints the result): raw moments of the forcing term whose
 * central moments are R^CM, i.e. M T(u)^-1 R^CM (reading R9). */
void orc19_Rrm(double ux, double uy, double uz, double Fx, double Fy, double Fz, double *R)
{
    double T[Q * Q], M[Q * Q], Rc[Q], Fi[Q];
    orc19_T(ux, uy, uz, T);
    orc19_Rcm(Fx, Fy, Fz, Rc);
    solve19(T, Rc, Fi);
    orc19_M(M);
    for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += M[r * Q + i] * Fi[i];
        R[r] = s;
    }
}

enum { ORC_DEFINITION = 0, ORC_RM_DEFINITION = 2 };

/*
 * One collision at one node, Sec. II.B eqs. (posColl0) and (system):
 *   rho, u from f (reading R2); k = T(u) f; k_eq; R = CMs of the force;
 *   k* = (I - K) k + K k_eq + (I - K/2) R;
 *   f* = T(u)^-1 k*   (mode ORC_DEFINITION: dense solve of T(u) f* = k*).
 * Mode ORC_RM_DEFINITION: the raw-moment variant of App. C (N = I, T = M):
 * k = M f, the raw moments of the same equilibrium and forcing term (reading
 * R9), the same relaxation, f* = M^-1 k* by a dense solve.  Any other mode
 * returns -2.
 * K holds the 19 diagonal entries of the relaxation matrix.  If kout/uout are
 * given they receive k (pre-collision moments) and the shifted velocity.
 */
int orc19_collide(const double *f, const double *F, const double *K, int mode, double *fstar,
                  double *kout, double *rho_out, double *uout)
{
    double rho, u[3];
    macro(f, F, &rho, u);
    if (mode != ORC_DEFINITION && mode != ORC_RM_DEFINITION) return -2;
    const int raw = mode == ORC_RM_DEFINITION;
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
    double b[Q];
    memcpy(b, ks, sizeof ks);
    return solve19(T, b, fstar);
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
