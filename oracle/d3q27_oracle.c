/*
 * D3Q27 central-moment LBM -- plain FP64 CPU oracle (test infrastructure only;
 * see d3q19_oracle.c for the rules that apply to this directory).
 *
 * Paper: App. D (velocity set, CM basis T = N M, population formulas of M^-1).
 * The paper does not print the D3Q27 equilibrium, K, k* or R (it defers them
 * to the authors' earlier D3Q27 work).  Readings taken here:
 *   Q1  equilibrium: tensor product of the D1Q3 equilibrium per axis,
 *       phi(0,u) = 2/3 - u^2, phi(+-1,u) = (u^2 + 1/3 +- u)/2, f_eq = rho
 *       phi(cx,ux) phi(cy,uy) phi(cz,uz); its central moments are
 *       rho (1/3)^(number of squared axes) when no exponent is 1, else 0.
 *   Q2  K: omega on the five deviatoric second-order rows (4..8: xy, xz, yz,
 *       x^2-y^2, x^2-z^2), 1 on every other row (bulk and higher orders are
 *       equilibrated, as in the D3Q19 scheme of Sec. II.B).
 *   Q3  forcing CMs by the Gaussian (Hermite) rule
 *       R_pqr = sum_a p_a F_a k^eq_{pqr - e_a} / rho, which reproduces the
 *       D3Q19 list of App. B eq. (CMQ19) on the shared monomials.
 *   Q4  force-shifted velocity and halfway bounce-back, as for D3Q19.
 *   Q6  raw-moment variant (timed in App. D, not written out): N = I, i.e.
 *       T = T(0) = M; k_eq and R are the raw moments of the same equilibrium
 *       and forcing term, rho mu_p(ux) mu_q(uy) mu_r(uz) with
 *       mu = (1, u, u^2 + 1/3) and R_pqr = sum_a p_a F_a (raw eq moment with
 *       p_a lowered by one)/rho; the same K.
 * f* = T(u)^-1 k* by a dense solve per node (N^-1 is not printed).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define Q27 27

/* App. D velocity order (swap trick: opposite(i) = i +- 13). */
static const int CX[Q27] = {0, -1, 0, 0, -1, -1, -1, -1, 0, 0, -1, -1, -1, -1, 1, 0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1};
static const int CY[Q27] = {0, 0, -1, 0, -1, 1, 0, 0, -1, -1, -1, -1, 1, 1, 0, 1, 0, 1, -1, 0, 0, 1, 1, 1, 1, -1, -1};
static const int CZ[Q27] = {0, 0, 0, -1, 0, 0, -1, 1, -1, 1, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};

static int opposite27(int i) { return i == 0 ? 0 : (i <= 13 ? i + 13 : i - 13); }

/* D1Q3 weights 2/3, 1/6; D3Q27 weight = product. */
static double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }

void orc27_tables(int *c, double *w, int *opp)
{
    for (int i = 0; i < Q27; ++i) {
        c[3 * i] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
        w[i] = w1(CX[i]) * w1(CY[i]) * w1(CZ[i]);
        opp[i] = opposite27(i);
    }
}

/* Reading Q1. */
static double phi(int c, double u)
{
    if (c == 0) return 2.0 / 3.0 - u * u;
    return 0.5 * (u * u + 1.0 / 3.0 + c * u);
}

void orc27_feq(double rho, double ux, double uy, double uz, double *feq)
{
    for (int i = 0; i < Q27; ++i) feq[i] = rho * phi(CX[i], ux) * phi(CY[i], uy) * phi(CZ[i], uz);
}

/* App. D basis row r on shifted velocity (a, b, c) = c_i - u. */
static double t27_row(int r, double a, double b, double c)
{
    const double a2 = a * a, b2 = b * b, c2 = c * c;
    switch (r) {
    case 0: return 1.0;
    case 1: return a;
    case 2: return b;
    case 3: return c;
    case 4: return a * b;
    case 5: return a * c;
    case 6: return b * c;
    case 7: return a2 - b2;
    case 8: return a2 - c2;
    case 9: return a2 + b2 + c2;
    case 10: return a * b2 + a * c2;
    case 11: return a2 * b + b * c2;
    case 12: return a2 * c + b2 * c;
    case 13: return a * b2 - a * c2;
    case 14: return a2 * b - b * c2;
    case 15: return a2 * c - b2 * c;
    case 16: return a * b * c;
    case 17: return a2 * b2 + a2 * c2 + b2 * c2;
    case 18: return a2 * b2 + a2 * c2 - b2 * c2;
    case 19: return a2 * b2 - a2 * c2;
    case 20: return a2 * b * c;
    case 21: return a * b2 * c;
    case 22: return a * b * c2;
    case 23: return a * b2 * c2;
    case 24: return a2 * b * c2;
    case 25: return a2 * b2 * c;
    default: return a2 * b2 * c2;
    }
}

void orc27_T(double ux, double uy, double uz, double *T)
{
    for (int r = 0; r < Q27; ++r)
        for (int i = 0; i < Q27; ++i) T[r * Q27 + i] = t27_row(r, CX[i] - ux, CY[i] - uy, CZ[i] - uz);
}

/* Monomial exponents (p,q,r) <= 2 of the basis rows, as linear combinations:
 * row value = sum_k coef[k] * monomial(exps[k]).  Used for k_eq and R. */
typedef struct { int n; int e[3][3]; double coef[3]; } row_def;

static row_def row_monomials(int r)
{
    row_def d;
    memset(&d, 0, sizeof d);
#define M1(p, q, s) do { d.n = 1; d.e[0][0] = p; d.e[0][1] = q; d.e[0][2] = s; d.coef[0] = 1.0; } while (0)
#define M2(p1, q1, s1, c1, p2, q2, s2, c2) do { d.n = 2; d.e[0][0] = p1; d.e[0][1] = q1; d.e[0][2] = s1; d.coef[0] = c1; \
        d.e[1][0] = p2; d.e[1][1] = q2; d.e[1][2] = s2; d.coef[1] = c2; } while (0)
    switch (r) {
    case 0: M1(0, 0, 0); break;
    case 1: M1(1, 0, 0); break;
    case 2: M1(0, 1, 0); break;
    case 3: M1(0, 0, 1); break;
    case 4: M1(1, 1, 0); break;
    case 5: M1(1, 0, 1); break;
    case 6: M1(0, 1, 1); break;
    case 7: M2(2, 0, 0, 1, 0, 2, 0, -1); break;
    case 8: M2(2, 0, 0, 1, 0, 0, 2, -1); break;
    case 9: d.n = 3; d.e[0][0] = 2; d.e[1][1] = 2; d.e[2][2] = 2; d.coef[0] = d.coef[1] = d.coef[2] = 1; break;
    case 10: M2(1, 2, 0, 1, 1, 0, 2, 1); break;
    case 11: M2(2, 1, 0, 1, 0, 1, 2, 1); break;
    case 12: M2(2, 0, 1, 1, 0, 2, 1, 1); break;
    case 13: M2(1, 2, 0, 1, 1, 0, 2, -1); break;
    case 14: M2(2, 1, 0, 1, 0, 1, 2, -1); break;
    case 15: M2(2, 0, 1, 1, 0, 2, 1, -1); break;
    case 16: M1(1, 1, 1); break;
    case 17: d.n = 3; d.e[0][0] = 2; d.e[0][1] = 2; d.e[1][0] = 2; d.e[1][2] = 2; d.e[2][1] = 2; d.e[2][2] = 2;
        d.coef[0] = d.coef[1] = d.coef[2] = 1; break;
    case 18: d.n = 3; d.e[0][0] = 2; d.e[0][1] = 2; d.e[1][0] = 2; d.e[1][2] = 2; d.e[2][1] = 2; d.e[2][2] = 2;
        d.coef[0] = d.coef[1] = 1; d.coef[2] = -1; break;
    case 19: M2(2, 2, 0, 1, 2, 0, 2, -1); break;
    case 20: M1(2, 1, 1); break;
    case 21: M1(1, 2, 1); break;
    case 22: M1(1, 1, 2); break;
    case 23: M1(1, 2, 2); break;
    case 24: M1(2, 1, 2); break;
    case 25: M1(2, 2, 1); break;
    default: M1(2, 2, 2); break;
    }
#undef M1
#undef M2
    return d;
}

/* central moment of the Q1 equilibrium divided by rho, per monomial */
static double g1(int p) { return p == 0 ? 1.0 : (p == 1 ? 0.0 : 1.0 / 3.0); }
static double keq_mono(int p, int q, int s) { return g1(p) * g1(q) * g1(s); }

void orc27_keq(double rho, double *keq)
{
    for (int r = 0; r < Q27; ++r) {
        row_def d = row_monomials(r);
        double v = 0.0;
        for (int k = 0; k < d.n; ++k) v += d.coef[k] * keq_mono(d.e[k][0], d.e[k][1], d.e[k][2]);
        keq[r] = rho * v;
    }
}

/* Reading Q3. */
static double rcm_mono(int p, int q, int s, double Fx, double Fy, double Fz)
{
    double v = 0.0;
    if (p > 0) v += p * Fx * keq_mono(p - 1, q, s);
    if (q > 0) v += q * Fy * keq_mono(p, q - 1, s);
    if (s > 0) v += s * Fz * keq_mono(p, q, s - 1);
    return v;
}

void orc27_Rcm(double Fx, double Fy, double Fz, double *R)
{
    for (int r = 0; r < Q27; ++r) {
        row_def d = row_monomials(r);
        double v = 0.0;
        for (int k = 0; k < d.n; ++k) v += d.coef[k] * rcm_mono(d.e[k][0], d.e[k][1], d.e[k][2], Fx, Fy, Fz);
        R[r] = v;
    }
}

/* Reading Q6: raw moments of the Q1 equilibrium over rho, per monomial. */
static double mu1(int p, double u) { return p == 0 ? 1.0 : (p == 1 ? u : u * u + 1.0 / 3.0); }
static double keq_raw_mono(int p, int q, int s, double ux, double uy, double uz)
{
    return mu1(p, ux) * mu1(q, uy) * mu1(s, uz);
}

void orc27_keq_rm(double rho, double ux, double uy, double uz, double *keq)
{
    for (int r = 0; r < Q27; ++r) {
        row_def d = row_monomials(r);
        double v = 0.0;
        for (int k = 0; k < d.n; ++k) v += d.coef[k] * keq_raw_mono(d.e[k][0], d.e[k][1], d.e[k][2], ux, uy, uz);
        keq[r] = rho * v;
    }
}

/* Reading Q6: Gaussian rule on the raw equilibrium moments. */
static double rrm_mono(int p, int q, int s, double ux, double uy, double uz, double Fx, double Fy, double Fz)
{
    double v = 0.0;
    if (p > 0) v += p * Fx * keq_raw_mono(p - 1, q, s, ux, uy, uz);
    if (q > 0) v += q * Fy * keq_raw_mono(p, q - 1, s, ux, uy, uz);
    if (s > 0) v += s * Fz * keq_raw_mono(p, q, s - 1, ux, uy, uz);
    return v;
}

void orc27_Rrm(double ux, double uy, double uz, double Fx, double Fy, double Fz, double *R)
{
    for (int r = 0; r < Q27; ++r) {
        row_def d = row_monomials(r);
        double v = 0.0;
        for (int k = 0; k < d.n; ++k) v += d.coef[k] * rrm_mono(d.e[k][0], d.e[k][1], d.e[k][2], ux, uy, uz, Fx, Fy, Fz);
        R[r] = v;
    }
}

/* Reading Q2. */
void orc27_K(double omega, double *K)
{
    for (int r = 0; r < Q27; ++r) K[r] = (r >= 4 && r <= 8) ? omega : 1.0;
}

static int solve27(double *A, double *b, double *x)
{
    const int n = Q27;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        double best = fabs(A[col * n + col]);
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > best) { best = fabs(A[r * n + col]); piv = r; }
        if (best == 0.0) return -1;
        if (piv != col) {
            for (int c = 0; c < n; ++c) { double t = A[col * n + c]; A[col * n + c] = A[piv * n + c]; A[piv * n + c] = t; }
            double t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            const double m = A[r * n + col] / A[col * n + col];
            if (m == 0.0) continue;
            for (int c = col; c < n; ++c) A[r * n + c] -= m * A[col * n + c];
            b[r] -= m * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < n; ++c) s -= A[r * n + c] * x[c];
        x[r] = s / A[r * n + r];
    }
    return 0;
}

/* One D3Q27 collision: k = T(u) f, k* = (I-K)k + K k_eq + (I-K/2) R, f* = T^-1 k*;
 * raw != 0: the raw-moment variant (reading Q6), T = T(0). */
int orc27_collide_mode(const double *f, const double *F, const double *K, int raw, double *fstar, double *rho_out,
                       double *uout)
{
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int i = 0; i < Q27; ++i) {
        rho += f[i];
        jx += f[i] * CX[i];
        jy += f[i] * CY[i];
        jz += f[i] * CZ[i];
    }
    const double ux = (jx + 0.5 * F[0]) / rho, uy = (jy + 0.5 * F[1]) / rho, uz = (jz + 0.5 * F[2]) / rho;
    double T[Q27 * Q27], k[Q27], keq[Q27], R[Q27], ks[Q27];
    if (raw)
        orc27_T(0.0, 0.0, 0.0, T);
    else
        orc27_T(ux, uy, uz, T);
    for (int r = 0; r < Q27; ++r) {
        double s = 0.0;
        for (int i = 0; i < Q27; ++i) s += T[r * Q27 + i] * f[i];
        k[r] = s;
    }
    if (raw) {
        orc27_keq_rm(rho, ux, uy, uz, keq);
        orc27_Rrm(ux, uy, uz, F[0], F[1], F[2], R);
    } else {
        orc27_keq(rho, keq);
        orc27_Rcm(F[0], F[1], F[2], R);
    }
    for (int r = 0; r < Q27; ++r) ks[r] = (1.0 - K[r]) * k[r] + K[r] * keq[r] + (1.0 - 0.5 * K[r]) * R[r];
    if (rho_out) *rho_out = rho;
    if (uout) { uout[0] = ux; uout[1] = uy; uout[2] = uz; }
    return solve27(T, ks, fstar);
}

int orc27_collide(const double *f, const double *F, const double *K, double *fstar, double *rho_out, double *uout)
{
    return orc27_collide_mode(f, F, K, 0, fstar, rho_out, uout);
}

static inline int64_t node27(int x, int y, int z, int nx, int ny) { return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z); }
static inline int wrap27(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

/* Full step with streaming (periodic, or halfway bounce-back walls in y);
 * raw selects the raw-moment variant. */
int orc27_step_mode(int nx, int ny, int nz, int walls_y, const double *f, double *fnew, const double *F,
                    const double *K, int raw)
{
    const int64_t N = (int64_t)nx * ny * nz;
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int64_t n = 0; n < N; ++n) {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        double fl[Q27], fs[Q27], Fl[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q27; ++i) fl[i] = f[(int64_t)i * N + n];
        if (F)
            for (int d = 0; d < 3; ++d) Fl[d] = F[(int64_t)d * N + n];
        if (orc27_collide_mode(fl, Fl, K, raw, fs, NULL, NULL) != 0) err |= 1;
        for (int i = 0; i < Q27; ++i) {
            int yd = y + CY[i];
            if (walls_y && (yd < 0 || yd >= ny)) {
                fnew[(int64_t)opposite27(i) * N + n] = fs[i];
                continue;
            }
            fnew[(int64_t)i * N + node27(wrap27(x + CX[i], nx), wrap27(yd, ny), wrap27(z + CZ[i], nz), nx, ny)] = fs[i];
        }
    }
    return err ? -1 : 0;
}

int orc27_step(int nx, int ny, int nz, int walls_y, const double *f, double *fnew, const double *F, const double *K)
{
    return orc27_step_mode(nx, ny, nz, walls_y, f, fnew, F, K, 0);
}

void orc27_init(int nx, int ny, int nz, const double *rho, const double *u, double *f)
{
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double fe[Q27];
        orc27_feq(rho[n], u[n], u[N + n], u[2 * N + n], fe);
        for (int i = 0; i < Q27; ++i) f[(int64_t)i * N + n] = fe[i];
    }
}

void orc27_moments(int nx, int ny, int nz, const double *f, const double *F, double *rho, double *u)
{
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q27; ++i) {
            const double v = f[(int64_t)i * N + n];
            r += v;
            j[0] += v * CX[i];
            j[1] += v * CY[i];
            j[2] += v * CZ[i];
        }
        rho[n] = r;
        for (int d = 0; d < 3; ++d) u[(int64_t)d * N + n] = (j[d] + 0.5 * (F ? F[(int64_t)d * N + n] : 0.0)) / r;
    }
}
