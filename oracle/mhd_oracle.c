/*
 * Magnetohydrodynamics with a vector magnetic lattice -- plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously-correct reference the GPU
 * coupled magnetic lattice is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU leg may load it; it shares nothing with
 * the GPU path.
 *
 * The paper runs Hartmann flow (Sec. III, the MHD case) with a separate
 * magnetic lattice that it cites but does not write out; the induction
 * equation is taken here in the vector-valued lattice Boltzmann form of
 * P. J. Dellar, J. Comput. Phys. 179 (2002) 95, on a D3Q7 lattice.
 *
 * Readings:
 *   M1  Magnetic populations g_{i,a} (i in D3Q7: weights 1/4, 1/8, cs^2 = 1/4;
 *       a = x, y, z) with b_a = sum_i g_{i,a} and equilibrium
 *       g_eq_{i,a} = w_i (b_a + c_{i,c} (u_c b_a - b_c u_a) / cs^2),
 *       relaxed at one rate: g* = g - w_m (g - g_eq), w_m = 1/(eta/cs^2 + 1/2)
 *       (induction equation d_t b = curl(u x b) + eta lap b).
 *   M2  Current j = curl b from the non-equilibrium first moments,
 *       Lambda_{c,a} = sum_i c_{i,c} g_{i,a} - (u0_c b_a - b_c u0_a),
 *       j_e = -(w_m / cs^2) eps_{e,c,a} Lambda_{c,a}, with u0 = sum_i f_i c_i / rho
 *       (the flow velocity before the force; the force depends on j).
 *   M3  Lorentz force F_L = j x b (units with mu0 = 1) added to the external
 *       force and handed to the paper's collision (Sec. II.B, App. B) as F;
 *       the magnetic equilibrium then uses the force-shifted u of that
 *       collision.
 *   M4  Walls (walls_y): flow populations bounce back halfway (as the plain
 *       lattice); magnetic populations are anti-bounced back,
 *       g_{opp(i),a}(x, t+1) = -g*_{i,a}(x, t) + 2 w_i b_wall_a, which puts
 *       b = b_wall (the field imposed at the walls, Sec. III) on the wall.
 *
 * Parameters prm[4]: eta, b_wall (3).  Flow rates: omega on k5..k9, 1
 * elsewhere (the paper's).
 * Layout: f[i*N + n] (19), g[(a*7 + i)*N + n] (21), F[d*N + n];
 * n = x + nx*(y + ny*z).  D3Q7 order: rest, -x, -y, -z, +x, +y, +z.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* from d3q19_oracle.c */
void orc19_tables(int *c, double *w, int *opp);
void orc19_feq(double rho, double ux, double uy, double uz, double *feq);
int orc19_collide(const double *f, const double *F, const double *K, int mode, double *fstar, double *kout,
                  double *rho_out, double *uout);
void orc19_K(double omega, double omega_bulk, const double *omega_hi, double *K);

#define Q 19
#define Q7 7
static const double CS2M = 0.25;
static const int C7[Q7][3] = {{0, 0, 0}, {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
static const double W7[Q7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};
static int opp7(int i) { return i == 0 ? 0 : (i <= 3 ? i + 3 : i - 3); }

static inline int64_t node(int x, int y, int z, int nx, int ny) { return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z); }
static inline int wrap(int a, int n) { return ((a % n) + n) % n; }

/* Reading M1: the 21 equilibrium values geq[a*7 + i]. */
void orc_mhd_geq(const double *b, const double *u, double *geq)
{
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < Q7; ++i) {
            double s = b[a];
            for (int c = 0; c < 3; ++c) s += C7[i][c] * (u[c] * b[a] - b[c] * u[a]) / CS2M;
            geq[a * Q7 + i] = W7[i] * s;
        }
}

/* Reading M2: b and j of one node from its 21 magnetic populations. */
void orc_mhd_current(const double *g, const double *u0, double omega_m, double *b, double *j)
{
    for (int a = 0; a < 3; ++a) {
        b[a] = 0.0;
        for (int i = 0; i < Q7; ++i) b[a] += g[a * Q7 + i];
    }
    double lam[3][3]; /* lam[c][a] */
    for (int c = 0; c < 3; ++c)
        for (int a = 0; a < 3; ++a) {
            double s = 0.0;
            for (int i = 0; i < Q7; ++i) s += C7[i][c] * g[a * Q7 + i];
            lam[c][a] = s - (u0[c] * b[a] - b[c] * u0[a]);
        }
    /* j_e = -(w_m/cs^2) eps_{e c a} lam[c][a] */
    const double k = -omega_m / CS2M;
    j[0] = k * (lam[1][2] - lam[2][1]);
    j[1] = k * (lam[2][0] - lam[0][2]);
    j[2] = k * (lam[0][1] - lam[1][0]);
}

/* Readings M2, M3 at one node: rho, u0, b, j and the total force. */
static void node_state(const double *fl, const double *gl, const double *Fext, double omega_m, double *rho,
                       double *u0, double *b, double *j, double *F)
{
    int c[3 * Q], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    double r = 0.0, m[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        r += fl[i];
        for (int d = 0; d < 3; ++d) m[d] += fl[i] * c[3 * i + d];
    }
    *rho = r;
    for (int d = 0; d < 3; ++d) u0[d] = m[d] / r;
    orc_mhd_current(gl, u0, omega_m, b, j);
    F[0] = Fext[0] + j[1] * b[2] - j[2] * b[1];
    F[1] = Fext[1] + j[2] * b[0] - j[0] * b[2];
    F[2] = Fext[2] + j[0] * b[1] - j[1] * b[0];
}

/*
 * One time step.  Flow: the paper's collision (f* = T(u)^-1 k*, K from omega)
 * with F = F_ext + j x b, streaming with periodic wrap and, if walls_y,
 * halfway bounce-back at y = -1/2 and ny - 1/2.  Magnetic: BGK at w_m with
 * the force-shifted u, streaming likewise with anti-bounce-back (M4).
 * Fext: 3*N or NULL.  Returns 0, or -1 if a collision failed.
 */
int orc_mhd_step(int nx, int ny, int nz, int walls_y, const double *prm, double omega, const double *f,
                 const double *g, const double *Fext, double *fnew, double *gnew)
{
    const int64_t N = (int64_t)nx * ny * nz;
    const double eta = prm[0];
    const double *bw = prm + 1;
    const double omega_m = 1.0 / (eta / CS2M + 0.5);
    int c[3 * Q], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    double K[Q];
    orc19_K(omega, 1.0, NULL, K);
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int64_t n = 0; n < N; ++n) {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        double fl[Q], gl[3 * Q7], fs[Q], Fe[3] = {0, 0, 0}, rho, u0[3], b[3], j[3], F[3], u[3];
        for (int i = 0; i < Q; ++i) fl[i] = f[(int64_t)i * N + n];
        for (int k = 0; k < 3 * Q7; ++k) gl[k] = g[(int64_t)k * N + n];
        if (Fext)
            for (int d = 0; d < 3; ++d) Fe[d] = Fext[(int64_t)d * N + n];
        node_state(fl, gl, Fe, omega_m, &rho, u0, b, j, F);
        if (orc19_collide(fl, F, K, 0, fs, NULL, NULL, u) != 0) err |= 1;
        double geq[3 * Q7];
        orc_mhd_geq(b, u, geq);
        for (int i = 0; i < Q; ++i) {
            int yd = y + c[3 * i + 1];
            if (walls_y && (yd < 0 || yd >= ny)) {
                fnew[(int64_t)opp[i] * N + n] = fs[i];
                continue;
            }
            fnew[(int64_t)i * N + node(wrap(x + c[3 * i], nx), wrap(yd, ny), wrap(z + c[3 * i + 2], nz), nx, ny)] = fs[i];
        }
        for (int a = 0; a < 3; ++a)
            for (int i = 0; i < Q7; ++i) {
                const double gs = gl[a * Q7 + i] - omega_m * (gl[a * Q7 + i] - geq[a * Q7 + i]);
                int yd = y + C7[i][1];
                if (walls_y && (yd < 0 || yd >= ny)) {
                    gnew[(int64_t)(a * Q7 + opp7(i)) * N + n] = -gs + 2.0 * W7[i] * bw[a];
                    continue;
                }
                gnew[(int64_t)(a * Q7 + i) * N + node(wrap(x + C7[i][0], nx), wrap(yd, ny), wrap(z + C7[i][2], nz), nx, ny)] = gs;
            }
    }
    return err ? -1 : 0;
}

/* Equilibrium start: f = f_eq(rho, u), g = g_eq(b, u). */
void orc_mhd_init(int nx, int ny, int nz, const double *rho, const double *u, const double *b, double *f, double *g)
{
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t n = 0; n < N; ++n) {
        double fe[Q], ge[3 * Q7];
        const double ul[3] = {u[n], u[N + n], u[2 * N + n]}, bl[3] = {b[n], b[N + n], b[2 * N + n]};
        orc19_feq(rho[n], ul[0], ul[1], ul[2], fe);
        orc_mhd_geq(bl, ul, ge);
        for (int i = 0; i < Q; ++i) f[(int64_t)i * N + n] = fe[i];
        for (int k = 0; k < 3 * Q7; ++k) g[(int64_t)k * N + n] = ge[k];
    }
}

/* Fields of a state: rho, force-shifted u (with the Lorentz force), b, j. */
void orc_mhd_fields(int nx, int ny, int nz, const double *prm, const double *f, const double *g, const double *Fext,
                    double *rho_out, double *u_out, double *b_out, double *j_out)
{
    const int64_t N = (int64_t)nx * ny * nz;
    const double omega_m = 1.0 / (prm[0] / CS2M + 0.5);
    int c[3 * Q], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double fl[Q], gl[3 * Q7], Fe[3] = {0, 0, 0}, rho, u0[3], b[3], j[3], F[3];
        for (int i = 0; i < Q; ++i) fl[i] = f[(int64_t)i * N + n];
        for (int k = 0; k < 3 * Q7; ++k) gl[k] = g[(int64_t)k * N + n];
        if (Fext)
            for (int d = 0; d < 3; ++d) Fe[d] = Fext[(int64_t)d * N + n];
        node_state(fl, gl, Fe, omega_m, &rho, u0, b, j, F);
        if (rho_out) rho_out[n] = rho;
        for (int d = 0; d < 3; ++d) {
            if (u_out) u_out[(int64_t)d * N + n] = u0[d] + 0.5 * F[d] / rho;
            if (b_out) b_out[(int64_t)d * N + n] = b[d];
            if (j_out) j_out[(int64_t)d * N + n] = j[d];
        }
    }
}
