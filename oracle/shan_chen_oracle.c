/*
 * Shan-Chen pseudo-potential two-phase flow -- plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously-correct reference the GPU
 * Shan-Chen lattice is checked against.  Only the test suite, the smoke check
 * and the benchmark's CPU leg may load it; it shares nothing with the GPU
 * path.
 *
 * Static-bubble case of Sec. III: pseudo-potential psi = 1 - exp(-rho) and the
 * interaction force F(x) = -G psi(x) sum_i w_i c_i psi(x + c_i) (X. Shan &
 * H. Chen, Phys. Rev. E 47, 1993), handed to the paper's D3Q19 CM collision
 * (Sec. II.B, forcing of App. B) as the force density F, on a periodic box.
 *
 * Readings:
 *   S1  psi and F of one step use the density of that step's populations
 *       before the collision (rho = sum_i f_i, no force shift: F depends on
 *       rho only).
 *   S2  An optional uniform force (e.g. gravity) adds to the interaction
 *       force.
 *
 * Layout: f[i*N + n], F[d*N + n], n = x + nx*(y + ny*z), velocity order of
 * Sec. II.A.  Rates: any K (the paper's: omega on k5..k9, 1 elsewhere).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* from d3q19_oracle.c */
void orc19_tables(int *c, double *w, int *opp);
int orc19_step(int nx, int ny, int nz, int walls_y, const double *f, double *fnew, const double *F,
               const double *Krates, int per_node_K, int mode);

#define Q 19

static inline int64_t node(int x, int y, int z, int nx, int ny) { return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z); }
static inline int wrap(int a, int n) { return ((a % n) + n) % n; }

/* Sec. III static bubble: the pseudo-potential. */
double orc_sc_psi(double rho) { return 1.0 - exp(-rho); }

/* Sec. III static bubble: interaction force at every node from the density
 * field rho[N], plus the uniform force Fu[3] (reading S2). */
void orc_sc_force(int nx, int ny, int nz, const double *rho, double G, const double *Fu, double *F)
{
    int c[Q * 3], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        double s[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            const int64_t m = node(wrap(x + c[3 * i], nx), wrap(y + c[3 * i + 1], ny), wrap(z + c[3 * i + 2], nz), nx, ny);
            const double p = orc_sc_psi(rho[m]);
            for (int d = 0; d < 3; ++d) s[d] += w[i] * c[3 * i + d] * p;
        }
        const double pn = orc_sc_psi(rho[n]);
        for (int d = 0; d < 3; ++d) F[(int64_t)d * N + n] = -G * pn * s[d] + (Fu ? Fu[d] : 0.0);
    }
}

/* Density of every node (reading S1). */
static void density(int nx, int ny, int nz, const double *f, double *rho)
{
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double r = 0.0;
        for (int i = 0; i < Q; ++i) r += f[(int64_t)i * N + n];
        rho[n] = r;
    }
}

/*
 * One step: rho from f, the force field above, then the paper's collision
 * with the 19 relaxation rates K and periodic streaming (the D3Q19 oracle's
 * step, f* = T(u)^-1 k*).  F_out
 * (3N, optional) receives the force used.  Returns 0, -1 on a singular
 * collision system, -2 on allocation failure.
 */
int orc_sc_step(int nx, int ny, int nz, double G, const double *Fu, const double *K, const double *f, double *fnew,
                double *F_out)
{
    const int64_t N = (int64_t)nx * ny * nz;
    double *rho = (double *)malloc(sizeof(double) * N);
    double *F = F_out ? F_out : (double *)malloc(sizeof(double) * 3 * N);
    if (!rho || !F) {
        free(rho);
        if (!F_out) free(F);
        return -2;
    }
    density(nx, ny, nz, f, rho);
    orc_sc_force(nx, ny, nz, rho, G, Fu, F);
    const int rc = orc19_step(nx, ny, nz, 0, f, fnew, F, K, 0, 0);
    free(rho);
    if (!F_out) free(F);
    return rc;
}

/* Macroscopic fields: rho, the force-shifted velocity u = (sum_i f_i c_i +
 * F/2)/rho with the interaction force (Sec. II.A eq. "macro", App. E), and the
 * bulk pressure of the model p = cs^2 rho + G cs^2 psi^2 / 2 (Shan & Chen's
 * equation of state, cs^2 = 1/3).  Any output may be NULL. */
int orc_sc_fields(int nx, int ny, int nz, double G, const double *Fu, const double *f, double *rho_out, double *u_out,
                  double *p_out)
{
    int c[Q * 3], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    const int64_t N = (int64_t)nx * ny * nz;
    double *rho = (double *)malloc(sizeof(double) * N);
    double *F = (double *)malloc(sizeof(double) * 3 * N);
    if (!rho || !F) {
        free(rho);
        free(F);
        return -2;
    }
    density(nx, ny, nz, f, rho);
    orc_sc_force(nx, ny, nz, rho, G, Fu, F);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i)
            for (int d = 0; d < 3; ++d) j[d] += c[3 * i + d] * f[(int64_t)i * N + n];
        if (rho_out) rho_out[n] = rho[n];
        if (u_out)
            for (int d = 0; d < 3; ++d) u_out[(int64_t)d * N + n] = (j[d] + 0.5 * F[(int64_t)d * N + n]) / rho[n];
        if (p_out) {
            const double ps = orc_sc_psi(rho[n]);
            p_out[n] = rho[n] / 3.0 + G * ps * ps / 6.0;
        }
    }
    free(rho);
    free(F);
    return 0;
}
