/*
 * Two-phase flow with a conservative phase field -- plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously-correct reference the GPU
 * coupled lattice is checked against.  Only the test suite, the smoke check
 * and the benchmark's CPU leg may load it; it shares nothing with the GPU path.
 *
 * The paper's own multiphase models are Shan-Chen and the colour gradient;
 * the phase-field coupling is taken from the published literature:
 *   - interface: conservative Allen-Cahn equation of P.-H. Chiu & Y.-T. Lin,
 *     J. Comput. Phys. 230 (2011) 185, in the lattice Boltzmann form of
 *     A. Fakhari, T. Mitchell, C. Leonardi & D. Bolster, Phys. Rev. E 96
 *     (2017) 053301, on a D3Q7 lattice;
 *   - flow: pressure-based populations (zeroth moment p/cs^2, first moment
 *     rho u with rho = rho(phi)) after X. He, S. Chen & R. Zhang, J. Comput.
 *     Phys. 152 (1999) 642 and H. Liang, J. Xu, J. Chen, H. Wang, Z. Chai &
 *     B. Shi, Phys. Rev. E 97 (2018) 033309, with the collision of the
 *     paper's Sec. II.B (central moments, relaxation matrix K, CM forcing of
 *     App. B) applied to them.
 *
 * Readings:
 *   P1  Flow populations g: Pi = sum g + S0/2 is p / cs^2 (p the hydrodynamic
 *       pressure), u = (sum g c + F/2) / rho(phi), S0 = u . grad(rho) is the
 *       zeroth-moment source that turns the pressure equation into
 *       d(p/cs^2)/dt + rho div u = 0.  Equilibrium: the paper's equilibrium at
 *       the local density plus the pressure excess on the rest weights,
 *       g_eq = f_eq(rho, u) + (Pi - rho) w.  The collision is the paper's,
 *       k = T(u) g, k* = (I - K) k + K T(u) g_eq + (I - K/2) R,
 *       g* = T(u)^-1 k*, with R the CM forcing of App. B built from F, plus
 *       R0 = S0 on the zeroth row (so S0 enters half before and half after
 *       the collision, like F on the first rows), -u S0 on the first rows
 *       (the central zeroth-row source would otherwise add u S0 to the raw
 *       momentum source, which must stay F) and second-order source
 *       moments C = cs^2 (u grad(rho) + grad(rho) u + (u.grad rho) I) on rows
 *       4..9: a density that varies in space adds cs^2 (u grad rho +
 *       grad rho u) and cs^2 S0 I to the first-order non-equilibrium stress
 *       (Chapman-Enskog), which C removes, leaving rho nu (grad u + grad u^T).
 *       With phi uniform and Pi = rho this is exactly the paper's scheme at
 *       density rho.
 *   P2  rho(phi) = rho_l + phi (rho_h - rho_l), phi in [0, 1].
 *   P3  Force: surface tension F = mu grad(phi) with the chemical potential
 *       mu = 4 beta phi (phi - 1)(phi - 1/2) - kappa lap(phi),
 *       beta = 12 sigma / W, kappa = 3 sigma W / 2.  The viscous stress is
 *       the scheme's own (momentum rho u), no correction force.
 *   P4  Derivatives of phi: isotropic D3Q19 stencils,
 *       grad = (1/cs^2) sum_i w_i c_i phi(x + c_i),
 *       lap = (2/cs^2) sum_i w_i (phi(x + c_i) - phi(x)).
 *   P5  Phase lattice D3Q7 (weights 1/4, 1/8; cs^2 = 1/4):
 *       h_eq = phi w_i (1 + c_i.u / cs^2),
 *       h* = h - w_phi (h - h_eq) + (1 - w_phi/2) w_i (4/W) phi (1 - phi) c_i.n,
 *       n = grad(phi)/|grad(phi)| (0 where grad(phi) = 0),
 *       mobility M = cs^2 (1/w_phi - 1/2); phi = sum h.
 *   P6  Uniform kinematic viscosity nu = cs^2 (1/omega - 1/2) in both phases.
 *
 * Parameters prm[6]: rho_l, rho_h, sigma, W, M, omega.
 * Layout: g[i*N + n] (19), h[i*N + n] (7), n = x + nx*(y + ny*z); periodic.
 * D3Q7 order: 0 rest, 1..3 = -x,-y,-z, 4..6 = +x,+y,+z.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* from d3q19_oracle.c */
void orc19_tables(int *c, double *w, int *opp);
void orc19_feq(double rho, double ux, double uy, double uz, double *feq);
void orc19_T(double ux, double uy, double uz, double *T);
void orc19_Rcm(double Fx, double Fy, double Fz, double *R);
int orc_solve19(double *A, double *b, double *x);

#define Q 19
#define Q7 7
static const double CS2 = 1.0 / 3.0;
static const double CS2_7 = 0.25;
static const int C7[Q7][3] = {{0, 0, 0}, {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
static const double W7[Q7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};

void orc_pf_tables7(int *c, double *w)
{
    for (int i = 0; i < Q7; ++i) {
        for (int d = 0; d < 3; ++d) c[3 * i + d] = C7[i][d];
        w[i] = W7[i];
    }
}

static inline int64_t node(int x, int y, int z, int nx, int ny) { return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z); }
static inline int wrap(int a, int n) { return ((a % n) + n) % n; }

/* Reading P4: gradient and Laplacian of phi from its 19 stencil values
 * phin[i] = phi(x + c_i) (phin[0] = phi(x)). */
void orc_pf_derivs(const double *phin, double *grad, double *lap)
{
    int c[3 * Q], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    double gx = 0.0, gy = 0.0, gz = 0.0, l = 0.0;
    for (int i = 0; i < Q; ++i) {
        gx += w[i] * c[3 * i] * phin[i];
        gy += w[i] * c[3 * i + 1] * phin[i];
        gz += w[i] * c[3 * i + 2] * phin[i];
        l += w[i] * (phin[i] - phin[0]);
    }
    grad[0] = gx / CS2;
    grad[1] = gy / CS2;
    grad[2] = gz / CS2;
    *lap = 2.0 * l / CS2;
}

/* Readings P1-P3: density, chemical potential, force, velocity, source and
 * pressure at a node from its phi stencil and flow populations g.
 * out: [0] Pi, [1] rho, [2..4] u, [5..7] F, [8] mu, [9] S0. */
void orc_pf_macro(const double *prm, const double *g, const double *phin, double *out)
{
    const double rl = prm[0], rh = prm[1], sigma = prm[2], W = prm[3];
    const double beta = 12.0 * sigma / W, kappa = 1.5 * sigma * W;
    int c[3 * Q], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    double grad[3], lap;
    orc_pf_derivs(phin, grad, &lap);
    const double phi = phin[0];
    const double rho = rl + phi * (rh - rl);
    const double mu = 4.0 * beta * phi * (phi - 1.0) * (phi - 0.5) - kappa * lap;
    double sum = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        sum += g[i];
        for (int a = 0; a < 3; ++a) j[a] += g[i] * c[3 * i + a];
    }
    double S0 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double F = mu * grad[a];
        out[5 + a] = F;
        out[2 + a] = (j[a] + 0.5 * F) / rho;
        S0 += out[2 + a] * (rh - rl) * grad[a];
    }
    out[0] = sum + 0.5 * S0;
    out[1] = rho;
    out[8] = mu;
    out[9] = S0;
}

/* Reading P1: collision of the flow populations at one node (definition:
 * dense T(u) solve).  K rates: 1 on the conserved rows, bulk 1, omega on
 * k5..k9, 1 on k10..k18 (Sec. II.B). */
int orc_pf_collide_g(double omega, const double *g, double Pi, double rho, const double *u, const double *F,
                     const double *grho, double *gs)
{
    int c[3 * Q], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    double T[Q * Q], k[Q], keq[Q], R[Q], ks[Q], geq[Q];
    orc19_feq(rho, u[0], u[1], u[2], geq);
    for (int i = 0; i < Q; ++i) geq[i] += (Pi - rho) * w[i];
    orc19_T(u[0], u[1], u[2], T);
    for (int r = 0; r < Q; ++r) {
        double s = 0.0, se = 0.0;
        for (int i = 0; i < Q; ++i) {
            s += T[r * Q + i] * g[i];
            se += T[r * Q + i] * geq[i];
        }
        k[r] = s;
        keq[r] = se;
    }
    orc19_Rcm(F[0], F[1], F[2], R);
    /* reading P1: zeroth-row source and second-order source moments
     * C_ab = cs^2 (u_a d_b rho + u_b d_a rho + delta_ab u.grad rho) in the rows
     * of T (k4 trace, k5 = xx - yy, k6 = yy - zz, k7..k9 = xy, xz, yz) */
    const double ug = u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2];
    double C[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) C[a][b] = CS2 * (u[a] * grho[b] + u[b] * grho[a] + (a == b ? ug : 0.0));
    R[0] = ug;
    for (int a = 0; a < 3; ++a) R[1 + a] -= u[a] * ug; /* raw momentum source stays F */
    R[4] = C[0][0] + C[1][1] + C[2][2];
    R[5] = C[0][0] - C[1][1];
    R[6] = C[1][1] - C[2][2];
    R[7] = C[0][1];
    R[8] = C[0][2];
    R[9] = C[1][2];
    for (int r = 0; r < Q; ++r) {
        const double K = (r >= 5 && r <= 9) ? omega : 1.0;
        ks[r] = (1.0 - K) * k[r] + K * keq[r] + (1.0 - 0.5 * K) * R[r];
    }
    return orc_solve19(T, ks, gs);
}

/* Reading P5: collision of the phase populations at one node. */
void orc_pf_collide_h(double W, double M, const double *h, const double *phin, const double *u, double *hs)
{
    double grad[3], lap;
    orc_pf_derivs(phin, grad, &lap);
    const double phi = phin[0];
    const double g2 = grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2];
    double n[3] = {0.0, 0.0, 0.0};
    if (g2 > 0.0)
        for (int d = 0; d < 3; ++d) n[d] = grad[d] / sqrt(g2);
    const double wphi = 1.0 / (M / CS2_7 + 0.5);
    const double theta = 4.0 / W * phi * (1.0 - phi);
    for (int i = 0; i < Q7; ++i) {
        const double cu = C7[i][0] * u[0] + C7[i][1] * u[1] + C7[i][2] * u[2];
        const double cn = C7[i][0] * n[0] + C7[i][1] * n[1] + C7[i][2] * n[2];
        const double heq = phi * W7[i] * (1.0 + cu / CS2_7);
        const double F = W7[i] * theta * cn;
        hs[i] = h[i] - wphi * (h[i] - heq) + (1.0 - 0.5 * wphi) * F;
    }
}

static void gather_phi(int nx, int ny, int nz, const double *phi, int x, int y, int z, double *phin)
{
    int c[3 * Q], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    for (int i = 0; i < Q; ++i)
        phin[i] = phi[node(wrap(x + c[3 * i], nx), wrap(y + c[3 * i + 1], ny), wrap(z + c[3 * i + 2], nz), nx, ny)];
}

static void phase_sum(int64_t N, const double *h, double *phi)
{
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double s = 0.0;
        for (int i = 0; i < Q7; ++i) s += h[(int64_t)i * N + n];
        phi[n] = s;
    }
}

/* One time step: phi = sum h everywhere, then at every node the macroscopic
 * step (orc_pf_macro), both collisions and streaming
 * g_i(x + c_i, t+1) = g_i*(x, t), h_i(x + c_i, t+1) = h_i*(x, t) (periodic).
 * Returns 0, or -1 if a collision system was singular. */
int orc_pf_step(int nx, int ny, int nz, const double *prm, const double *g, const double *h, double *gnew,
                double *hnew)
{
    const int64_t N = (int64_t)nx * ny * nz;
    double *phi = (double *)malloc(sizeof(double) * N);
    if (!phi) return -2;
    phase_sum(N, h, phi);
    int c[3 * Q], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int64_t n = 0; n < N; ++n) {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        double phin[Q], gl[Q], hl[Q7], gs[Q], hs[Q7], mac[10];
        gather_phi(nx, ny, nz, phi, x, y, z, phin);
        for (int i = 0; i < Q; ++i) gl[i] = g[(int64_t)i * N + n];
        for (int i = 0; i < Q7; ++i) hl[i] = h[(int64_t)i * N + n];
        orc_pf_macro(prm, gl, phin, mac);
        double grho[3], gphi[3], lap;
        orc_pf_derivs(phin, gphi, &lap);
        for (int d = 0; d < 3; ++d) grho[d] = (prm[1] - prm[0]) * gphi[d];
        if (orc_pf_collide_g(prm[5], gl, mac[0], mac[1], mac + 2, mac + 5, grho, gs) != 0) err |= 1;
        orc_pf_collide_h(prm[3], prm[4], hl, phin, mac + 2, hs);
        for (int i = 0; i < Q; ++i)
            gnew[(int64_t)i * N + node(wrap(x + c[3 * i], nx), wrap(y + c[3 * i + 1], ny), wrap(z + c[3 * i + 2], nz), nx, ny)] = gs[i];
        for (int i = 0; i < Q7; ++i)
            hnew[(int64_t)i * N + node(wrap(x + C7[i][0], nx), wrap(y + C7[i][1], ny), wrap(z + C7[i][2], nz), nx, ny)] = hs[i];
    }
    free(phi);
    return err ? -1 : 0;
}

/* Initial populations at equilibrium from phi, the pressure p and u:
 * g = f_eq(rho(phi), u) + (p/cs^2 - rho(phi)) w, h = h_eq(phi, u). */
void orc_pf_init(int nx, int ny, int nz, const double *prm, const double *phi, const double *p, const double *u,
                 double *g, double *h)
{
    const int64_t N = (int64_t)nx * ny * nz;
    int c[3 * Q], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    for (int64_t n = 0; n < N; ++n) {
        const double rho = prm[0] + phi[n] * (prm[1] - prm[0]);
        double fe[Q];
        orc19_feq(rho, u[n], u[N + n], u[2 * N + n], fe);
        for (int i = 0; i < Q; ++i) g[(int64_t)i * N + n] = fe[i] + (p[n] / CS2 - rho) * w[i];
        for (int i = 0; i < Q7; ++i) {
            const double cu = C7[i][0] * u[n] + C7[i][1] * u[N + n] + C7[i][2] * u[2 * N + n];
            h[(int64_t)i * N + n] = phi[n] * W7[i] * (1.0 + cu / CS2_7);
        }
    }
}

/* Macroscopic fields of a state: phi, pressure p = cs^2 Pi, rho(phi) and the
 * force-shifted velocity u (what the next step would use). */
void orc_pf_fields(int nx, int ny, int nz, const double *prm, const double *g, const double *h, double *phi_out,
                   double *p_out, double *rho_out, double *u_out)
{
    const int64_t N = (int64_t)nx * ny * nz;
    double *phi = (double *)malloc(sizeof(double) * N);
    if (!phi) return;
    phase_sum(N, h, phi);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        double phin[Q], gl[Q], mac[10];
        gather_phi(nx, ny, nz, phi, x, y, z, phin);
        for (int i = 0; i < Q; ++i) gl[i] = g[(int64_t)i * N + n];
        orc_pf_macro(prm, gl, phin, mac);
        if (phi_out) phi_out[n] = phi[n];
        if (p_out) p_out[n] = mac[0] * CS2;
        if (rho_out) rho_out[n] = mac[1];
        if (u_out)
            for (int d = 0; d < 3; ++d) u_out[(int64_t)d * N + n] = mac[2 + d];
    }
    free(phi);
}
