/*
 * Colour-gradient two-phase flow on the D3Q19 CM lattice -- plain FP64 CPU
 * oracle.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously-correct reference the GPU
 * colour-gradient lattice is checked against.  Only the test suite, the smoke
 * check and the benchmark's CPU leg may load it; it shares nothing with the
 * GPU path.
 *
 * Method: App. E (colour-gradient method on the D3Q19 CM collision; the
 * Rayleigh-Taylor case of Sec. III).  Red and blue populations f^r, f^b;
 * f = f^r + f^b collides with the scheme of Sec. II.B towards
 * h_eq = f_eq(rho, u) + rho (phi_i(alpha) - w_i); the perturbation operator
 * adds interfacial tension; the recolouring operator splits the result
 * between the colours; each colour streams.
 *
 * Readings:
 *   G1  Perturbation: (A/2) |grad phi| [w_i (c_i . grad phi)^2 / |grad phi|^2
 *       - B_i], the projection squared (as printed, linear, it would not
 *       conserve mass: sum_i B_i = 1/3), applied once to the total f after
 *       the collision, with A = A_r + A_b; the paper's sigma = (2/9) A / omega.
 *   G2  Recolouring equilibrium g_eq(rho, 0) = rho phi_i(alpha) (the
 *       zero-velocity h_eq, = sum_k rho_k phi_i(alpha_k)); cos(theta_0) = 0;
 *       where grad phi = 0 neither perturbation nor recolouring bias acts.
 *   G3  grad phi = (1/cs^2) sum_i w_i c_i phi(x + c_i); beyond a wall the
 *       neighbour's phi is the wall-side node's own (zero normal gradient).
 *   G4  Body force F = (rho - rho_ref) g with g the gravity vector (the heavy
 *       fluid is driven along g; printed with the opposite sign, which would
 *       drive it away from the wall the instability grows towards).
 *   G5  alpha = (rho_r alpha_r + rho_b alpha_b) / rho; pressure
 *       p = rho (1 - alpha) / 2, a third of the trace CM k4 = 3 rho (1 - alpha)/2
 *       of h_eq.
 *   G6  Initial colours from (rho_r, rho_b, u): f^k = (rho_k / rho) h_eq(rho, u).
 *
 * Parameters prm[9]: omega, alpha_r, alpha_b, A, beta, g (3), rho_ref.
 * Layout: f^r[i*N + n], f^b[i*N + n]; n = x + nx*(y + ny*z).  Rates: omega
 * on k5..k9, 1 elsewhere (the paper's).  Walls (walls_y): halfway bounce-back
 * of both colours at y = -1/2 and ny - 1/2.
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
void orc19_K(double omega, double omega_bulk, const double *omega_hi, double *K);
int orc_solve19(double *A, double *b, double *x);

#define Q 19

static inline int64_t node(int x, int y, int z, int nx, int ny) { return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z); }
static inline int wrap(int a, int n) { return ((a % n) + n) % n; }

/* App. E: phi_i(alpha) = alpha (rest), (1 - alpha)/12 (|c|^2 = 1), (1 - alpha)/24 (|c|^2 = 2). */
double orc_cg_phi_i(int c2, double alpha)
{
    return c2 == 0 ? alpha : (c2 == 1 ? (1.0 - alpha) / 12.0 : (1.0 - alpha) / 24.0);
}

/* App. E: B_i = -1/3, 1/18, 1/36 by |c|^2. */
static double B_i(int c2) { return c2 == 0 ? -1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0); }

/* App. E eq. (feqCG): h_eq = f_eq(rho, u) + rho (phi_i(alpha) - w_i). */
void orc_cg_heq(double rho, double ux, double uy, double uz, double alpha, double *h)
{
    int c[Q * 3], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    orc19_feq(rho, ux, uy, uz, h);
    for (int i = 0; i < Q; ++i) {
        const int c2 = c[3 * i] * c[3 * i] + c[3 * i + 1] * c[3 * i + 1] + c[3 * i + 2] * c[3 * i + 2];
        h[i] += rho * (orc_cg_phi_i(c2, alpha) - w[i]);
    }
}

/*
 * One colour-gradient collision at one node.  fr, fb: the colours' 19
 * populations; grad: grad phi at the node (reading G3); prm as above.
 * Writes the post-collision colours.  Returns 0 or -1 (singular system).
 */
int orc_cg_collide(const double *fr, const double *fb, const double *grad, const double *prm, double *fr_out,
                   double *fb_out, double *rho_out, double *u_out)
{
    int c[Q * 3], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    const double omega = prm[0], ar = prm[1], ab = prm[2], A = prm[3], beta = prm[4];
    double rr = 0.0, rb = 0.0, f[Q], j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        rr += fr[i];
        rb += fb[i];
        f[i] = fr[i] + fb[i];
        for (int d = 0; d < 3; ++d) j[d] += c[3 * i + d] * f[i];
    }
    const double rho = rr + rb;
    const double alpha = (rr * ar + rb * ab) / rho; /* reading G5 */
    double F[3];
    for (int d = 0; d < 3; ++d) F[d] = (rho - prm[8]) * prm[5 + d]; /* reading G4 */
    double u[3];
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * F[d]) / rho;
    /* single-phase operator: the CM collision of Sec. II.B towards h_eq */
    double T[Q * Q], k[Q], heq[Q], keq[Q], R[Q], K[Q], ks[Q], fs[Q];
    orc19_T(u[0], u[1], u[2], T);
    orc_cg_heq(rho, u[0], u[1], u[2], alpha, heq);
    for (int r = 0; r < Q; ++r) {
        double s = 0.0, e = 0.0;
        for (int i = 0; i < Q; ++i) {
            s += T[r * Q + i] * f[i];
            e += T[r * Q + i] * heq[i];
        }
        k[r] = s;
        keq[r] = e;
    }
    /* conserved rows: k0 = rho exactly, k1..3 of h_eq vanish by construction */
    orc19_Rcm(F[0], F[1], F[2], R);
    orc19_K(omega, 1.0, NULL, K);
    for (int r = 0; r < Q; ++r) ks[r] = (1.0 - K[r]) * k[r] + K[r] * keq[r] + (1.0 - 0.5 * K[r]) * R[r];
    if (orc_solve19(T, ks, fs) != 0) return -1;
    /* perturbation (reading G1) and recolouring (reading G2) */
    const double g2 = grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2];
    const double gn = sqrt(g2);
    for (int i = 0; i < Q; ++i) {
        const int c2 = c[3 * i] * c[3 * i] + c[3 * i + 1] * c[3 * i + 1] + c[3 * i + 2] * c[3 * i + 2];
        const double cg = c[3 * i] * grad[0] + c[3 * i + 1] * grad[1] + c[3 * i + 2] * grad[2];
        double cos_t = 0.0;
        if (gn > 0.0) {
            fs[i] += 0.5 * A * gn * (w[i] * cg * cg / g2 - B_i(c2));
            if (c2 > 0) cos_t = cg / (sqrt((double)c2) * gn);
        }
        const double geq = rho * orc_cg_phi_i(c2, alpha);
        const double bias = beta * rr * rb / (rho * rho) * cos_t * geq;
        fr_out[i] = rr / rho * fs[i] + bias;
        fb_out[i] = rb / rho * fs[i] - bias;
    }
    if (rho_out) *rho_out = rho;
    if (u_out)
        for (int d = 0; d < 3; ++d) u_out[d] = u[d];
    return 0;
}

/* phi = (rho_r - rho_b)/(rho_r + rho_b) at every node. */
static void order_parameter(int64_t N, const double *fr, const double *fb, double *phi)
{
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double rr = 0.0, rb = 0.0;
        for (int i = 0; i < Q; ++i) {
            rr += fr[(int64_t)i * N + n];
            rb += fb[(int64_t)i * N + n];
        }
        phi[n] = (rr - rb) / (rr + rb);
    }
}

/* Reading G3 at node (x, y, z). */
static void grad_phi(int nx, int ny, int nz, int walls_y, const double *phi, int x, int y, int z, const int *c,
                     const double *w, double *g)
{
    g[0] = g[1] = g[2] = 0.0;
    for (int i = 1; i < Q; ++i) {
        int yy = y + c[3 * i + 1];
        if (walls_y && (yy < 0 || yy >= ny))
            yy = y; /* beyond a wall: mirrored, phi(x', -1) = phi(x', 0) */
        else
            yy = wrap(yy, ny);
        const double p = phi[node(wrap(x + c[3 * i], nx), yy, wrap(z + c[3 * i + 2], nz), nx, ny)];
        for (int d = 0; d < 3; ++d) g[d] += 3.0 * w[i] * c[3 * i + d] * p;
    }
}

/*
 * One step: phi from the colours, then at every node grad phi, the collision
 * above and streaming of both colours (periodic in x and z, and in y unless
 * walls_y, where halfway bounce-back applies).  Returns 0, -1 (singular
 * system) or -2 (allocation).
 */
int orc_cg_step(int nx, int ny, int nz, int walls_y, const double *prm, const double *fr, const double *fb, double *frn,
                double *fbn)
{
    int c[Q * 3], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    const int64_t N = (int64_t)nx * ny * nz;
    double *phi = (double *)malloc(sizeof(double) * N);
    if (!phi) return -2;
    order_parameter(N, fr, fb, phi);
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int64_t n = 0; n < N; ++n) {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        double a[Q], b[Q], ao[Q], bo[Q], g[3];
        for (int i = 0; i < Q; ++i) {
            a[i] = fr[(int64_t)i * N + n];
            b[i] = fb[(int64_t)i * N + n];
        }
        grad_phi(nx, ny, nz, walls_y, phi, x, y, z, c, w, g);
        if (orc_cg_collide(a, b, g, prm, ao, bo, NULL, NULL) != 0) err |= 1;
        for (int i = 0; i < Q; ++i) {
            int yd = y + c[3 * i + 1];
            if (walls_y && (yd < 0 || yd >= ny)) {
                frn[(int64_t)opp[i] * N + n] = ao[i];
                fbn[(int64_t)opp[i] * N + n] = bo[i];
                continue;
            }
            const int64_t m = node(wrap(x + c[3 * i], nx), wrap(yd, ny), wrap(z + c[3 * i + 2], nz), nx, ny);
            frn[(int64_t)i * N + m] = ao[i];
            fbn[(int64_t)i * N + m] = bo[i];
        }
    }
    free(phi);
    return err ? -1 : 0;
}

/* Reading G6. */
void orc_cg_init(int nx, int ny, int nz, const double *prm, const double *rr, const double *rb, const double *u,
                 double *fr, double *fb)
{
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        const double rho = rr[n] + rb[n];
        const double alpha = (rr[n] * prm[1] + rb[n] * prm[2]) / rho;
        double h[Q];
        orc_cg_heq(rho, u[n], u[N + n], u[2 * N + n], alpha, h);
        for (int i = 0; i < Q; ++i) {
            fr[(int64_t)i * N + n] = rr[n] / rho * h[i];
            fb[(int64_t)i * N + n] = rb[n] / rho * h[i];
        }
    }
}

/* Fields: rho_r, rho_b, phi, force-shifted u (with the body force of reading
 * G4) and p = rho (1 - alpha)/2 (reading G5).  Outputs may be NULL. */
void orc_cg_fields(int nx, int ny, int nz, const double *prm, const double *fr, const double *fb, double *rr_out,
                   double *rb_out, double *phi_out, double *u_out, double *p_out)
{
    int c[Q * 3], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double rr = 0.0, rb = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            const double a = fr[(int64_t)i * N + n], b = fb[(int64_t)i * N + n];
            rr += a;
            rb += b;
            for (int d = 0; d < 3; ++d) j[d] += c[3 * i + d] * (a + b);
        }
        const double rho = rr + rb;
        if (rr_out) rr_out[n] = rr;
        if (rb_out) rb_out[n] = rb;
        if (phi_out) phi_out[n] = (rr - rb) / rho;
        if (u_out)
            for (int d = 0; d < 3; ++d) u_out[(int64_t)d * N + n] = (j[d] + 0.5 * (rho - prm[8]) * prm[5 + d]) / rho;
        if (p_out) {
            const double alpha = (rr * prm[1] + rb * prm[2]) / rho;
            p_out[n] = 0.5 * rho * (1.0 - alpha);
        }
    }
}
