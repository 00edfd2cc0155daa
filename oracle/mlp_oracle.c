/*
 * Learned higher-order rates for the D3Q19 CM-LBM -- FP64 CPU oracle
 * (test infrastructure only; see d3q19_oracle.c for the rules of this
 * directory).
 *
 * The paper fixes the rates of the higher-order CMs k10..k18 to 1 (Sec. II.B).
 * The learned variant replaces them, per node, by the output of a small MLP;
 * the conserved (k0..k3), bulk (k4) and viscous (k5..k9) rates are untouched.
 * This part is not in the paper; the readings are:
 *   L1  inputs (11): rho - 1, (k4 - rho)/rho, k10..k15 / rho,
 *       (k16..k18 - rho cs^4)/rho, each divided by a fixed per-feature scale;
 *       k are the pre-collision CMs T(u) f of Sec. II.B.
 *   L2  network 11 -> 32 -> 32 -> 9, ReLU hidden layers (max(s, 0)), linear
 *       output z, rates omega_hi_j = 1 + z_j.  If any omega_hi_j leaves (0, 2)
 *       the node uses the paper's rates (all 1) -- the fallback.
 *   L3  parameter vector (1737 doubles): W1[32][11], b1[32], W2[32][32], b2[32],
 *       W3[9][32], b3[9]; W[out][in], row-major.
 *   L4  optional BF16 emulation of the GPU: the inputs of each matrix product
 *       (features, hidden activations) are rounded to float then to bfloat16
 *       (round to nearest even); weights are passed already rounded.  The
 *       gradient treats each rounding as the identity.
 *   L5  training target: one D3Q19 step (collide with learned rates, stream)
 *       from a state f(t); loss = mean over nodes of
 *       sum_k ((m_k(f(t+1)) - target_k) / sigma_k)^2 with the 10 raw moments
 *       m = (rho, j_x, j_y, j_z, Pi_xx, Pi_yy, Pi_zz, Pi_xy, Pi_xz, Pi_yz).
 *       Periodic lattice, F = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19
#define NIN 11
#define NH 32
#define NOUT 9
#define NPARAM (NH * NIN + NH + NH * NH + NH + NOUT * NH + NOUT)

/* from d3q19_oracle.c */
void orc19_T(double ux, double uy, double uz, double *T);
void orc19_K(double omega, double omega_bulk, const double *omega_hi, double *K);
int orc19_collide(const double *f, const double *F, const double *K, int mode, double *fstar, double *kout,
                  double *rho_out, double *uout);
void orc19_Rcm(double Fx, double Fy, double Fz, double *R);
void orc19_tables(int *c, double *w, int *opp);

int orc_mlp_nparam(void) { return NPARAM; }

/* round to float, then to bfloat16 with round-to-nearest-even (reading L4) */
double orc_bf16(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return v; /* NaN */
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static const double *W1(const double *P) { return P; }
static const double *B1(const double *P) { return P + NH * NIN; }
static const double *W2(const double *P) { return P + NH * NIN + NH; }
static const double *B2(const double *P) { return P + NH * NIN + NH + NH * NH; }
static const double *W3(const double *P) { return P + NH * NIN + NH + NH * NH + NH; }
static const double *B3(const double *P) { return P + NH * NIN + NH + NH * NH + NH + NOUT * NH; }

/* Reading L1: features from rho and the pre-collision CMs k[19]. */
void orc_mlp_features(double rho, const double *k, const double *scales, double *x)
{
    const double cs4 = 1.0 / 9.0;
    double raw[NIN];
    raw[0] = rho - 1.0;
    raw[1] = (k[4] - rho) / rho;
    for (int j = 0; j < 6; ++j) raw[2 + j] = k[10 + j] / rho;
    for (int j = 0; j < 3; ++j) raw[8 + j] = (k[16 + j] - rho * cs4) / rho;
    for (int j = 0; j < NIN; ++j) x[j] = raw[j] / scales[j];
}

/* Distance of v from the nearest bf16 rounding tie (a value halfway between
 * two adjacent bf16 numbers), in units of 2^-24 * scale: how far an FP32
 * evaluation of v, in error by a few 2^-24 * scale, can stray before it
 * rounds to a different bf16 value than v does.  Zero has no tie near it. */
static double bf16_tie_ulps(double v, double scale)
{
    float f = (float)v;
    if (f == 0.0f || !isfinite(f) || !(scale > 0.0) || !isfinite(scale)) return INFINITY;
    uint32_t u;
    memcpy(&u, &f, 4);
    const uint32_t mid = (u & 0xffff0000u) | 0x8000u; /* the tie inside v's bf16 interval */
    float m;
    memcpy(&m, &mid, 4);
    return fabs(v - (double)m) / (ldexp(1.0, -24) * scale);
}

/* The bf16 neighbour of v other than the one v rounds to (round to nearest
 * even): the value an FP32 evaluation of v on the other side of the tie
 * rounds to. */
static double bf16_other(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u; /* the rounded pattern */
    const uint32_t t = u & 0xffff0000u;                                 /* truncated towards zero */
    const uint32_t o = (r == t) ? t + 0x10000u : t;
    float g;
    memcpy(&g, &o, 4);
    return (double)g;
}

/* BF16-emulating forward (reading L4) in which rounding number `flip` (inputs
 * 0..10, first hidden layer 11..42, second 43..74; -1: none) takes the other
 * bf16 neighbour.  If list != NULL, the roundings whose value lies within
 * tol_ulps of a bf16 tie (bf16_tie_ulps; inputs against xscale[i], hidden
 * pre-activations against the sum of the magnitudes of their terms) are
 * written to list (*nlist entries, at most 75). */
static void forward_flip(const double *P, const double *x, int flip, const double *xscale, double tol_ulps, int *list,
                         int *nlist, double *z)
{
    double xin[NIN], a1[NH], a2[NH];
    int n = 0;
    for (int i = 0; i < NIN; ++i) {
        if (list && bf16_tie_ulps(x[i], xscale[i]) < tol_ulps) list[n++] = i;
        xin[i] = (i == flip) ? bf16_other(x[i]) : orc_bf16(x[i]);
    }
    for (int o = 0; o < NH; ++o) {
        double s = B1(P)[o], mag = fabs(B1(P)[o]);
        for (int i = 0; i < NIN; ++i) {
            s += W1(P)[o * NIN + i] * xin[i];
            mag += fabs(W1(P)[o * NIN + i] * xin[i]);
        }
        if (list && s > 0.0 && bf16_tie_ulps(s, mag) < tol_ulps) list[n++] = NIN + o;
        const double a = s > 0.0 ? s : 0.0;
        a1[o] = (NIN + o == flip && s > 0.0) ? bf16_other(a) : orc_bf16(a);
    }
    for (int o = 0; o < NH; ++o) {
        double s = B2(P)[o], mag = fabs(B2(P)[o]);
        for (int i = 0; i < NH; ++i) {
            s += W2(P)[o * NH + i] * a1[i];
            mag += fabs(W2(P)[o * NH + i] * a1[i]);
        }
        if (list && s > 0.0 && bf16_tie_ulps(s, mag) < tol_ulps) list[n++] = NIN + NH + o;
        const double a = s > 0.0 ? s : 0.0;
        a2[o] = (NIN + NH + o == flip && s > 0.0) ? bf16_other(a) : orc_bf16(a);
    }
    for (int o = 0; o < NOUT; ++o) {
        double s = B3(P)[o];
        for (int i = 0; i < NH; ++i) s += W3(P)[o * NH + i] * a2[i];
        z[o] = s;
    }
    if (nlist) *nlist = n;
}

/* Reading L2 forward; optional buffers receive the values used in the
 * products (after BF16 rounding when bf16 != 0). */
void orc_mlp_forward(const double *P, const double *x, int bf16, double *xq, double *h1, double *h2, double *z)
{
    double xin[NIN], a1[NH], a2[NH];
    for (int i = 0; i < NIN; ++i) xin[i] = bf16 ? orc_bf16(x[i]) : x[i];
    for (int o = 0; o < NH; ++o) {
        double s = B1(P)[o];
        for (int i = 0; i < NIN; ++i) s += W1(P)[o * NIN + i] * xin[i];
        a1[o] = s > 0.0 ? s : 0.0;
        if (bf16) a1[o] = orc_bf16(a1[o]);
    }
    for (int o = 0; o < NH; ++o) {
        double s = B2(P)[o];
        for (int i = 0; i < NH; ++i) s += W2(P)[o * NH + i] * a1[i];
        a2[o] = s > 0.0 ? s : 0.0;
        if (bf16) a2[o] = orc_bf16(a2[o]);
    }
    for (int o = 0; o < NOUT; ++o) {
        double s = B3(P)[o];
        for (int i = 0; i < NH; ++i) s += W3(P)[o * NH + i] * a2[i];
        z[o] = s;
    }
    if (xq) memcpy(xq, xin, sizeof xin);
    if (h1) memcpy(h1, a1, sizeof a1);
    if (h2) memcpy(h2, a2, sizeof a2);
}


/* Smallest distance of the rates 1 + z from the ends of (0, 2) (negative when
 * one is outside). */
static double rate_margin(const double *z)
{
    double m = INFINITY;
    for (int j = 0; j < NOUT; ++j) {
        const double w = 1.0 + z[j];
        const double d = w < 2.0 - w ? w : 2.0 - w;
        if (d < m) m = d;
    }
    return m;
}

/* rates 1 + z, or all 1 when any leaves (0, 2); returns 1 on fallback */
int orc_mlp_rates(const double *z, double *rates)
{
    int bad = 0;
    for (int j = 0; j < NOUT; ++j) {
        const double w = 1.0 + z[j];
        if (!(w > 0.0 && w < 2.0)) bad = 1;
        rates[j] = w;
    }
    if (bad)
        for (int j = 0; j < NOUT; ++j) rates[j] = 1.0;
    return bad;
}

/* macroscopic fields and pre-collision CMs k = T(u) f (Sec. II.B) */
static void node_cms(const double *f, const double *F, double *rho, double *u, double *k)
{
    int c[3 * Q], opp[Q];
    double w[Q];
    orc19_tables(c, w, opp);
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        for (int d = 0; d < 3; ++d) j[d] += f[i] * c[3 * i + d];
    }
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * F[d]) / r;
    *rho = r;
    double T[Q * Q];
    orc19_T(u[0], u[1], u[2], T);
    for (int rr = 0; rr < Q; ++rr) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += T[rr * Q + i] * f[i];
        k[rr] = s;
    }
}

static inline int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

/*
 * One D3Q19 step with learned rates (periodic or y walls, optional F):
 * per node the MLP sets omega_hi from the node's pre-collision CMs, then the
 * collision of Sec. II.B and streaming proceed as in orc19_step.  Returns the
 * number of nodes that fell back to the paper's rates (or -1 on error).
 * Optional per-node outputs (N each), with bf16: tie, how far the node's
 * post-collision populations can move if its FP32 values near a bf16 tie
 * round the other way -- every rounding within tie_ulps of a tie
 * (forward_flip; an input's scale is the sum of |f_i - w_i| over the node
 * divided by rho, times the input's 1/scale) is flipped alone and the largest
 * population change of each flip is summed; margin, the smallest distance of
 * the node's rates from the ends of (0, 2).
 */
int64_t orc19_step_mlp_info(int nx, int ny, int nz, int walls_y, const double *f, double *fnew, const double *F,
                            double omega, const double *P, const double *scales, int bf16, double tie_ulps,
                            double *tie, double *margin)
{
    int c[3 * Q], opp[Q];
    double wt[Q];
    orc19_tables(c, wt, opp);
    const int64_t N = (int64_t)nx * ny * nz;
    int64_t fallbacks = 0;
    int err = 0;
#pragma omp parallel for schedule(static) reduction(+ : fallbacks) reduction(| : err)
    for (int64_t n = 0; n < N; ++n) {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        double fl[Q], fs[Q], Fl[3] = {0.0, 0.0, 0.0}, Kd[Q], rho, u[3], k[Q], xf[NIN], zz[NOUT], rates[NOUT];
        for (int i = 0; i < Q; ++i) fl[i] = f[(int64_t)i * N + n];
        if (F)
            for (int d = 0; d < 3; ++d) Fl[d] = F[(int64_t)d * N + n];
        node_cms(fl, Fl, &rho, u, k);
        orc_mlp_features(rho, k, scales, xf);
        int list[NIN + 2 * NH], nlist = 0;
        if (bf16 && (tie || margin)) {
            double dev = 0.0, xsc[NIN];
            for (int i = 0; i < Q; ++i) dev += fabs(fl[i] - wt[i]);
            for (int j = 0; j < NIN; ++j) xsc[j] = dev / rho / scales[j];
            forward_flip(P, xf, -1, xsc, tie_ulps, list, &nlist, zz);
        } else {
            orc_mlp_forward(P, xf, bf16, NULL, NULL, NULL, zz);
        }
        if (margin) margin[n] = rate_margin(zz);
        fallbacks += orc_mlp_rates(zz, rates);
        orc19_K(omega, 1.0, rates, Kd);
        if (orc19_collide(fl, Fl, Kd, 0, fs, NULL, NULL, NULL) != 0) err |= 1;
        if (tie) {
            /* each listed rounding taken the other way, one at a time: the
             * sum of the largest changes of the node's post-collision
             * populations */
            double eff = 0.0;
            for (int q = 0; q < nlist; ++q) {
                double z2[NOUT], r2[NOUT], K2[Q], f2[Q];
                forward_flip(P, xf, list[q], NULL, 0.0, NULL, NULL, z2);
                orc_mlp_rates(z2, r2);
                orc19_K(omega, 1.0, r2, K2);
                if (orc19_collide(fl, Fl, K2, 0, f2, NULL, NULL, NULL) != 0) err |= 1;
                double d = 0.0;
                for (int i = 0; i < Q; ++i)
                    if (fabs(f2[i] - fs[i]) > d) d = fabs(f2[i] - fs[i]);
                eff += d;
            }
            tie[n] = eff;
        }
        for (int i = 0; i < Q; ++i) {
            int yd = y + c[3 * i + 1];
            if (walls_y && (yd < 0 || yd >= ny)) {
                fnew[(int64_t)opp[i] * N + n] = fs[i];
                continue;
            }
            const int64_t m = wrapi(x + c[3 * i], nx) + (int64_t)nx * (wrapi(yd, ny) + (int64_t)ny * wrapi(z + c[3 * i + 2], nz));
            fnew[(int64_t)i * N + m] = fs[i];
        }
    }
    return err ? -1 : fallbacks;
}

int64_t orc19_step_mlp(int nx, int ny, int nz, int walls_y, const double *f, double *fnew, const double *F,
                       double omega, const double *P, const double *scales, int bf16)
{
    return orc19_step_mlp_info(nx, ny, nz, walls_y, f, fnew, F, omega, P, scales, bf16, 0.0, NULL, NULL);
}

/* The 10 raw moments of reading L5 for one node's populations. */
static void moments10(const double *f, const int *c, double *m)
{
    for (int k = 0; k < 10; ++k) m[k] = 0.0;
    for (int i = 0; i < Q; ++i) {
        const double cx = c[3 * i], cy = c[3 * i + 1], cz = c[3 * i + 2];
        const double mono[10] = {1.0, cx, cy, cz, cx * cx, cy * cy, cz * cz, cx * cy, cx * cz, cy * cz};
        for (int k = 0; k < 10; ++k) m[k] += f[i] * mono[k];
    }
}

/*
 * Reading L5 loss and, if grad != NULL, its exact gradient with respect to
 * the 1737 parameters (FP64 backpropagation through the MLP, the collision
 * -- linear in the learned rates for a fixed input state -- and the
 * streaming).  f: 19*N state at t; target: 10*N moments at t+1 (component k
 * at [k*N + n]); sigma: 10 moment scales.  Nodes that fall back contribute no
 * gradient.  Returns the loss; *fallbacks receives the fallback count.
 */
double orc19_mlp_loss_grad(int nx, int ny, int nz, const double *f, const double *target, double omega,
                           const double *P, const double *scales, const double *sigma, int bf16, double *grad,
                           int64_t *fallbacks)
{
    int c[3 * Q], opp[Q];
    double wt[Q];
    orc19_tables(c, wt, opp);
    const int64_t N = (int64_t)nx * ny * nz;
    double *fstar = (double *)malloc(sizeof(double) * Q * N);
    double *fnext = (double *)malloc(sizeof(double) * Q * N);
    double *gnext = (double *)malloc(sizeof(double) * Q * N);
    int64_t fb = 0;
    /* forward: collide with learned rates */
    for (int64_t n = 0; n < N; ++n) {
        double fl[Q], fs[Q], Fz[3] = {0.0, 0.0, 0.0}, Kd[Q], rho, u[3], k[Q], xf[NIN], zz[NOUT], rates[NOUT];
        for (int i = 0; i < Q; ++i) fl[i] = f[(int64_t)i * N + n];
        node_cms(fl, Fz, &rho, u, k);
        orc_mlp_features(rho, k, scales, xf);
        orc_mlp_forward(P, xf, bf16, NULL, NULL, NULL, zz);
        fb += orc_mlp_rates(zz, rates);
        orc19_K(omega, 1.0, rates, Kd);
        orc19_collide(fl, Fz, Kd, 0, fs, NULL, NULL, NULL);
        for (int i = 0; i < Q; ++i) fstar[(int64_t)i * N + n] = fs[i];
    }
    /* stream (periodic) */
    for (int64_t n = 0; n < N; ++n) {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        for (int i = 0; i < Q; ++i) {
            const int64_t m = wrapi(x + c[3 * i], nx) + (int64_t)nx * (wrapi(y + c[3 * i + 1], ny) + (int64_t)ny * wrapi(z + c[3 * i + 2], nz));
            fnext[(int64_t)i * N + m] = fstar[(int64_t)i * N + n];
        }
    }
    /* loss and dL/df(t+1) */
    double loss = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        double fl[Q], m[10];
        for (int i = 0; i < Q; ++i) fl[i] = fnext[(int64_t)i * N + n];
        moments10(fl, c, m);
        double dm[10];
        for (int k = 0; k < 10; ++k) {
            const double r = (m[k] - target[(int64_t)k * N + n]) / sigma[k];
            loss += r * r;
            dm[k] = 2.0 * r / sigma[k] / (double)N;
        }
        for (int i = 0; i < Q; ++i) {
            const double cx = c[3 * i], cy = c[3 * i + 1], cz = c[3 * i + 2];
            const double mono[10] = {1.0, cx, cy, cz, cx * cx, cy * cy, cz * cz, cx * cy, cx * cz, cy * cz};
            double g = 0.0;
            for (int k = 0; k < 10; ++k) g += dm[k] * mono[k];
            gnext[(int64_t)i * N + n] = g;
        }
    }
    loss /= (double)N;
    if (grad) {
        for (int p = 0; p < NPARAM; ++p) grad[p] = 0.0;
        for (int64_t n = 0; n < N; ++n) {
            const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
            double fl[Q], Fz[3] = {0.0, 0.0, 0.0}, rho, u[3], k[Q], xf[NIN], xq[NIN], h1[NH], h2[NH], zz[NOUT],
                rates[NOUT], gs[Q];
            for (int i = 0; i < Q; ++i) fl[i] = f[(int64_t)i * N + n];
            node_cms(fl, Fz, &rho, u, k);
            orc_mlp_features(rho, k, scales, xf);
            orc_mlp_forward(P, xf, bf16, xq, h1, h2, zz);
            if (orc_mlp_rates(zz, rates)) continue;
            /* adjoint of streaming: dL/df*_i(x) = dL/df_i(x + c_i, t+1) */
            for (int i = 0; i < Q; ++i) {
                const int64_t m = wrapi(x + c[3 * i], nx) + (int64_t)nx * (wrapi(y + c[3 * i + 1], ny) + (int64_t)ny * wrapi(z + c[3 * i + 2], nz));
                gs[i] = gnext[(int64_t)i * N + m];
            }
            /* d(f*)/d(omega_j) = T(u)^-1 e_{10+j} times d(k*_{10+j})/d(omega_j), and
             * d(k*_r)/d(omega_r) = -(k_r - k_eq_r) - R_r/2 (eq. posColl0) */
            double T[Q * Q], Rv[Q];
            orc19_T(u[0], u[1], u[2], T);
            orc19_Rcm(0.0, 0.0, 0.0, Rv);
            double dz[NOUT];
            for (int j = 0; j < NOUT; ++j) {
                const int r = 10 + j;
                /* column r of T^-1 by a dense solve (Gaussian elimination) */
                double A[Q * Q], b[Q], col[Q];
                memcpy(A, T, sizeof A);
                for (int i = 0; i < Q; ++i) b[i] = (i == r) ? 1.0 : 0.0;
                for (int cc = 0; cc < Q; ++cc) {
                    int piv = cc;
                    for (int rr = cc + 1; rr < Q; ++rr)
                        if (fabs(A[rr * Q + cc]) > fabs(A[piv * Q + cc])) piv = rr;
                    if (piv != cc) {
                        for (int q = 0; q < Q; ++q) { double t = A[cc * Q + q]; A[cc * Q + q] = A[piv * Q + q]; A[piv * Q + q] = t; }
                        double t = b[cc]; b[cc] = b[piv]; b[piv] = t;
                    }
                    for (int rr = cc + 1; rr < Q; ++rr) {
                        const double mm = A[rr * Q + cc] / A[cc * Q + cc];
                        for (int q = cc; q < Q; ++q) A[rr * Q + q] -= mm * A[cc * Q + q];
                        b[rr] -= mm * b[cc];
                    }
                }
                for (int rr = Q - 1; rr >= 0; --rr) {
                    double s = b[rr];
                    for (int q = rr + 1; q < Q; ++q) s -= A[rr * Q + q] * col[q];
                    col[rr] = s / A[rr * Q + rr];
                }
                const double keq_r = (r >= 16) ? rho / 9.0 : 0.0;
                const double dk = -(k[r] - keq_r) - 0.5 * Rv[r];
                double g = 0.0;
                for (int i = 0; i < Q; ++i) g += gs[i] * col[i];
                dz[j] = g * dk; /* omega = 1 + z */
            }
            /* MLP backward */
            double *gW1 = grad, *gB1 = grad + NH * NIN, *gW2 = gB1 + NH, *gB2 = gW2 + NH * NH, *gW3 = gB2 + NH,
                   *gB3 = gW3 + NOUT * NH;
            double dh2[NH], dh1[NH];
            for (int o = 0; o < NOUT; ++o) {
                gB3[o] += dz[o];
                for (int i = 0; i < NH; ++i) gW3[o * NH + i] += dz[o] * h2[i];
            }
            for (int i = 0; i < NH; ++i) {
                double s = 0.0;
                for (int o = 0; o < NOUT; ++o) s += W3(P)[o * NH + i] * dz[o];
                dh2[i] = h2[i] > 0.0 ? s : 0.0; /* ReLU: slope 1 where active */
            }
            for (int o = 0; o < NH; ++o) {
                gB2[o] += dh2[o];
                for (int i = 0; i < NH; ++i) gW2[o * NH + i] += dh2[o] * h1[i];
            }
            for (int i = 0; i < NH; ++i) {
                double s = 0.0;
                for (int o = 0; o < NH; ++o) s += W2(P)[o * NH + i] * dh2[o];
                dh1[i] = h1[i] > 0.0 ? s : 0.0;
            }
            for (int o = 0; o < NH; ++o) {
                gB1[o] += dh1[o];
                for (int i = 0; i < NIN; ++i) gW1[o * NIN + i] += dh1[o] * xq[i];
            }
        }
    }
    free(fstar);
    free(fnext);
    free(gnext);
    if (fallbacks) *fallbacks = fb;
    return loss;
}
