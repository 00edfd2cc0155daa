// D3Q27 central-moment collision for gfx950 -- device functions.
//
// The D3Q27 lattice of App. D (velocity order with opposite(i) = i +- 13) is
// the tensor product of three D1Q3 lattices, so every moment with exponents
// (p, q, r) <= 2 exists and populations <-> raw moments <-> central moments
// factor into 1-D transforms along x, y and z over a 3x3x3 cube:
//   populations (cx = -1, 0, +1)  ->  raw (p = 0, 1, 2):  (s- + s0 + s+, s+ - s-, s+ + s-)
//   raw -> central: binomial shift by -u per axis; central -> raw: by +u.
// Equilibrium: product of D1Q3 equilibria (central moments rho (1/3)^#squares,
// zero if any exponent is 1); rates: omega on the five deviatoric second-order
// moments, 1 on everything else; forcing CMs by the Gaussian rule
// R_pqr = sum_a p_a F_a k^eq_{pqr - e_a} / rho.  As for D3Q19 everything is
// carried as deviations from the rest state rho0 w.
#pragma once

#include "d3q19_cm.hpp"

namespace lbm {

constexpr int Q27 = 27;

__host__ __device__ constexpr int cx27(int i)
{
    constexpr int v[27] = {0, -1, 0, 0, -1, -1, -1, -1, 0, 0, -1, -1, -1, -1, 1, 0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1};
    return v[i];
}
__host__ __device__ constexpr int cy27(int i)
{
    constexpr int v[27] = {0, 0, -1, 0, -1, 1, 0, 0, -1, -1, -1, -1, 1, 1, 0, 1, 0, 1, -1, 0, 0, 1, 1, 1, 1, -1, -1};
    return v[i];
}
__host__ __device__ constexpr int cz27(int i)
{
    constexpr int v[27] = {0, 0, 0, -1, 0, 0, -1, 1, -1, 1, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int opp27(int i) { return i == 0 ? 0 : (i <= 13 ? i + 13 : i - 13); }
__host__ __device__ constexpr double w27(int i)
{
    return (cx27(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0) * (cy27(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0) *
           (cz27(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0);
}
// population index of velocity (a, b, c), each in {-1, 0, 1}
__host__ __device__ constexpr int idx27(int a, int b, int c)
{
    for (int i = 0; i < 27; ++i)
        if (cx27(i) == a && cy27(i) == b && cz27(i) == c) return i;
    return -1;
}

// m[p][q][r] cube helpers ---------------------------------------------------
template <class R> struct Cube {
    R v[3][3][3];
};

// populations (as s[i]) -> deviation raw moments
template <class R> __host__ __device__ inline void cube_from_pops(const R s[27], Cube<R>& m)
{
    // along x: (cx = -1, 0, 1) -> (p = 0, 1, 2)
    R t[3][3][3]; // t[p][cy+1][cz+1]
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R sm = s[idx27(-1, b - 1, c - 1)], s0 = s[idx27(0, b - 1, c - 1)], sp = s[idx27(1, b - 1, c - 1)];
            t[0][b][c] = (sm + sp) + s0;
            t[1][b][c] = sp - sm;
            t[2][b][c] = sp + sm;
        }
    R t2[3][3][3]; // t2[p][q][cz+1]
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R sm = t[p][0][c], s0 = t[p][1][c], sp = t[p][2][c];
            t2[p][0][c] = (sm + sp) + s0;
            t2[p][1][c] = sp - sm;
            t2[p][2][c] = sp + sm;
        }
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const R sm = t2[p][q][0], s0 = t2[p][q][1], sp = t2[p][q][2];
            m.v[p][q][0] = (sm + sp) + s0;
            m.v[p][q][1] = sp - sm;
            m.v[p][q][2] = sp + sm;
        }
}

// inverse of cube_from_pops
template <class R> __host__ __device__ inline void pops_from_cube(const Cube<R>& m, R s[27])
{
    const R h = R(0.5);
    R t2[3][3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const R m0 = m.v[p][q][0], m1 = m.v[p][q][1], m2 = m.v[p][q][2];
            t2[p][q][0] = h * (m2 - m1);
            t2[p][q][1] = m0 - m2;
            t2[p][q][2] = h * (m2 + m1);
        }
    R t[3][3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R m0 = t2[p][0][c], m1 = t2[p][1][c], m2 = t2[p][2][c];
            t[p][0][c] = h * (m2 - m1);
            t[p][1][c] = m0 - m2;
            t[p][2][c] = h * (m2 + m1);
        }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R m0 = t[0][b][c], m1 = t[1][b][c], m2 = t[2][b][c];
            s[idx27(-1, b - 1, c - 1)] = h * (m2 - m1);
            s[idx27(0, b - 1, c - 1)] = m0 - m2;
            s[idx27(1, b - 1, c - 1)] = h * (m2 + m1);
        }
}

// binomial shift of every chain along each axis by (a, b, c)
template <class R> __host__ __device__ inline void cube_shift(Cube<R>& m, R a, R b, R c)
{
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int r = 0; r < 3; ++r) shift3(m.v[0][q][r], m.v[1][q][r], m.v[2][q][r], a);
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int r = 0; r < 3; ++r) shift3(m.v[p][0][r], m.v[p][1][r], m.v[p][2][r], b);
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) shift3(m.v[p][q][0], m.v[p][q][1], m.v[p][q][2], c);
}

// raw moments of the tensor-product equilibrium minus those of the rest state:
// rho prod mu_e(u_a) - rho0 prod W_e, with mu = (1, u, u^2 + 1/3), W = (1, 0, 1/3),
// telescoped so every term is small.
template <class R> __host__ __device__ inline void cube_eq_deviation(R drho, R rho, R ux, R uy, R uz, Cube<R>& d)
{
    const R t = R(1) / R(3);
    const R W[3] = {R(1), R(0), t};
    const R dx[3] = {R(0), ux, ux * ux}, dy[3] = {R(0), uy, uy * uy}, dz[3] = {R(0), uz, uz * uz};
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const R mx = W[p] + dx[p], my = W[q] + dy[q];
                // mu_p mu_q mu_r - W_p W_q W_r = dx mu_q mu_r + W_p dy mu_r + W_p W_q dz
                const R prod = dx[p] * my * (W[r] + dz[r]) + W[p] * dy[q] * (W[r] + dz[r]) + W[p] * W[q] * dz[r];
                d.v[p][q][r] = drho * (W[p] * W[q] * W[r]) + rho * prod;
                (void)mx;
            }
}

// One D3Q27 collision on deviations s (in place).
template <class R>
__host__ __device__ inline void collide_cm27(R s[27], R rho0, R Fx, R Fy, R Fz, R omega, NodeMacro<R>& mac)
{
    const R third = R(1) / R(3), ninth = R(1) / R(9);
    Cube<R> m;
    cube_from_pops(s, m);
    const R drho = m.v[0][0][0];
    const R rho = rho0 + drho;
    const R irho = R(1) / rho;
    const R ux = (m.v[1][0][0] + R(0.5) * Fx) * irho;
    const R uy = (m.v[0][1][0] + R(0.5) * Fy) * irho;
    const R uz = (m.v[0][0][1] + R(0.5) * Fz) * irho;
    mac.rho = rho;
    mac.ux = ux;
    mac.uy = uy;
    mac.uz = uz;
    Cube<R> e;
    cube_eq_deviation(drho, rho, ux, uy, uz, e);
    // non-equilibrium raw moments, then central
    Cube<R> n;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int r = 0; r < 3; ++r) n.v[p][q][r] = m.v[p][q][r] - e.v[p][q][r];
    n.v[0][0][0] = R(0);
    n.v[1][0][0] = R(-0.5) * Fx;
    n.v[0][1][0] = R(-0.5) * Fy;
    n.v[0][0][1] = R(-0.5) * Fz;
    // only second-order central moments survive relaxation (rate omega on the
    // deviators, 1 elsewhere); they need only moments of order <= 2
    const R k200 = n.v[2][0][0] + ux * (ux * n.v[0][0][0] - R(2) * n.v[1][0][0]);
    const R k020 = n.v[0][2][0] + uy * (uy * n.v[0][0][0] - R(2) * n.v[0][1][0]);
    const R k002 = n.v[0][0][2] + uz * (uz * n.v[0][0][0] - R(2) * n.v[0][0][1]);
    const R k110 = n.v[1][1][0] - ux * n.v[0][1][0] - uy * n.v[1][0][0];
    const R k101 = n.v[1][0][1] - ux * n.v[0][0][1] - uz * n.v[1][0][0];
    const R k011 = n.v[0][1][1] - uy * n.v[0][0][1] - uz * n.v[0][1][0];
    const R w1 = R(1) - omega;
    // post-collision non-equilibrium CMs
    Cube<R> p;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) p.v[a][b][c] = R(0);
    p.v[1][0][0] = R(0.5) * Fx;
    p.v[0][1][0] = R(0.5) * Fy;
    p.v[0][0][1] = R(0.5) * Fz;
    const R d1 = w1 * (k200 - k020), d2 = w1 * (k200 - k002); // trace relaxes with rate 1 -> 0
    p.v[2][0][0] = third * (d1 + d2);
    p.v[0][2][0] = p.v[2][0][0] - d1;
    p.v[0][0][2] = p.v[2][0][0] - d2;
    p.v[1][1][0] = w1 * k110;
    p.v[1][0][1] = w1 * k101;
    p.v[0][1][1] = w1 * k011;
    // half the forcing CMs on the equilibrated higher orders
    const R hf3 = R(0.5) * third, hf5 = R(0.5) * ninth;
    p.v[2][1][0] = hf3 * Fy;
    p.v[1][2][0] = hf3 * Fx;
    p.v[2][0][1] = hf3 * Fz;
    p.v[1][0][2] = hf3 * Fx;
    p.v[0][2][1] = hf3 * Fz;
    p.v[0][1][2] = hf3 * Fy;
    p.v[2][2][1] = hf5 * Fz;
    p.v[2][1][2] = hf5 * Fy;
    p.v[1][2][2] = hf5 * Fx;
    cube_shift(p, ux, uy, uz);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) p.v[a][b][c] += e.v[a][b][c];
    p.v[0][0][0] = drho;
    pops_from_cube(p, s);
}

// Raw-moment variant (N = I): the same rates applied to un-shifted moments of
// the cube, towards the raw equilibrium, with the raw forcing moments of the
// Gaussian rule R_pqr = sum_a p_a F_a mu_{pqr - e_a}, mu = (1, u, u^2 + 1/3)
// per axis.  No binomial shifts.
template <class R>
__host__ __device__ inline void collide_rm27(R s[27], R rho0, R Fx, R Fy, R Fz, R omega, NodeMacro<R>& mac)
{
    const R third = R(1) / R(3);
    Cube<R> m;
    cube_from_pops(s, m);
    const R drho = m.v[0][0][0];
    const R rho = rho0 + drho;
    const R irho = R(1) / rho;
    const R ux = (m.v[1][0][0] + R(0.5) * Fx) * irho;
    const R uy = (m.v[0][1][0] + R(0.5) * Fy) * irho;
    const R uz = (m.v[0][0][1] + R(0.5) * Fz) * irho;
    mac.rho = rho;
    mac.ux = ux;
    mac.uy = uy;
    mac.uz = uz;
    Cube<R> e;
    cube_eq_deviation(drho, rho, ux, uy, uz, e);
    const R mx[3] = {R(1), ux, ux * ux + third}, my[3] = {R(1), uy, uy * uy + third},
            mz[3] = {R(1), uz, uz * uz + third};
    Cube<R> f; // raw forcing moments
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                R v = R(0);
                if (a) v += R(a) * Fx * (mx[a - 1] * my[b] * mz[c]);
                if (b) v += R(b) * Fy * (mx[a] * my[b - 1] * mz[c]);
                if (c) v += R(c) * Fz * (mx[a] * my[b] * mz[c - 1]);
                f.v[a][b][c] = v;
            }
    // rate 1 everywhere but the deviatoric second-order moments
    Cube<R> p;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) p.v[a][b][c] = e.v[a][b][c] + R(0.5) * f.v[a][b][c];
    const R w1 = R(1) - omega, h1 = R(1) - R(0.5) * omega;
    p.v[1][1][0] = e.v[1][1][0] + w1 * (m.v[1][1][0] - e.v[1][1][0]) + h1 * f.v[1][1][0];
    p.v[1][0][1] = e.v[1][0][1] + w1 * (m.v[1][0][1] - e.v[1][0][1]) + h1 * f.v[1][0][1];
    p.v[0][1][1] = e.v[0][1][1] + w1 * (m.v[0][1][1] - e.v[0][1][1]) + h1 * f.v[0][1][1];
    const R n200 = m.v[2][0][0] - e.v[2][0][0], n020 = m.v[0][2][0] - e.v[0][2][0], n002 = m.v[0][0][2] - e.v[0][0][2];
    const R t = (e.v[2][0][0] + e.v[0][2][0] + e.v[0][0][2]) + R(0.5) * (f.v[2][0][0] + f.v[0][2][0] + f.v[0][0][2]);
    const R d1 = (e.v[2][0][0] - e.v[0][2][0]) + w1 * (n200 - n020) + h1 * (f.v[2][0][0] - f.v[0][2][0]);
    const R d2 = (e.v[2][0][0] - e.v[0][0][2]) + w1 * (n200 - n002) + h1 * (f.v[2][0][0] - f.v[0][0][2]);
    p.v[2][0][0] = third * (t + d1 + d2);
    p.v[0][2][0] = p.v[2][0][0] - d1;
    p.v[0][0][2] = p.v[2][0][0] - d2;
    p.v[0][0][0] = drho;
    pops_from_cube(p, s);
}

template <class R> __host__ __device__ inline void equilibrium_deviation27(R rho, R rho0, R ux, R uy, R uz, R s[27])
{
    Cube<R> e;
    cube_eq_deviation(rho - rho0, rho, ux, uy, uz, e);
    pops_from_cube(e, s);
}

} // namespace lbm
