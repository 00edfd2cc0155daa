// Two-phase flow with a conservative phase field: per-node device arithmetic.
//
// Not in the paper (its multiphase models are Shan-Chen and the colour
// gradient).  Interface: conservative Allen-Cahn equation (Chiu & Lin, J.
// Comput. Phys. 230, 2011) in the lattice Boltzmann form of Fakhari et al.
// (Phys. Rev. E 96, 2017) on D3Q7.  Flow: pressure-based populations g
// (zeroth moment p/cs^2, first moment rho u, rho = rho(phi); He, Chen & Zhang,
// J. Comput. Phys. 152, 1999; Liang et al., Phys. Rev. E 97, 2018) collided
// with the paper's CM scheme (Sec. II.B, forcing of App. B), in deviation
// variables s_i = g_i - w_i.
//
// Per node, given phi at the 19 stencil nodes x + c_i:
//   grad phi = 3 sum_i w_i c_i phi(x + c_i), lap phi = 6 sum_i w_i (phi(x + c_i) - phi(x));
//   rho = rho_l + phi (rho_h - rho_l);  mu = 4 beta phi (phi - 1)(phi - 1/2) - kappa lap phi;
//   F = mu grad phi;  u = (sum g c + F/2) / rho;  S0 = u . grad rho;  Pi = sum g + S0/2;
//   equilibrium raw moments = those of the paper's equilibrium at density rho
//   plus (Pi - rho) times the rest weights (eq_raw_deviation(Pi - 1, rho, u));
//   sources in CM rows: zeroth S0, first F - u S0, second
//   C = cs^2 (u grad rho + grad rho u + (u.grad rho) I), third as App. B from F;
//   rates: 1 on rows 0..4 and 10..18, omega on rows 5..9.
// Phase (D3Q7, cs^2 = 1/4, order rest, -x, -y, -z, +x, +y, +z):
//   h* = h - w_phi (h - phi w (1 + c.u/cs^2)) + (1 - w_phi/2) w (4/W) phi (1 - phi) c.n,
//   n = grad phi / |grad phi| (0 where grad phi = 0).
#pragma once

#include "d3q19_cm.hpp"

namespace lbm {

__host__ __device__ constexpr int cx7(int i) { return i == 1 ? -1 : (i == 4 ? 1 : 0); }
__host__ __device__ constexpr int cy7(int i) { return i == 2 ? -1 : (i == 5 ? 1 : 0); }
__host__ __device__ constexpr int cz7(int i) { return i == 3 ? -1 : (i == 6 ? 1 : 0); }
__host__ __device__ constexpr double w7(int i) { return i == 0 ? 0.25 : 0.125; }

// Constants of the two-phase model, precomputed on the host.
struct PhaseConst {
    double rho_l, drho;  // rho = rho_l + phi drho
    double beta, kappa;  // 12 sigma / W, 3 sigma W / 2
    double four_over_w;  // 4 / W
    double omega;        // flow shear rate (rows 5..9)
    double omega_phi;    // phase relaxation rate, 1 / (M / cs^2 + 1/2)
};

// Gradient and Laplacian of phi from its stencil values phin[i] = phi(x + c_i).
template <class R> __host__ __device__ inline void phase_derivs(const R phin[19], R& gx, R& gy, R& gz, R& lap)
{
    const R w1 = R(1) / R(18), w2 = R(1) / R(36);
    // axes: 1..3 negative, 10..12 positive; face diagonals weight 1/36
    R ax = phin[10] - phin[1], ay = phin[11] - phin[2], az = phin[12] - phin[3];
    // xy diagonals 4(-,-) 5(-,+) 13(+,+) 14(+,-); xz 6(-,-) 7(-,+) 15(+,+) 16(+,-); yz 8(-,-) 9(-,+) 17(+,+) 18(+,-)
    const R dxy_x = (phin[13] + phin[14]) - (phin[4] + phin[5]);
    const R dxy_y = (phin[13] + phin[5]) - (phin[4] + phin[14]);
    const R dxz_x = (phin[15] + phin[16]) - (phin[6] + phin[7]);
    const R dxz_z = (phin[15] + phin[7]) - (phin[6] + phin[16]);
    const R dyz_y = (phin[17] + phin[18]) - (phin[8] + phin[9]);
    const R dyz_z = (phin[17] + phin[9]) - (phin[8] + phin[18]);
    gx = R(3) * (w1 * ax + w2 * (dxy_x + dxz_x));
    gy = R(3) * (w1 * ay + w2 * (dxy_y + dyz_y));
    gz = R(3) * (w1 * az + w2 * (dxz_z + dyz_z));
    R s1 = R(0), s2 = R(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        if (i <= 3 || (i >= 10 && i <= 12))
            s1 += phin[i];
        else
            s2 += phin[i];
    }
    lap = R(6) * (w1 * (s1 - R(6) * phin[0]) + w2 * (s2 - R(12) * phin[0]));
}

// Macroscopic quantities of the flow at one node.
template <class R> struct PhaseMacro {
    R rho, ux, uy, uz, Fx, Fy, Fz, grx, gry, grz, S0, dPi; // dPi = Pi - 1
};

template <class R>
__host__ __device__ inline void phase_macro(const RawMoments<R>& m, const R phin[19], const PhaseConst& pc,
                                            PhaseMacro<R>& o, R& gx, R& gy, R& gz)
{
    R lap;
    phase_derivs(phin, gx, gy, gz, lap);
    const R phi = phin[0];
    const R drho = (R)pc.drho;
    o.rho = (R)pc.rho_l + phi * drho;
    const R mu = R(4) * (R)pc.beta * phi * (phi - R(1)) * (phi - R(0.5)) - (R)pc.kappa * lap;
    o.Fx = mu * gx;
    o.Fy = mu * gy;
    o.Fz = mu * gz;
    const R ir = R(1) / o.rho;
    o.ux = (m.m100 + R(0.5) * o.Fx) * ir;
    o.uy = (m.m010 + R(0.5) * o.Fy) * ir;
    o.uz = (m.m001 + R(0.5) * o.Fz) * ir;
    o.grx = drho * gx;
    o.gry = drho * gy;
    o.grz = drho * gz;
    o.S0 = o.ux * o.grx + o.uy * o.gry + o.uz * o.grz;
    o.dPi = m.m000 + R(0.5) * o.S0;
}

// Collision of the flow deviations s (in place) given the node's macroscopic state.
template <class R> __host__ __device__ inline void phase_collide_g(R s[19], const RawMoments<R>& m, const PhaseMacro<R>& o, R omega)
{
    const R cs2 = R(1) / R(3);
    RawMoments<R> e;
    eq_raw_deviation(o.dPi, o.rho, o.ux, o.uy, o.uz, e);
    // non-equilibrium raw moments (third and fourth order: relaxed at rate 1,
    // so only their equilibrium and sources survive)
    RawMoments<R> n;
    n.m000 = m.m000 - e.m000;
    n.m100 = m.m100 - e.m100;
    n.m010 = m.m010 - e.m010;
    n.m001 = m.m001 - e.m001;
    n.m200 = m.m200 - e.m200;
    n.m020 = m.m020 - e.m020;
    n.m002 = m.m002 - e.m002;
    n.m110 = m.m110 - e.m110;
    n.m101 = m.m101 - e.m101;
    n.m011 = m.m011 - e.m011;
    n.m210 = n.m120 = n.m201 = n.m102 = n.m021 = n.m012 = n.m220 = n.m202 = n.m022 = R(0);
    shift_all(n, -o.ux, -o.uy, -o.uz);
    const R k5 = n.m200 - n.m020, k6 = n.m020 - n.m002;
    // second-order source C (central)
    const R ug = o.S0;
    const R Cxx = cs2 * (R(2) * o.ux * o.grx + ug), Cyy = cs2 * (R(2) * o.uy * o.gry + ug),
            Czz = cs2 * (R(2) * o.uz * o.grz + ug);
    const R Cxy = cs2 * (o.ux * o.gry + o.uy * o.grx), Cxz = cs2 * (o.ux * o.grz + o.uz * o.grx),
            Cyz = cs2 * (o.uy * o.grz + o.uz * o.gry);
    const R w1 = R(1) - omega, wh = R(1) - R(0.5) * omega;
    const R s4 = R(0.5) * (Cxx + Cyy + Czz);       // k4: rate 1
    const R s5 = w1 * k5 + wh * (Cxx - Cyy);
    const R s6 = w1 * k6 + wh * (Cyy - Czz);
    RawMoments<R> p;
    p.m000 = R(0.5) * o.S0;
    p.m100 = R(0.5) * (o.Fx - o.ux * o.S0);
    p.m010 = R(0.5) * (o.Fy - o.uy * o.S0);
    p.m001 = R(0.5) * (o.Fz - o.uz * o.S0);
    const R third = R(1) / R(3);
    p.m200 = third * (s4 + R(2) * s5 + s6);
    p.m020 = third * (s4 - s5 + s6);
    p.m002 = third * (s4 - s5 - R(2) * s6);
    p.m110 = w1 * n.m110 + wh * Cxy;
    p.m101 = w1 * n.m101 + wh * Cxz;
    p.m011 = w1 * n.m011 + wh * Cyz;
    const R hf = R(0.5) * cs2;
    p.m210 = hf * o.Fy;
    p.m120 = hf * o.Fx;
    p.m201 = hf * o.Fz;
    p.m102 = hf * o.Fx;
    p.m021 = hf * o.Fz;
    p.m012 = hf * o.Fy;
    p.m220 = p.m202 = p.m022 = R(0);
    // back to raw moments (the central zeroth source shifts into the higher
    // raw moments), add the equilibrium, populations
    shift_all(p, o.ux, o.uy, o.uz);
    p.m000 += e.m000;
    p.m100 += e.m100;
    p.m010 += e.m010;
    p.m001 += e.m001;
    p.m200 += e.m200;
    p.m020 += e.m020;
    p.m002 += e.m002;
    p.m110 += e.m110;
    p.m101 += e.m101;
    p.m011 += e.m011;
    p.m210 += e.m210;
    p.m120 += e.m120;
    p.m201 += e.m201;
    p.m102 += e.m102;
    p.m021 += e.m021;
    p.m012 += e.m012;
    p.m220 += e.m220;
    p.m202 += e.m202;
    p.m022 += e.m022;
    pops_from_raw(p, s);
}

// Collision of the seven phase populations h (in place).
template <class R>
__host__ __device__ inline void phase_collide_h(R h[7], R phi, R gx, R gy, R gz, R ux, R uy, R uz, const PhaseConst& pc)
{
    const R g2 = gx * gx + gy * gy + gz * gz;
    R nx = R(0), ny = R(0), nz = R(0);
    if (g2 > R(0)) {
        const R ig = R(1) / sqrt(g2);
        nx = gx * ig;
        ny = gy * ig;
        nz = gz * ig;
    }
    const R wp = (R)pc.omega_phi, keep = R(1) - wp, fw = R(1) - R(0.5) * wp;
    const R theta = (R)pc.four_over_w * phi * (R(1) - phi);
    const R a = R(0.125) * phi, b = R(0.125) * fw * theta;
    // rest: equilibrium phi/4, no forcing
    h[0] = keep * h[0] + wp * (R(0.25) * phi);
    // +-x, +-y, +-z: h_eq = phi/8 (1 +- 4 u_d), forcing +- (1/8) theta n_d
    const R ex = R(4) * ux, ey = R(4) * uy, ez = R(4) * uz;
    h[1] = keep * h[1] + wp * (a * (R(1) - ex)) - b * nx;
    h[4] = keep * h[4] + wp * (a * (R(1) + ex)) + b * nx;
    h[2] = keep * h[2] + wp * (a * (R(1) - ey)) - b * ny;
    h[5] = keep * h[5] + wp * (a * (R(1) + ey)) + b * ny;
    h[3] = keep * h[3] + wp * (a * (R(1) - ez)) - b * nz;
    h[6] = keep * h[6] + wp * (a * (R(1) + ez)) + b * nz;
}

} // namespace lbm
