// Launchers of the coupled lattices (two-phase phase field; magnetic field).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.hpp"
#include "phase_cm.hpp"

namespace lbm {

// Constants of the magnetic lattice.
struct MhdConst {
    double omega_m;   // 1 / (eta / cs^2 + 1/2), cs^2 = 1/4
    double b_wall[3]; // field imposed at the y walls
};

// Constants of the colour-gradient lattice.
struct CgConst {
    double omega;            // shear rate
    double alpha_r, alpha_b; // rest fractions of the colours (App. E)
    double A;                // perturbation amplitude A_r + A_b
    double beta;             // recolouring parameter
    double g[3];             // gravity; body force (rho - rho_ref) g
    double rho_ref;
};

// One step of the two-phase lattice: phi = sum h into `phi`, then the fused
// flow + phase collide-stream from (gsrc, hsrc) into (gdst, hdst).
// grid/block: k_phase_sum and, when rblock.x == 0, k_phase_step on geometry g;
// rblock.x > 0: k_phase_step_rows on gr with rgrid/rblock (whole x rows of
// nx <= 256 nodes, periodic)
void launch_phase_step(int precision, bool nt, const void* gsrc, void* gdst, const void* hsrc, void* hdst, void* phi,
                       const Geom& g, const PhaseConst& pc, dim3 grid, dim3 block, const Geom& gr, dim3 rgrid,
                       dim3 rblock, hipStream_t st);
void launch_phase_init(int precision, void* gbuf, void* hbuf, const Geom& g, const PhaseConst& pc, const double* phi,
                       const double* p, const double* u, dim3 grid, dim3 block, hipStream_t st);
// phi (scratch, refreshed from hsrc), then macroscopic fields and partials.
void launch_phase_fields(int precision, const void* gsrc, const void* hsrc, void* phi, const Geom& g,
                         const PhaseConst& pc, double* phi_out, double* p_out, double* rho_out, double* u_out,
                         double* partials, dim3 grid, dim3 block, hipStream_t st);
void launch_phase_get_h(int precision, const void* hbuf, const Geom& g, double* out, dim3 grid, dim3 block,
                        hipStream_t st);
void launch_phase_set_h(int precision, void* hbuf, const Geom& g, const double* in, dim3 grid, dim3 block,
                        hipStream_t st);

// One step of the magnetic coupling (flow + magnetic lattice, one launch).
void launch_mhd_step(int precision, bool walls, bool nt, const void* fsrc, void* fdst, const void* gsrc, void* gdst,
                     const Geom& g, const Phys& ph, const MhdConst& mc, dim3 grid, dim3 block, hipStream_t st);
void launch_mhd_init(int precision, bool walls, void* fbuf, void* gbuf, const Geom& g, double rho0, const MhdConst& mc,
                     const double* rho, const double* u, const double* b, dim3 grid, dim3 block, hipStream_t st);
void launch_mhd_fields(int precision, bool walls, const void* fsrc, const void* gsrc, const Geom& g, const Phys& ph,
                       const MhdConst& mc, double* rho, double* u, double* b, double* j, double* partials, dim3 grid,
                       dim3 block, hipStream_t st);
void launch_mhd_get_g(int precision, bool walls, const void* gbuf, const Geom& g, const MhdConst& mc, double* out,
                      dim3 grid, dim3 block, hipStream_t st);
void launch_mhd_set_g(int precision, bool walls, void* gbuf, const Geom& g, const MhdConst& mc, const double* in,
                      dim3 grid, dim3 block, hipStream_t st);

// Shan-Chen two-phase flow: psi from the pulled densities into `psi`, then
// the fused step with the interaction force.
void launch_sc_step(int precision, bool general, bool nt, const void* src, void* dst, void* psi, const Geom& g,
                    const Phys& ph, double G, dim3 grid, dim3 block, hipStream_t st);
// psi refreshed from src, then rho, force-shifted u and the partial sums.
void launch_sc_fields(int precision, const void* src, void* psi, const Geom& g, const Phys& ph, double G, double* rho,
                      double* u, double* partials, dim3 grid, dim3 block, hipStream_t st);

// Colour-gradient two-phase flow: phi from the pulled colours into `phi`,
// then the fused step of both colours.
void launch_cg_step(int precision, bool walls, bool nt, const void* rsrc, void* rdst, const void* bsrc, void* bdst,
                    void* phi, const Geom& g, const CgConst& cc, dim3 grid, dim3 block, hipStream_t st);
void launch_cg_init(int precision, bool walls, void* red, void* blue, const Geom& g, const CgConst& cc,
                    const double* rho_r, const double* rho_b, const double* u, dim3 grid, dim3 block, hipStream_t st);
void launch_cg_fields(int precision, bool walls, const void* red, const void* blue, const Geom& g, const CgConst& cc,
                      double* rho, double* u, double* rho_r, double* rho_b, double* partials, dim3 grid, dim3 block,
                      hipStream_t st);

} // namespace lbm
