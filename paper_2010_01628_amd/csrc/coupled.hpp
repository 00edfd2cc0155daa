// Launchers of the coupled lattices (two-phase phase field; magnetic field).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.hpp"
#include "phase_cm.hpp"

namespace lbm {

// One step of the two-phase lattice: phi = sum h into `phi`, then the fused
// flow + phase collide-stream from (gsrc, hsrc) into (gdst, hdst).
void launch_phase_step(int precision, bool nt, const void* gsrc, void* gdst, const void* hsrc, void* hdst, void* phi,
                       const Geom& g, const PhaseConst& pc, dim3 grid, dim3 block, hipStream_t st);
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

} // namespace lbm
