// Step kernels with the raw-moment collision (N = I): D3Q19 (App. C) for every
// storage precision, D3Q27 for FP64 and FP32.  Initialisation, import/export
// and moments are those of the central-moment lattices (same populations,
// same equilibria).
#include "lattice_kernels.hpp"

namespace lbm {

void launch_step_q19rm(int precision, int pattern, bool walls, bool general, bool nt, const void* src, void* dst,
                       const Geom& g, const Phys& ph, dim3 grid, dim3 block, hipStream_t st)
{
    switch (precision) {
    case PREC_FP64: Launch<LatD3Q19RM, double>::step(pattern, walls, general, nt, src, dst, g, ph, grid, block, st); break;
    case PREC_FP32: Launch<LatD3Q19RM, float>::step(pattern, walls, general, nt, src, dst, g, ph, grid, block, st); break;
    case PREC_FP16: Launch<LatD3Q19RM, _Float16>::step(pattern, walls, general, nt, src, dst, g, ph, grid, block, st); break;
    default: Launch<LatD3Q19RM, bf16_t>::step(pattern, walls, general, nt, src, dst, g, ph, grid, block, st); break;
    }
}

void launch_step_q27rm(int precision, int pattern, bool walls, bool nt, const void* src, void* dst, const Geom& g,
                       const Phys& ph, dim3 grid, dim3 block, hipStream_t st)
{
    if (precision == PREC_FP64) Launch<LatD3Q27RM, double>::step(pattern, walls, false, nt, src, dst, g, ph, grid, block, st);
    else Launch<LatD3Q27RM, float>::step(pattern, walls, false, nt, src, dst, g, ph, grid, block, st);
}

} // namespace lbm
