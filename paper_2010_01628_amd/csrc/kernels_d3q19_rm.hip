// D3Q19 step kernels with the raw-moment collision (App. C, N = I) for every
// storage precision.  Initialisation, import/export and moments are those of
// the central-moment lattice (same populations, same equilibrium).
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

} // namespace lbm
