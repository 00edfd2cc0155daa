// D3Q19 instantiations of the lattice kernels (FP64, FP32, FP16, BF16 storage;
// BF16 with stochastic rounding).
#include "lattice_kernels.hpp"

namespace lbm {

template <class F> static void by_precision19(int precision, F&& f)
{
    switch (precision) {
    case PREC_FP64: f(Launch<LatD3Q19, double>{}); break;
    case PREC_FP32: f(Launch<LatD3Q19, float>{}); break;
    case PREC_FP16: f(Launch<LatD3Q19, _Float16>{}); break;
    case PREC_BF16SR: f(Launch<LatD3Q19, bf16sr_t>{}); break;
    default: f(Launch<LatD3Q19, bf16_t>{}); break;
    }
}

#define LBM_DEFINE_LAUNCHERS(SUFFIX, BY)                                                                             \
    void launch_step_##SUFFIX(int precision, int pattern, bool walls, bool general, bool nt, const void* src,        \
                              void* dst, const Geom& g, const Phys& ph, dim3 grid, dim3 block, hipStream_t st)      \
    {                                                                                                                \
        BY(precision, [&](auto L) { L.step(pattern, walls, general, nt, src, dst, g, ph, grid, block, st); });    \
    }                                                                                                                \
    void launch_init_##SUFFIX(int precision, int pattern, bool walls, void* buf, const Geom& g, double rho0,         \
                              const double* rho, const double* u, dim3 grid, dim3 block, hipStream_t st)            \
    {                                                                                                                \
        BY(precision, [&](auto L) { L.init(pattern, walls, buf, g, rho0, rho, u, grid, block, st); });             \
    }                                                                                                                \
    void launch_set_pops_##SUFFIX(int precision, int pattern, bool walls, void* buf, const Geom& g, double rho0,     \
                                  const double* f, dim3 grid, dim3 block, hipStream_t st)                           \
    {                                                                                                                \
        BY(precision, [&](auto L) { L.set_pops(pattern, walls, buf, g, rho0, f, grid, block, st); });              \
    }                                                                                                                \
    void launch_get_pops_##SUFFIX(int precision, int pattern, bool walls, const void* buf, const Geom& g,           \
                                  double rho0, double* f, dim3 grid, dim3 block, hipStream_t st)                    \
    {                                                                                                                \
        BY(precision, [&](auto L) { L.get_pops(pattern, walls, buf, g, rho0, f, grid, block, st); });              \
    }                                                                                                                \
    void launch_moments_##SUFFIX(int precision, int pattern, bool walls, const void* buf, const Geom& g,            \
                                 const Phys& ph, double* rho, double* u, double* partials, dim3 grid, dim3 block,   \
                                 hipStream_t st)                                                                     \
    {                                                                                                                \
        BY(precision, [&](auto L) { L.moments(pattern, walls, buf, g, ph, rho, u, partials, grid, block, st); });  \
    }

LBM_DEFINE_LAUNCHERS(q19, by_precision19)

} // namespace lbm
