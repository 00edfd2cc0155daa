// Shan-Chen pseudo-potential two-phase flow on the D3Q19 CM lattice (static
// bubble case of Sec. III): pseudo-potential psi = 1 - exp(-rho) and the
// interaction force F(x) = -G psi(x) sum_i w_i c_i psi(x + c_i) (X. Shan &
// H. Chen, Phys. Rev. E 47, 1993), handed to the paper's collision as F.
//
// One step is two launches over all nodes (A-B pull streaming, periodic):
//   k_sc_psi:  psi(x) from the density of the populations node x pulls
//              (4 or 8 bytes per node written);
// Both take a 1-D grid over all nodes (Geom::flat) or the 3-D one.
//   k_sc_step: psi at the 19 stencil nodes (cached reads of a small field),
//              the force, then the fused gather-collide-store of the plain
//              lattice.
// The force needs psi of the neighbours at the same time level, so it cannot
// be formed inside the collide launch that produces those densities.
#include "lattice_kernels.hpp"
#include "coupled.hpp"

namespace lbm {

template <class S, bool O32>
__global__ __launch_bounds__(256) void k_sc_psi(const S* __restrict__ src, typename Codec<S>::R* __restrict__ psi, Geom g,
                                               double rho0)
{
    using R = typename Codec<S>::R;
    int x, y, z;
    if (!thread_node(g, x, y, z)) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    R s[19];
    gather<LatD3Q19, S, AB, false, false, O32>(src, g.stride, d, s);
    R m = s[0];
#pragma unroll
    for (int i = 1; i < 19; ++i) m += s[i];
    psi[nb(d, 0, 0, 0)] = R(1) - exp(-((R)rho0 + m));
}

// Interaction force (plus the uniform force) at node d from the psi field.
// Opposite velocities (i, i + 9) are taken as differences
// psi(x + c_i) - psi(x - c_i), so a uniform psi gives exactly zero.
template <class R>
__device__ inline void sc_force(const R* __restrict__ psi, const NodeIdx& d, R G, const Phys& ph, R& Fx, R& Fy, R& Fz)
{
    R sx = R(0), sy = R(0), sz = R(0);
#pragma unroll
    for (int i = 1; i < 10; ++i) {
        const R p = (R)w19(i) * (psi[nb(d, cx19(i), cy19(i), cz19(i))] - psi[nb(d, -cx19(i), -cy19(i), -cz19(i))]);
        if (cx19(i)) sx += R(cx19(i)) * p;
        if (cy19(i)) sy += R(cy19(i)) * p;
        if (cz19(i)) sz += R(cz19(i)) * p;
    }
    const R a = -G * psi[nb(d, 0, 0, 0)];
    const bool uni = ph.force_mode == FORCE_UNIFORM;
    Fx = a * sx + (uni ? (R)ph.force[0] : R(0));
    Fy = a * sy + (uni ? (R)ph.force[1] : R(0));
    Fz = a * sz + (uni ? (R)ph.force[2] : R(0));
}

template <class S, bool GENERAL, bool NT, bool O32>
__global__ __launch_bounds__(256) void k_sc_step(const S* __restrict__ src, S* __restrict__ dst,
                                                const typename Codec<S>::R* __restrict__ psi, Geom g, Phys ph, double G)
{
    using R = typename Codec<S>::R;
    int x, y, z;
    if (!thread_node(g, x, y, z)) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    R Fx, Fy, Fz;
    sc_force(psi, d, (R)G, ph, Fx, Fy, Fz);
    R s[19];
    gather<LatD3Q19, S, AB, false, NT, O32>(src, g.stride, d, s);
    NodeMacro<R> mac;
    collide_cm<R, GENERAL, Codec<S>::increment>(s, (R)ph.rho0, Fx, Fy, Fz, rates_of<R>(ph), mac);
    scatter<LatD3Q19, S, AB, false, NT, O32>(dst, g.stride, d, s);
}

// rho, force-shifted u (any output may be NULL) and FP64 partial sums of the
// diagnostics, in the layout of the plain lattice's moments kernel.
template <class S>
__global__ __launch_bounds__(256) void k_sc_fields(const S* __restrict__ src, const typename Codec<S>::R* __restrict__ psi,
                                                  Geom g, Phys ph, double G, double* __restrict__ rho_out,
                                                  double* __restrict__ u_out, double* __restrict__ partials)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double v[NDIAG] = {0, 0, 0, 0, 0, 0, 0, 1e300};
    if (x < g.nx && y < g.ny) {
        NodeIdx d;
        node_idx(g, x, y, z, d);
        const int n = nb(d, 0, 0, 0);
        R s[19];
        gather<LatD3Q19, S, AB, false>(src, g.stride, d, s);
        double m0 = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const double si = (double)s[i];
            m0 += si;
            if (cx19(i)) jx += cx19(i) * si;
            if (cy19(i)) jy += cy19(i) * si;
            if (cz19(i)) jz += cz19(i) * si;
        }
        R Fx, Fy, Fz;
        sc_force(psi, d, (R)G, ph, Fx, Fy, Fz);
        const double rho = ph.rho0 + m0;
        const double ux = (jx + 0.5 * (double)Fx) / rho;
        const double uy = (jy + 0.5 * (double)Fy) / rho;
        const double uz = (jz + 0.5 * (double)Fz) / rho;
        if (rho_out) rho_out[n] = rho;
        if (u_out) {
            u_out[n] = ux;
            u_out[g.N + n] = uy;
            u_out[2 * (int64_t)g.N + n] = uz;
        }
        const double u2 = ux * ux + uy * uy + uz * uz;
        v[0] = rho;
        v[1] = rho * ux;
        v[2] = rho * uy;
        v[3] = rho * uz;
        v[4] = 0.5 * rho * u2;
        v[5] = sqrt(u2);
        v[6] = (isfinite(rho) && isfinite(u2) && rho > 0.0) ? 0.0 : 1.0;
        v[7] = rho;
    }
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    block_reduce_store(v, partials + (int64_t)bid * NDIAG);
}

template <class S, bool O32>
static void sc_step_o(bool general, bool nt, const void* src, void* dst, void* psi, const Geom& g, const Phys& ph,
                      double G, dim3 grid, dim3 block, hipStream_t st)
{
    using R = typename Codec<S>::R;
    const S* a = (const S*)src;
    S* b = (S*)dst;
    R* p = (R*)psi;
    // the lattice's cap on resident wavefronts per SIMD (by LDS allocation):
    // the 100^3 bubble 0.566 -> 0.577 of 8 TB/s with five; the colour-
    // gradient and magnetic steps measured 1 % slower and neutral with it
    hipLaunchKernelGGL((k_sc_psi<S, O32>), grid, block, occ_pad(g, 0, block), st, a, p, g, ph.rho0);
#define SC_STEP(GEN, NTV) hipLaunchKernelGGL((k_sc_step<S, GEN, NTV, O32>), grid, block, occ_pad(g, 0, block), st, a, b, p, g, ph, G)
    if (general) {
        if (nt) SC_STEP(true, true);
        else SC_STEP(true, false);
    } else {
        if (nt) SC_STEP(false, true);
        else SC_STEP(false, false);
    }
#undef SC_STEP
}

template <class S>
static void sc_step_t(bool general, bool nt, const void* src, void* dst, void* psi, const Geom& g, const Phys& ph,
                      double G, dim3 grid, dim3 block, hipStream_t st)
{
    if (g.off32) sc_step_o<S, true>(general, nt, src, dst, psi, g, ph, G, grid, block, st);
    else sc_step_o<S, false>(general, nt, src, dst, psi, g, ph, G, grid, block, st);
}

void launch_sc_step(int precision, bool general, bool nt, const void* src, void* dst, void* psi, const Geom& g,
                    const Phys& ph, double G, dim3 grid, dim3 block, hipStream_t st)
{
    if (precision == PREC_FP64) sc_step_t<double>(general, nt, src, dst, psi, g, ph, G, grid, block, st);
    else sc_step_t<float>(general, nt, src, dst, psi, g, ph, G, grid, block, st);
}

void launch_sc_fields(int precision, const void* src, void* psi, const Geom& g, const Phys& ph, double G, double* rho,
                      double* u, double* partials, dim3 grid, dim3 block, hipStream_t st)
{
    if (precision == PREC_FP64) {
        hipLaunchKernelGGL((k_sc_psi<double, false>), grid, block, 0, st, (const double*)src, (double*)psi, g, ph.rho0);
        hipLaunchKernelGGL((k_sc_fields<double>), grid, block, 0, st, (const double*)src, (const double*)psi, g, ph, G,
                           rho, u, partials);
    } else {
        hipLaunchKernelGGL((k_sc_psi<float, false>), grid, block, 0, st, (const float*)src, (float*)psi, g, ph.rho0);
        hipLaunchKernelGGL((k_sc_fields<float>), grid, block, 0, st, (const float*)src, (const float*)psi, g, ph, G,
                           rho, u, partials);
    }
}

} // namespace lbm
