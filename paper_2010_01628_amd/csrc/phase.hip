// Kernels of the two-phase (conservative phase-field) coupled lattice.
//
// One step is two launches over all nodes (A-B pull streaming on both
// lattices, periodic):
//   k_phase_sum:  phi(x) = sum_i h_i(x) with h_i(x) = h*_i(x - c_i) pulled from
//                 the previous step's post-collision phase populations;
//   k_phase_step: phi at the 19 stencil nodes (gradient, Laplacian, chemical
//                 potential, force), flow populations pulled, collided and
//                 stored, phase populations pulled, collided and stored.
// Flow populations use the D3Q19 layout of the plain lattice (deviations
// g_i - w_i, SoA with padded stride); phase populations are stored as is,
// seven arrays with the same stride.
#include "lattice_kernels.hpp"
#include "phase_cm.hpp"
#include "coupled.hpp"

namespace lbm {

template <class S, bool O32 = false>
__device__ inline void gather7(const S* __restrict__ buf, int64_t stride, const NodeIdx& d, typename Codec<S>::R h[7])
{
#pragma unroll
    for (int i = 0; i < 7; ++i)
        h[i] = Codec<S>::dec(*pop_at<S, O32, true>(buf, stride, i, nb(d, -cx7(i), -cy7(i), -cz7(i))));
}

template <class S, bool NT, bool O32 = false>
__device__ inline void store7(S* __restrict__ buf, int64_t stride, int n, const typename Codec<S>::R h[7])
{
#pragma unroll
    for (int i = 0; i < 7; ++i) st<S, NT>(pop_at<S, O32, true>(buf, stride, i, n), Codec<S>::enc(h[i]));
}

template <class S, bool O32>
__global__ __launch_bounds__(256) void k_phase_sum(const S* __restrict__ hsrc, typename Codec<S>::R* __restrict__ phi,
                                                  Geom g)
{
    using R = typename Codec<S>::R;
    int x, y, z;
    if (!thread_node(g, x, y, z)) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    R h[7];
    gather7<S, O32>(hsrc, g.stride, d, h);
    R s = h[0];
#pragma unroll
    for (int i = 1; i < 7; ++i) s += h[i];
    phi[nb(d, 0, 0, 0)] = s;
}

template <class R> __device__ inline void phi_stencil(const R* __restrict__ phi, const NodeIdx& d, R phin[19])
{
#pragma unroll
    for (int i = 0; i < 19; ++i) phin[i] = phi[nb(d, cx19(i), cy19(i), cz19(i))];
}

template <class S, bool NT, bool O32>
__global__ __launch_bounds__(256) void k_phase_step(const S* __restrict__ gsrc, S* __restrict__ gdst,
                                                   const S* __restrict__ hsrc, S* __restrict__ hdst,
                                                   const typename Codec<S>::R* __restrict__ phi, Geom g, PhaseConst pc)
{
    using R = typename Codec<S>::R;
    int x, y, z;
    if (!thread_node(g, x, y, z)) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    const int n = nb(d, 0, 0, 0);
    R phin[19];
    phi_stencil(phi, d, phin);
    R s[19];
    gather<LatD3Q19, S, AB, false, NT, O32>(gsrc, g.stride, d, s);
    RawMoments<R> m;
    raw_from_pops(s, m);
    PhaseMacro<R> o;
    R gx, gy, gz;
    phase_macro(m, phin, pc, o, gx, gy, gz);
    phase_collide_g(s, m, o, (R)pc.omega);
    scatter<LatD3Q19, S, AB, false, NT, O32>(gdst, g.stride, d, s);
    R h[7];
    gather7<S, O32>(hsrc, g.stride, d, h);
    phase_collide_h(h, phin[0], gx, gy, gz, o.ux, o.uy, o.uz, pc);
    store7<S, NT, O32>(hdst, g.stride, n, h);
}

// k_phase_step with work-groups of whole x rows (blockDim.x == nx <= 256,
// periodic): the x-moving populations of both lattices (10 flow, 2 phase)
// are read as aligned source rows into LDS, each element once, and node x
// takes element x - c_x there, as in the plain staged step.  Same values as
// k_phase_step, bit for bit.
template <class S, bool NT, bool O32>
__global__ __launch_bounds__(256) void k_phase_step_rows(const S* __restrict__ gsrc, S* __restrict__ gdst,
                                                        const S* __restrict__ hsrc, S* __restrict__ hdst,
                                                        const typename Codec<S>::R* __restrict__ phi, Geom g,
                                                        PhaseConst pc)
{
    using R = typename Codec<S>::R;
    constexpr int QX = moving_x_count<LatD3Q19>();
    __shared__ S rows[QX + 2][256];
    const int x = threadIdx.x;
    const int yr = blockIdx.y * blockDim.y + threadIdx.y;
    const bool valid = yr < g.ny;
    const int y = valid ? yr : g.ny - 1;
    const int z = blockIdx.z;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    const int row0 = threadIdx.y * blockDim.x;
    {
        int k = 0;
#pragma unroll
        for (int i = 0; i < 19; ++i)
            if (cx19(i) != 0) {
                rows[k][row0 + x] = ld<S, NT>(pop_at<S, O32, true>(gsrc, g.stride, i, nb(d, 0, -cy19(i), -cz19(i))));
                ++k;
            }
        rows[QX][row0 + x] = *pop_at<S, O32, true>(hsrc, g.stride, 1, nb(d, 0, 0, 0));     // -x population
        rows[QX + 1][row0 + x] = *pop_at<S, O32, true>(hsrc, g.stride, 4, nb(d, 0, 0, 0)); // +x population
    }
    __syncthreads();
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int n = nb(d, 0, 0, 0);
    R phin[19];
    phi_stencil(phi, d, phin);
    R s[19];
    {
        int k = 0;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            if (cx19(i) != 0) {
                s[i] = Codec<S>::dec(rows[k][row0 + (cx19(i) > 0 ? xm : xp)]);
                ++k;
            } else {
                s[i] = Codec<S>::dec(ld<S, NT>(pop_at<S, O32, true>(gsrc, g.stride, i, nb(d, 0, -cy19(i), -cz19(i)))));
            }
        }
    }
    RawMoments<R> m;
    raw_from_pops(s, m);
    PhaseMacro<R> o;
    R gx, gy, gz;
    phase_macro(m, phin, pc, o, gx, gy, gz);
    phase_collide_g(s, m, o, (R)pc.omega);
    if (valid) scatter<LatD3Q19, S, AB, false, NT, O32>(gdst, g.stride, d, s);
    R h[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        if (i == 1) h[i] = Codec<S>::dec(rows[QX][row0 + xp]);          // pulled from x + 1
        else if (i == 4) h[i] = Codec<S>::dec(rows[QX + 1][row0 + xm]); // pulled from x - 1
        else h[i] = Codec<S>::dec(*pop_at<S, O32, true>(hsrc, g.stride, i, nb(d, -cx7(i), -cy7(i), -cz7(i))));
    }
    phase_collide_h(h, phin[0], gx, gy, gz, o.ux, o.uy, o.uz, pc);
    if (valid) store7<S, NT, O32>(hdst, g.stride, n, h);
}

// Equilibrium of the initial fields, written where the first step pulls it:
// flow population i of node x at x - c_i, phase population likewise.
template <class S>
__global__ __launch_bounds__(256) void k_phase_init(S* __restrict__ gbuf, S* __restrict__ hbuf, Geom g, PhaseConst pc,
                                                   const double* __restrict__ phi_in, const double* __restrict__ p_in,
                                                   const double* __restrict__ u_in)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    const int n = nb(d, 0, 0, 0);
    const R phi = (R)phi_in[n];
    const R ux = (R)u_in[n], uy = (R)u_in[g.N + n], uz = (R)u_in[2 * (int64_t)g.N + n];
    const R rho = (R)pc.rho_l + phi * (R)pc.drho;
    const R Pi = (R)(3.0 * p_in[n]);
    RawMoments<R> e;
    eq_raw_deviation(Pi - R(1), rho, ux, uy, uz, e);
    R s[19];
    pops_from_raw(e, s);
    place_state<LatD3Q19, S, AB, false>(gbuf, g.stride, d, s);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const R cu = R(cx7(i)) * ux + R(cy7(i)) * uy + R(cz7(i)) * uz;
        hbuf[(int64_t)i * g.stride + nb(d, -cx7(i), -cy7(i), -cz7(i))] =
            Codec<S>::enc(phi * R(w7(i)) * (R(1) + R(4) * cu));
    }
}

// Macroscopic fields (double outputs, any may be NULL) and FP64 partial sums
// [sum rho, sum rho u (3), 1/2 sum rho |u|^2, max |u|, bad count, min rho].
template <class S>
__global__ __launch_bounds__(256) void k_phase_fields(const S* __restrict__ gsrc,
                                                     const typename Codec<S>::R* __restrict__ phi, Geom g, PhaseConst pc,
                                                     double* __restrict__ phi_out, double* __restrict__ p_out,
                                                     double* __restrict__ rho_out, double* __restrict__ u_out,
                                                     double* __restrict__ partials)
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
        R phin[19];
        phi_stencil(phi, d, phin);
        R s[19];
        gather<LatD3Q19, S, AB, false>(gsrc, g.stride, d, s);
        RawMoments<R> m;
        raw_from_pops(s, m);
        PhaseMacro<R> o;
        R gx, gy, gz;
        phase_macro(m, phin, pc, o, gx, gy, gz);
        const double rho = (double)o.rho, ux = (double)o.ux, uy = (double)o.uy, uz = (double)o.uz;
        if (phi_out) phi_out[n] = (double)phin[0];
        if (p_out) p_out[n] = (1.0 + (double)o.dPi) / 3.0;
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
        v[6] = (isfinite(rho) && isfinite(u2) && isfinite((double)o.dPi)) ? 0.0 : 1.0;
        v[7] = rho;
    }
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    block_reduce_store(v, partials + (int64_t)bid * NDIAG);
}

template <class S>
__global__ __launch_bounds__(256) void k_phase_get_h(const S* __restrict__ hbuf, Geom g, double* __restrict__ out)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    R h[7];
    gather7<S>(hbuf, g.stride, d, h);
    const int n = nb(d, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 7; ++i) out[(int64_t)i * g.N + n] = (double)h[i];
}

template <class S>
__global__ __launch_bounds__(256) void k_phase_set_h(S* __restrict__ hbuf, Geom g, const double* __restrict__ in)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    const int n = nb(d, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 7; ++i)
        hbuf[(int64_t)i * g.stride + nb(d, -cx7(i), -cy7(i), -cz7(i))] = Codec<S>::enc((R)in[(int64_t)i * g.N + n]);
}

// ---------------------------------------------------------------------------
template <class S, bool O32>
static void phase_step_o(bool nt, const void* gsrc, void* gdst, const void* hsrc, void* hdst, void* phi, const Geom& g,
                         const PhaseConst& pc, dim3 grid, dim3 block, const Geom& gr, dim3 rgrid, dim3 rblock,
                         hipStream_t st)
{
    using R = typename Codec<S>::R;
    hipLaunchKernelGGL((k_phase_sum<S, O32>), grid, block, 0, st, (const S*)hsrc, (R*)phi, g);
    const bool rows = rblock.x > 0;
    // the lattice's cap on resident wavefronts per SIMD (by LDS allocation):
    // 192^3 two-phase step 0.711 -> 0.717 of 8 TB/s with five
    const unsigned pad_rows =
        rows ? occ_pad(gr, (unsigned)((moving_x_count<LatD3Q19>() + 2) * 256 * sizeof(S)), rblock) : 0;
    const unsigned pad_flat = occ_pad(g, 0, block);
#define PH_STEP(NTV)                                                                                              \
    do {                                                                                                          \
        if (rows)                                                                                                 \
            hipLaunchKernelGGL((k_phase_step_rows<S, NTV, O32>), rgrid, rblock, pad_rows, st, (const S*)gsrc, (S*)gdst,   \
                               (const S*)hsrc, (S*)hdst, (const R*)phi, gr, pc);                                  \
        else                                                                                                      \
            hipLaunchKernelGGL((k_phase_step<S, NTV, O32>), grid, block, pad_flat, st, (const S*)gsrc, (S*)gdst,          \
                               (const S*)hsrc, (S*)hdst, (const R*)phi, g, pc);                                   \
    } while (0)
    if (nt) PH_STEP(true);
    else PH_STEP(false);
#undef PH_STEP
}

void launch_phase_step(int precision, bool nt, const void* gsrc, void* gdst, const void* hsrc, void* hdst, void* phi,
                       const Geom& g, const PhaseConst& pc, dim3 grid, dim3 block, const Geom& gr, dim3 rgrid,
                       dim3 rblock, hipStream_t st)
{
#define PH_ARGS nt, gsrc, gdst, hsrc, hdst, phi, g, pc, grid, block, gr, rgrid, rblock, st
    if (precision == PREC_FP64) {
        if (g.off32) phase_step_o<double, true>(PH_ARGS);
        else phase_step_o<double, false>(PH_ARGS);
    } else {
        if (g.off32) phase_step_o<float, true>(PH_ARGS);
        else phase_step_o<float, false>(PH_ARGS);
    }
#undef PH_ARGS
}

void launch_phase_init(int precision, void* gbuf, void* hbuf, const Geom& g, const PhaseConst& pc, const double* phi,
                       const double* p, const double* u, dim3 grid, dim3 block, hipStream_t st)
{
    if (precision == PREC_FP64)
        hipLaunchKernelGGL(k_phase_init<double>, grid, block, 0, st, (double*)gbuf, (double*)hbuf, g, pc, phi, p, u);
    else
        hipLaunchKernelGGL(k_phase_init<float>, grid, block, 0, st, (float*)gbuf, (float*)hbuf, g, pc, phi, p, u);
}

void launch_phase_fields(int precision, const void* gsrc, const void* hsrc, void* phi, const Geom& g,
                         const PhaseConst& pc, double* phi_out, double* p_out, double* rho_out, double* u_out,
                         double* partials, dim3 grid, dim3 block, hipStream_t st)
{
    if (precision == PREC_FP64) {
        hipLaunchKernelGGL((k_phase_sum<double, false>), grid, block, 0, st, (const double*)hsrc, (double*)phi, g);
        hipLaunchKernelGGL(k_phase_fields<double>, grid, block, 0, st, (const double*)gsrc, (const double*)phi, g, pc,
                           phi_out, p_out, rho_out, u_out, partials);
    } else {
        hipLaunchKernelGGL((k_phase_sum<float, false>), grid, block, 0, st, (const float*)hsrc, (float*)phi, g);
        hipLaunchKernelGGL(k_phase_fields<float>, grid, block, 0, st, (const float*)gsrc, (const float*)phi, g, pc,
                           phi_out, p_out, rho_out, u_out, partials);
    }
}

void launch_phase_get_h(int precision, const void* hbuf, const Geom& g, double* out, dim3 grid, dim3 block,
                        hipStream_t st)
{
    if (precision == PREC_FP64)
        hipLaunchKernelGGL(k_phase_get_h<double>, grid, block, 0, st, (const double*)hbuf, g, out);
    else
        hipLaunchKernelGGL(k_phase_get_h<float>, grid, block, 0, st, (const float*)hbuf, g, out);
}

void launch_phase_set_h(int precision, void* hbuf, const Geom& g, const double* in, dim3 grid, dim3 block,
                        hipStream_t st)
{
    if (precision == PREC_FP64)
        hipLaunchKernelGGL(k_phase_set_h<double>, grid, block, 0, st, (double*)hbuf, g, in);
    else
        hipLaunchKernelGGL(k_phase_set_h<float>, grid, block, 0, st, (float*)hbuf, g, in);
}

} // namespace lbm
