// Magnetohydrodynamics: D3Q19 CM flow coupled to a D3Q7 vector magnetic
// lattice (induction equation in the vector-valued BGK form of P. J.
// Dellar, J. Comput. Phys. 179, 2002), one fused launch per step.
//
// Per node: flow populations pulled (halfway bounce-back at y walls),
// rho and the force-free velocity u0; magnetic populations g_{i,a} pulled
// (anti-bounce-back at y walls: g_i(x) = -g*_opp(i)(x) + 2 w_i b_wall, which
// puts b = b_wall on the wall); b = sum_i g_i; current
// j = -(w_m / cs^2) eps Lambda_neq with Lambda_neq = sum_i c_i g_i - (u0 b - b u0);
// Lorentz force j x b added to the external force; the paper's collision
// (Sec. II.B, App. B) with that force; magnetic BGK at rate w_m towards
// g_eq_{i,a} = w_i (b_a + c_i.(u b_a - b u_a) / cs^2) with the force-shifted u.
// D3Q7: cs^2 = 1/4, weights 1/4 (rest), 1/8; order rest, -x, -y, -z, +x, +y, +z.
// Storage: g as is (21 arrays, SoA, the flow lattice's stride), A-B.
#include "coupled.hpp"
#include "lattice_kernels.hpp"

namespace lbm {

__host__ __device__ constexpr int opp7(int i) { return i == 0 ? 0 : (i <= 3 ? i + 3 : i - 3); }

// Pull the 21 magnetic populations of node d: g[a*7 + i].
template <class S, bool WALLS>
__device__ inline void gather_mag(const S* __restrict__ buf, int64_t stride, const NodeIdx& d, const MhdConst& mc,
                                  typename Codec<S>::R g[21])
{
    using R = typename Codec<S>::R;
    const int n = nb(d, 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            if (beyond<WALLS>(d, -cy7(i))) {
                const R v = Codec<S>::dec(buf[(int64_t)(a * 7 + opp7(i)) * stride + n]);
                g[a * 7 + i] = R(2) * R(w7(i)) * (R)mc.b_wall[a] - v;
            } else {
                g[a * 7 + i] = Codec<S>::dec(buf[(int64_t)(a * 7 + i) * stride + nb(d, -cx7(i), -cy7(i), -cz7(i))]);
            }
        }
}

// b and j of one node (u0: velocity before the force).
template <class R>
__host__ __device__ inline void mag_current(const R g[21], R u0x, R u0y, R u0z, R omega_m, R b[3], R j[3])
{
    R lam[3][3]; // lam[c][a] = sum_i c_{i,c} g_{i,a}
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R* ga = g + a * 7;
        b[a] = ((ga[0] + ga[1]) + (ga[2] + ga[3])) + ((ga[4] + ga[5]) + ga[6]);
        lam[0][a] = ga[4] - ga[1];
        lam[1][a] = ga[5] - ga[2];
        lam[2][a] = ga[6] - ga[3];
    }
    const R u0[3] = {u0x, u0y, u0z};
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) lam[c][a] -= u0[c] * b[a] - b[c] * u0[a];
    const R k = -omega_m * R(4); // -(w_m / cs^2), cs^2 = 1/4
    j[0] = k * (lam[1][2] - lam[2][1]);
    j[1] = k * (lam[2][0] - lam[0][2]);
    j[2] = k * (lam[0][1] - lam[1][0]);
}

// BGK of the magnetic populations towards g_eq(b, u), in place.
template <class R> __host__ __device__ inline void mag_collide(R g[21], const R b[3], R ux, R uy, R uz, R omega_m)
{
    const R u[3] = {ux, uy, uz};
    const R keep = R(1) - omega_m;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // E_c = (u_c b_a - b_c u_a) / cs^2 along axis c
        R E[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) E[c] = R(4) * (u[c] * b[a] - b[c] * u[a]);
        R* ga = g + a * 7;
        ga[0] = keep * ga[0] + omega_m * (R(0.25) * b[a]);
        const R wb = R(0.125) * b[a];
        ga[1] = keep * ga[1] + omega_m * (wb - R(0.125) * E[0]);
        ga[4] = keep * ga[4] + omega_m * (wb + R(0.125) * E[0]);
        ga[2] = keep * ga[2] + omega_m * (wb - R(0.125) * E[1]);
        ga[5] = keep * ga[5] + omega_m * (wb + R(0.125) * E[1]);
        ga[3] = keep * ga[3] + omega_m * (wb - R(0.125) * E[2]);
        ga[6] = keep * ga[6] + omega_m * (wb + R(0.125) * E[2]);
    }
}

template <class R> __host__ __device__ inline void mag_eq(const R b[3], R ux, R uy, R uz, R g[21])
{
#pragma unroll
    for (int k = 0; k < 21; ++k) g[k] = R(0);
    mag_collide(g, b, ux, uy, uz, R(1));
}

// rho, u0 (force-free), b, j and the total force of one node from its pulled
// flow deviations s and magnetic populations g.
template <class R>
__device__ inline void mhd_node(const R s[19], const R g[21], const Geom& gm, const Phys& ph, const MhdConst& mc,
                                int n, int y, R& rho, R u0[3], R b[3], R j[3], R F[3])
{
    RawMoments<R> m;
    raw_from_pops(s, m);
    rho = (R)ph.rho0 + m.m000;
    const R ir = R(1) / rho;
    u0[0] = m.m100 * ir;
    u0[1] = m.m010 * ir;
    u0[2] = m.m001 * ir;
    mag_current(g, u0[0], u0[1], u0[2], (R)mc.omega_m, b, j);
    R Fx, Fy, Fz;
    node_force(ph, gm, n, y, Fx, Fy, Fz);
    F[0] = Fx + (j[1] * b[2] - j[2] * b[1]);
    F[1] = Fy + (j[2] * b[0] - j[0] * b[2]);
    F[2] = Fz + (j[0] * b[1] - j[1] * b[0]);
}

template <class S, bool WALLS, bool NT>
__global__ __launch_bounds__(256) void k_mhd_step(const S* __restrict__ fsrc, S* __restrict__ fdst,
                                                 const S* __restrict__ gsrc, S* __restrict__ gdst, Geom gm, Phys ph,
                                                 MhdConst mc)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= gm.nx || y >= gm.ny) return;
    NodeIdx d;
    node_idx(gm, x, y, z, d);
    const int n = nb(d, 0, 0, 0);
    R s[19];
    gather<LatD3Q19, S, AB, WALLS, NT>(fsrc, gm.stride, d, s);
    R g[21];
    gather_mag<S, WALLS>(gsrc, gm.stride, d, mc, g);
    R rho, u0[3], b[3], j[3], F[3];
    mhd_node(s, g, gm, ph, mc, n, y, rho, u0, b, j, F);
    NodeMacro<R> mac;
    collide_cm<R, false, Codec<S>::increment>(s, (R)ph.rho0, F[0], F[1], F[2], rates_of<R>(ph), mac);
    scatter<LatD3Q19, S, AB, WALLS, NT>(fdst, gm.stride, d, s);
    mag_collide(g, b, mac.ux, mac.uy, mac.uz, (R)mc.omega_m);
#pragma unroll
    for (int k = 0; k < 21; ++k) st<S, NT>(gdst + (int64_t)k * gm.stride + n, Codec<S>::enc(g[k]));
}

// Equilibrium start, placed where the first step pulls it (the inverse of
// gather_mag for the magnetic populations).
template <class S, bool WALLS>
__global__ __launch_bounds__(256) void k_mhd_init(S* __restrict__ fbuf, S* __restrict__ gbuf, Geom gm, double rho0,
                                                 MhdConst mc, const double* __restrict__ rho_in,
                                                 const double* __restrict__ u_in, const double* __restrict__ b_in)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= gm.nx || y >= gm.ny) return;
    NodeIdx d;
    node_idx(gm, x, y, z, d);
    const int n = nb(d, 0, 0, 0);
    const R ux = (R)u_in[n], uy = (R)u_in[gm.N + n], uz = (R)u_in[2 * (int64_t)gm.N + n];
    R s[19];
    equilibrium_deviation<R>((R)rho_in[n], (R)rho0, ux, uy, uz, s);
    place_state<LatD3Q19, S, AB, WALLS>(fbuf, gm.stride, d, s);
    const R b[3] = {(R)b_in[n], (R)b_in[gm.N + n], (R)b_in[2 * (int64_t)gm.N + n]};
    R g[21];
    mag_eq(b, ux, uy, uz, g);
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < 7; ++i) {
            const R v = g[a * 7 + i];
            if (beyond<WALLS>(d, -cy7(i)))
                gbuf[(int64_t)(a * 7 + opp7(i)) * gm.stride + n] = Codec<S>::enc(R(2) * R(w7(i)) * (R)mc.b_wall[a] - v);
            else
                gbuf[(int64_t)(a * 7 + i) * gm.stride + nb(d, -cx7(i), -cy7(i), -cz7(i))] = Codec<S>::enc(v);
        }
}

// Fields: rho, force-shifted u (with the Lorentz force), b, j (double, each
// may be NULL) and FP64 partials for the diagnostics.
template <class S, bool WALLS>
__global__ __launch_bounds__(256) void k_mhd_fields(const S* __restrict__ fsrc, const S* __restrict__ gsrc, Geom gm,
                                                   Phys ph, MhdConst mc, double* __restrict__ rho_out,
                                                   double* __restrict__ u_out, double* __restrict__ b_out,
                                                   double* __restrict__ j_out, double* __restrict__ partials)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double v[NDIAG] = {0, 0, 0, 0, 0, 0, 0, 1e300};
    if (x < gm.nx && y < gm.ny) {
        NodeIdx d;
        node_idx(gm, x, y, z, d);
        const int n = nb(d, 0, 0, 0);
        R s[19], g[21];
        gather<LatD3Q19, S, AB, WALLS>(fsrc, gm.stride, d, s);
        gather_mag<S, WALLS>(gsrc, gm.stride, d, mc, g);
        R rho, u0[3], b[3], j[3], F[3];
        mhd_node(s, g, gm, ph, mc, n, y, rho, u0, b, j, F);
        double u[3];
        for (int c = 0; c < 3; ++c) u[c] = (double)u0[c] + 0.5 * (double)F[c] / (double)rho;
        if (rho_out) rho_out[n] = (double)rho;
        for (int c = 0; c < 3; ++c) {
            if (u_out) u_out[(int64_t)c * gm.N + n] = u[c];
            if (b_out) b_out[(int64_t)c * gm.N + n] = (double)b[c];
            if (j_out) j_out[(int64_t)c * gm.N + n] = (double)j[c];
        }
        const double r = (double)rho, u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        v[0] = r;
        v[1] = r * u[0];
        v[2] = r * u[1];
        v[3] = r * u[2];
        v[4] = 0.5 * r * u2;
        v[5] = sqrt(u2);
        v[6] = (isfinite(r) && isfinite(u2) && r > 0.0) ? 0.0 : 1.0;
        v[7] = r;
    }
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    block_reduce_store(v, partials + (int64_t)bid * NDIAG);
}

template <class S, bool WALLS>
__global__ __launch_bounds__(256) void k_mhd_get_g(const S* __restrict__ gbuf, Geom gm, MhdConst mc,
                                                  double* __restrict__ out)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= gm.nx || y >= gm.ny) return;
    NodeIdx d;
    node_idx(gm, x, y, z, d);
    R g[21];
    gather_mag<S, WALLS>(gbuf, gm.stride, d, mc, g);
    const int n = nb(d, 0, 0, 0);
    for (int k = 0; k < 21; ++k) out[(int64_t)k * gm.N + n] = (double)g[k];
}

template <class S, bool WALLS>
__global__ __launch_bounds__(256) void k_mhd_set_g(S* __restrict__ gbuf, Geom gm, MhdConst mc, const double* __restrict__ in)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= gm.nx || y >= gm.ny) return;
    NodeIdx d;
    node_idx(gm, x, y, z, d);
    const int n = nb(d, 0, 0, 0);
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < 7; ++i) {
            const R v = (R)in[(int64_t)(a * 7 + i) * gm.N + n];
            if (beyond<WALLS>(d, -cy7(i)))
                gbuf[(int64_t)(a * 7 + opp7(i)) * gm.stride + n] = Codec<S>::enc(R(2) * R(w7(i)) * (R)mc.b_wall[a] - v);
            else
                gbuf[(int64_t)(a * 7 + i) * gm.stride + nb(d, -cx7(i), -cy7(i), -cz7(i))] = Codec<S>::enc(v);
        }
}

// ---------------------------------------------------------------------------
template <class S>
static void mhd_step_t(bool walls, bool nt, const void* fsrc, void* fdst, const void* gsrc, void* gdst, const Geom& g,
                       const Phys& ph, const MhdConst& mc, dim3 grid, dim3 block, hipStream_t st)
{
    const S* a = (const S*)fsrc;
    S* b = (S*)fdst;
    const S* c = (const S*)gsrc;
    S* e = (S*)gdst;
    if (walls) {
        if (nt) hipLaunchKernelGGL((k_mhd_step<S, true, true>), grid, block, 0, st, a, b, c, e, g, ph, mc);
        else hipLaunchKernelGGL((k_mhd_step<S, true, false>), grid, block, 0, st, a, b, c, e, g, ph, mc);
    } else {
        if (nt) hipLaunchKernelGGL((k_mhd_step<S, false, true>), grid, block, 0, st, a, b, c, e, g, ph, mc);
        else hipLaunchKernelGGL((k_mhd_step<S, false, false>), grid, block, 0, st, a, b, c, e, g, ph, mc);
    }
}

void launch_mhd_step(int precision, bool walls, bool nt, const void* fsrc, void* fdst, const void* gsrc, void* gdst,
                     const Geom& g, const Phys& ph, const MhdConst& mc, dim3 grid, dim3 block, hipStream_t st)
{
    if (precision == PREC_FP64) mhd_step_t<double>(walls, nt, fsrc, fdst, gsrc, gdst, g, ph, mc, grid, block, st);
    else mhd_step_t<float>(walls, nt, fsrc, fdst, gsrc, gdst, g, ph, mc, grid, block, st);
}

void launch_mhd_init(int precision, bool walls, void* fbuf, void* gbuf, const Geom& g, double rho0, const MhdConst& mc,
                     const double* rho, const double* u, const double* b, dim3 grid, dim3 block, hipStream_t st)
{
    if (precision == PREC_FP64) {
        if (walls) hipLaunchKernelGGL((k_mhd_init<double, true>), grid, block, 0, st, (double*)fbuf, (double*)gbuf, g, rho0, mc, rho, u, b);
        else hipLaunchKernelGGL((k_mhd_init<double, false>), grid, block, 0, st, (double*)fbuf, (double*)gbuf, g, rho0, mc, rho, u, b);
    } else {
        if (walls) hipLaunchKernelGGL((k_mhd_init<float, true>), grid, block, 0, st, (float*)fbuf, (float*)gbuf, g, rho0, mc, rho, u, b);
        else hipLaunchKernelGGL((k_mhd_init<float, false>), grid, block, 0, st, (float*)fbuf, (float*)gbuf, g, rho0, mc, rho, u, b);
    }
}

void launch_mhd_fields(int precision, bool walls, const void* fsrc, const void* gsrc, const Geom& g, const Phys& ph,
                       const MhdConst& mc, double* rho, double* u, double* b, double* j, double* partials, dim3 grid,
                       dim3 block, hipStream_t st)
{
    if (precision == PREC_FP64) {
        if (walls) hipLaunchKernelGGL((k_mhd_fields<double, true>), grid, block, 0, st, (const double*)fsrc, (const double*)gsrc, g, ph, mc, rho, u, b, j, partials);
        else hipLaunchKernelGGL((k_mhd_fields<double, false>), grid, block, 0, st, (const double*)fsrc, (const double*)gsrc, g, ph, mc, rho, u, b, j, partials);
    } else {
        if (walls) hipLaunchKernelGGL((k_mhd_fields<float, true>), grid, block, 0, st, (const float*)fsrc, (const float*)gsrc, g, ph, mc, rho, u, b, j, partials);
        else hipLaunchKernelGGL((k_mhd_fields<float, false>), grid, block, 0, st, (const float*)fsrc, (const float*)gsrc, g, ph, mc, rho, u, b, j, partials);
    }
}

void launch_mhd_get_g(int precision, bool walls, const void* gbuf, const Geom& g, const MhdConst& mc, double* out,
                      dim3 grid, dim3 block, hipStream_t st)
{
    if (precision == PREC_FP64) {
        if (walls) hipLaunchKernelGGL((k_mhd_get_g<double, true>), grid, block, 0, st, (const double*)gbuf, g, mc, out);
        else hipLaunchKernelGGL((k_mhd_get_g<double, false>), grid, block, 0, st, (const double*)gbuf, g, mc, out);
    } else {
        if (walls) hipLaunchKernelGGL((k_mhd_get_g<float, true>), grid, block, 0, st, (const float*)gbuf, g, mc, out);
        else hipLaunchKernelGGL((k_mhd_get_g<float, false>), grid, block, 0, st, (const float*)gbuf, g, mc, out);
    }
}

void launch_mhd_set_g(int precision, bool walls, void* gbuf, const Geom& g, const MhdConst& mc, const double* in,
                      dim3 grid, dim3 block, hipStream_t st)
{
    if (precision == PREC_FP64) {
        if (walls) hipLaunchKernelGGL((k_mhd_set_g<double, true>), grid, block, 0, st, (double*)gbuf, g, mc, in);
        else hipLaunchKernelGGL((k_mhd_set_g<double, false>), grid, block, 0, st, (double*)gbuf, g, mc, in);
    } else {
        if (walls) hipLaunchKernelGGL((k_mhd_set_g<float, true>), grid, block, 0, st, (float*)gbuf, g, mc, in);
        else hipLaunchKernelGGL((k_mhd_set_g<float, false>), grid, block, 0, st, (float*)gbuf, g, mc, in);
    }
}

} // namespace lbm
