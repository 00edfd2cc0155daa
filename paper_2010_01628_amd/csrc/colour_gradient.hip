// Colour-gradient two-phase flow on the D3Q19 CM lattice (App. E; the
// Rayleigh-Taylor case of Sec. III).
//
// Red and blue populations f^r, f^b, each in the layout of the plain lattice
// (A-B pull streaming, SoA, padded stride), stored whole (no rest-state
// shift).  One step is two launches over all nodes:
//   k_cg_phi:  phi = (rho_r - rho_b)/(rho_r + rho_b) of the pulled colours;
//   k_cg_step: grad phi from the phi stencil (mirrored at the y walls), both
//              colours pulled, the total collided with the CM scheme of
//              Sec. II.B towards h_eq = f_eq + rho (phi_i(alpha) - w_i) under
//              the gravity force, the perturbation (interfacial tension) added,
//              the result recoloured into red and blue and stored.
// The equilibrium's extra term rho (phi_i - w_i) is isotropic: it moves only
// the raw moments m200 = m020 = m002 (by rho (1 - 3 alpha)/6) and
// m220 = m202 = m022 (by rho (1 - 3 alpha)/18), so the relaxation of the
// paper's scheme is unchanged and only the equilibrium added back differs.
#include "lattice_kernels.hpp"
#include "coupled.hpp"

namespace lbm {

// phi_i(alpha) of App. E by |c_i|^2, and the perturbation weights B_i.
template <class R> __host__ __device__ inline R cg_phi_i(int c2, R alpha)
{
    return c2 == 0 ? alpha : (c2 == 1 ? (R(1) - alpha) * R(1.0 / 12.0) : (R(1) - alpha) * R(1.0 / 24.0));
}
__host__ __device__ constexpr double cg_B(int c2) { return c2 == 0 ? -1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0); }
__host__ __device__ constexpr int c2_19(int i) { return cx19(i) * cx19(i) + cy19(i) * cy19(i) + cz19(i) * cz19(i); }

template <class S, bool WALLS, bool O32>
__global__ __launch_bounds__(256) void k_cg_phi(const S* __restrict__ red, const S* __restrict__ blue,
                                               typename Codec<S>::R* __restrict__ phi, Geom g)
{
    using R = typename Codec<S>::R;
    int x, y, z;
    if (!thread_node(g, x, y, z)) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    R a[19], b[19];
    gather<LatD3Q19, S, AB, WALLS, false, O32>(red, g.stride, d, a);
    gather<LatD3Q19, S, AB, WALLS, false, O32>(blue, g.stride, d, b);
    R rr = R(0), rb = R(0);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        rr += a[i];
        rb += b[i];
    }
    phi[nb(d, 0, 0, 0)] = (rr - rb) / (rr + rb);
}

// phi at x + c (mirrored across a y wall: phi(x', -1) = phi(x', 0)).
template <class R, bool WALLS>
__device__ inline R phi_at(const R* __restrict__ phi, const NodeIdx& d, int cx, int cy, int cz)
{
    return phi[nb(d, cx, beyond<WALLS>(d, cy) ? 0 : cy, cz)];
}

// The paper's collision (rates omega on k5..k9, 1 elsewhere) of the total
// populations s (whole, not shifted) towards h_eq, in place.
template <class R>
__host__ __device__ inline void cg_collide(R s[19], R alpha, R Fx, R Fy, R Fz, R omega, R& rho)
{
    Rates<R> rt;
    rt.omega = omega;
    rt.omega_bulk = R(1);
#pragma unroll
    for (int j = 0; j < 9; ++j) rt.omega_hi[j] = R(1);
    CMState<R> st;
    pre_collide<R, false>(s, R(0), Fx, Fy, Fz, st);
    RawMoments<R> p;
    relax<R, false>(st, rt, p);
    rho = st.rho;
    const R d = st.rho * (R(1) - R(3) * alpha);
    const R a2 = d * R(1.0 / 6.0), a4 = d * R(1.0 / 18.0);
    st.e.m200 += a2;
    st.e.m020 += a2;
    st.e.m002 += a2;
    st.e.m220 += a4;
    st.e.m202 += a4;
    st.e.m022 += a4;
    post_collide(st, p, s);
}

// One node: collision of the total towards h_eq under gravity, perturbation,
// recolouring; a, b hold the pulled red and blue populations on entry and the
// post-collision ones on return.
template <class R>
__host__ __device__ inline void cg_node(R a[19], R b[19], R gx, R gy, R gz, const CgConst& cc)
{
    R s[19];
    R rr = R(0), rb = R(0);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        rr += a[i];
        rb += b[i];
        s[i] = a[i] + b[i];
    }
    const R rho_n = rr + rb;
    const R alpha = (rr * (R)cc.alpha_r + rb * (R)cc.alpha_b) / rho_n;
    const R fr = rho_n - (R)cc.rho_ref;
    R rho;
    cg_collide(s, alpha, fr * (R)cc.g[0], fr * (R)cc.g[1], fr * (R)cc.g[2], (R)cc.omega, rho);
    const R g2 = gx * gx + gy * gy + gz * gz;
    const bool iface = g2 > R(0);
    const R gn = iface ? sqrt(g2) : R(0);
    const R ig2 = iface ? R(1) / g2 : R(0);
    const R ign = iface ? R(1) / gn : R(0);
    const R halfA = R(0.5) * (R)cc.A * gn;
    const R bias0 = (R)cc.beta * rr * rb / rho; // beta rho_r rho_b / rho^2 times the rho of rho phi_i
    const R cr = rr / rho, cb = rb / rho;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        constexpr double rs2 = 0.70710678118654752440; // 1/sqrt(2)
        const R cg = R(cx19(i)) * gx + R(cy19(i)) * gy + R(cz19(i)) * gz;
        const int c2 = c2_19(i);
        const R f = s[i] + halfA * ((R)w19(i) * cg * cg * ig2 - (R)cg_B(c2));
        const R cos_t = c2 == 0 ? R(0) : cg * ign * (c2 == 1 ? R(1) : R(rs2));
        const R bias = bias0 * cos_t * cg_phi_i<R>(c2, alpha);
        a[i] = cr * f + bias;
        b[i] = cb * f - bias;
    }
}

template <class S, bool WALLS, bool NT, bool O32>
__global__ __launch_bounds__(256) void k_cg_step(const S* __restrict__ rsrc, S* __restrict__ rdst,
                                                const S* __restrict__ bsrc, S* __restrict__ bdst,
                                                const typename Codec<S>::R* __restrict__ phi, Geom g, CgConst cc)
{
    using R = typename Codec<S>::R;
    int x, y, z;
    if (!thread_node(g, x, y, z)) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    // grad phi = 3 sum_i w_i c_i phi(x + c_i), opposite pairs as differences
    R gx = R(0), gy = R(0), gz = R(0);
#pragma unroll
    for (int i = 1; i < 10; ++i) {
        const R dp = (R)(3.0 * w19(i)) * (phi_at<R, WALLS>(phi, d, cx19(i), cy19(i), cz19(i)) -
                                          phi_at<R, WALLS>(phi, d, -cx19(i), -cy19(i), -cz19(i)));
        if (cx19(i)) gx += R(cx19(i)) * dp;
        if (cy19(i)) gy += R(cy19(i)) * dp;
        if (cz19(i)) gz += R(cz19(i)) * dp;
    }
    R a[19], b[19];
    gather<LatD3Q19, S, AB, WALLS, NT, O32>(rsrc, g.stride, d, a);
    gather<LatD3Q19, S, AB, WALLS, NT, O32>(bsrc, g.stride, d, b);
    cg_node(a, b, gx, gy, gz, cc);
    scatter<LatD3Q19, S, AB, WALLS, NT, O32>(rdst, g.stride, d, a);
    scatter<LatD3Q19, S, AB, WALLS, NT, O32>(bdst, g.stride, d, b);
}

// f^k = (rho_k / rho) h_eq(rho, u), placed where the first step pulls it.
template <class S, bool WALLS>
__global__ __launch_bounds__(256) void k_cg_init(S* __restrict__ red, S* __restrict__ blue, Geom g, CgConst cc,
                                                const double* __restrict__ rr_in, const double* __restrict__ rb_in,
                                                const double* __restrict__ u)
{
    using R = typename Codec<S>::R;
    int x, y, z;
    if (!thread_node(g, x, y, z)) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    const int n = nb(d, 0, 0, 0);
    const R rr = (R)rr_in[n], rb = (R)rb_in[n], rho = rr + rb;
    const R alpha = (rr * (R)cc.alpha_r + rb * (R)cc.alpha_b) / rho;
    RawMoments<R> e;
    eq_raw_deviation(rho, rho, (R)u[n], (R)u[g.N + n], (R)u[2 * (int64_t)g.N + n], e);
    const R dd = rho * (R(1) - R(3) * alpha);
    const R a2 = dd * R(1.0 / 6.0), a4 = dd * R(1.0 / 18.0);
    e.m200 += a2;
    e.m020 += a2;
    e.m002 += a2;
    e.m220 += a4;
    e.m202 += a4;
    e.m022 += a4;
    R h[19], a[19], b[19];
    pops_from_raw(e, h);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        a[i] = rr / rho * h[i];
        b[i] = rb / rho * h[i];
    }
    place_state<LatD3Q19, S, AB, WALLS>(red, g.stride, d, a);
    place_state<LatD3Q19, S, AB, WALLS>(blue, g.stride, d, b);
}

// rho, force-shifted u, colour densities (outputs may be NULL) and the FP64
// partial sums of the plain lattice's diagnostics.
template <class S, bool WALLS>
__global__ __launch_bounds__(256) void k_cg_fields(const S* __restrict__ red, const S* __restrict__ blue, Geom g,
                                                  CgConst cc, double* __restrict__ rho_out, double* __restrict__ u_out,
                                                  double* __restrict__ rr_out, double* __restrict__ rb_out,
                                                  double* __restrict__ partials)
{
    using R = typename Codec<S>::R;
    int x, y, z;
    double v[NDIAG] = {0, 0, 0, 0, 0, 0, 0, 1e300};
    if (thread_node(g, x, y, z)) {
        NodeIdx d;
        node_idx(g, x, y, z, d);
        const int n = nb(d, 0, 0, 0);
        R a[19], b[19];
        gather<LatD3Q19, S, AB, WALLS>(red, g.stride, d, a);
        gather<LatD3Q19, S, AB, WALLS>(blue, g.stride, d, b);
        double rr = 0.0, rb = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const double si = (double)a[i] + (double)b[i];
            rr += (double)a[i];
            rb += (double)b[i];
            if (cx19(i)) jx += cx19(i) * si;
            if (cy19(i)) jy += cy19(i) * si;
            if (cz19(i)) jz += cz19(i) * si;
        }
        const double rho = rr + rb;
        const double f = rho - cc.rho_ref;
        const double ux = (jx + 0.5 * f * cc.g[0]) / rho;
        const double uy = (jy + 0.5 * f * cc.g[1]) / rho;
        const double uz = (jz + 0.5 * f * cc.g[2]) / rho;
        if (rho_out) rho_out[n] = rho;
        if (rr_out) rr_out[n] = rr;
        if (rb_out) rb_out[n] = rb;
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
static void cg_step_o(bool walls, bool nt, const void* rs, void* rd, const void* bs, void* bd, void* phi, const Geom& g,
                      const CgConst& cc, dim3 grid, dim3 block, hipStream_t st)
{
    using R = typename Codec<S>::R;
    const S *a = (const S*)rs, *b = (const S*)bs;
    S *ad = (S*)rd, *bdd = (S*)bd;
    R* p = (R*)phi;
#define CG_STEP(W, NTV)                                                                                     \
    do {                                                                                                    \
        hipLaunchKernelGGL((k_cg_phi<S, W, O32>), grid, block, 0, st, a, b, p, g);                          \
        hipLaunchKernelGGL((k_cg_step<S, W, NTV, O32>), grid, block, 0, st, a, ad, b, bdd, (const R*)p, g, cc); \
    } while (0)
    if (walls) {
        if (nt) CG_STEP(true, true);
        else CG_STEP(true, false);
    } else {
        if (nt) CG_STEP(false, true);
        else CG_STEP(false, false);
    }
#undef CG_STEP
}

template <class S>
static void cg_step_t(bool walls, bool nt, const void* rs, void* rd, const void* bs, void* bd, void* phi, const Geom& g,
                      const CgConst& cc, dim3 grid, dim3 block, hipStream_t st)
{
    if (g.off32) cg_step_o<S, true>(walls, nt, rs, rd, bs, bd, phi, g, cc, grid, block, st);
    else cg_step_o<S, false>(walls, nt, rs, rd, bs, bd, phi, g, cc, grid, block, st);
}

void launch_cg_step(int precision, bool walls, bool nt, const void* rsrc, void* rdst, const void* bsrc, void* bdst,
                    void* phi, const Geom& g, const CgConst& cc, dim3 grid, dim3 block, hipStream_t st)
{
    if (precision == PREC_FP64) cg_step_t<double>(walls, nt, rsrc, rdst, bsrc, bdst, phi, g, cc, grid, block, st);
    else cg_step_t<float>(walls, nt, rsrc, rdst, bsrc, bdst, phi, g, cc, grid, block, st);
}

void launch_cg_init(int precision, bool walls, void* red, void* blue, const Geom& g, const CgConst& cc,
                    const double* rho_r, const double* rho_b, const double* u, dim3 grid, dim3 block, hipStream_t st)
{
#define CG_INIT(S, W) hipLaunchKernelGGL((k_cg_init<S, W>), grid, block, 0, st, (S*)red, (S*)blue, g, cc, rho_r, rho_b, u)
    if (precision == PREC_FP64) {
        if (walls) CG_INIT(double, true);
        else CG_INIT(double, false);
    } else {
        if (walls) CG_INIT(float, true);
        else CG_INIT(float, false);
    }
#undef CG_INIT
}

void launch_cg_fields(int precision, bool walls, const void* red, const void* blue, const Geom& g, const CgConst& cc,
                      double* rho, double* u, double* rho_r, double* rho_b, double* partials, dim3 grid, dim3 block,
                      hipStream_t st)
{
#define CG_FIELDS(S, W)                                                                                     \
    hipLaunchKernelGGL((k_cg_fields<S, W>), grid, block, 0, st, (const S*)red, (const S*)blue, g, cc, rho, u, \
                       rho_r, rho_b, partials)
    if (precision == PREC_FP64) {
        if (walls) CG_FIELDS(double, true);
        else CG_FIELDS(double, false);
    } else {
        if (walls) CG_FIELDS(float, true);
        else CG_FIELDS(float, false);
    }
#undef CG_FIELDS
}

} // namespace lbm
