// Ensemble of independent periodic cubic boxes of different sizes, advanced
// by one persistent launch per step.
//
// All boxes live in one allocation: box b's populations start at element
// offset off_b and are SoA with its own stride (N_b padded).  The work list is
// every box cut into tiles of 256 consecutive nodes (x fastest); tile t
// belongs to box tile_box[t].  A launch has a fixed number of workgroups that
// walk the tile list with stride gridDim.x, so uneven boxes need no separate
// launches and the whole step is one kernel node in a captured graph.
#include "lattice_kernels.hpp"
#include "mlp_device.hpp"

namespace lbm {

struct BoxDesc {
    int L;          // side
    int N;          // L^3
    int tile0;      // first tile of the box
    int pad_;
    int64_t off;    // element offset of the box's first population array
    int64_t stride; // elements between its population arrays
    double omega;
};

constexpr int ENS_TILE = 256;

__device__ inline void box_node(const BoxDesc& bd, int n, int& x, int& y, int& z)
{
    x = n % bd.L;
    const int r = n / bd.L;
    y = r % bd.L;
    z = r / bd.L;
}

__device__ inline Geom box_geom(const BoxDesc& bd)
{
    Geom g;
    g.nx = g.ny = g.nz = bd.L;
    g.nxy = bd.L * bd.L;
    g.N = bd.N;
    g.stride = bd.stride;
    return g;
}

template <class L, class S, bool O32>
__global__ __launch_bounds__(256) void k_ens_step(const S* __restrict__ src_all, S* __restrict__ dst_all,
                                                  const BoxDesc* __restrict__ boxes, const int* __restrict__ tile_box,
                                                  int ntiles, float rho0)
{
    using R = typename Codec<S>::R;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BoxDesc bd = boxes[tile_box[t]];
        const int n = (t - bd.tile0) * ENS_TILE + threadIdx.x;
        if (n >= bd.N) continue;
        int x, y, z;
        box_node(bd, n, x, y, z);
        const Geom g = box_geom(bd);
        NodeIdx d;
        node_idx(g, x, y, z, d);
        R s[L::Q];
        gather<L, S, AB, false, true, O32>(src_all + bd.off, g.stride, d, s);
        Phys ph{};
        ph.omega = bd.omega;
        ph.omega_bulk = 1.0;
        for (int j = 0; j < 9; ++j) ph.omega_hi[j] = 1.0;
        NodeMacro<R> mac;
        L::template collide<R, false, Codec<S>::increment>(s, (R)rho0, R(0), R(0), R(0), ph, mac);
        scatter<L, S, AB, false, true, O32>(dst_all + bd.off, g.stride, d, s);
    }
}

// Learned rates (D3Q19, FP32 collision): every thread of a block takes part in
// the network each iteration (tiles past a box's end work on a clamped node).
template <class S, bool O32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_ens_step_mlp(const S* __restrict__ src_all, S* __restrict__ dst_all,
                                                      const BoxDesc* __restrict__ boxes, const int* __restrict__ tile_box,
                                                      int ntiles, float rho0, const MlpPacked* __restrict__ net,
                                                      uint32_t* __restrict__ fb_counts)
{
    __shared__ uint32_t wave_fb[4];
    __shared__ __align__(16) uint32_t net_lds[MLP_INFER_WORDS];
    load_net(net_lds, net, MLP_INFER_WORDS);
    const int w = threadIdx.x >> 6;
    uint32_t my_fb = 0;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BoxDesc bd = boxes[tile_box[t]];
        const int nr = (t - bd.tile0) * ENS_TILE + threadIdx.x;
        const bool valid = nr < bd.N;
        const int n = valid ? nr : bd.N - 1;
        int x, y, z;
        box_node(bd, n, x, y, z);
        const Geom g = box_geom(bd);
        NodeIdx d;
        node_idx(g, x, y, z, d);
        float s[19];
        gather<LatD3Q19, S, AB, false, true, O32>(src_all + bd.off, g.stride, d, s);
        float xin[MLP_NIN], zout[MLP_NOUT];
        {
            CMState<float> st0;
            pre_collide<float, true>(s, rho0, 0.0f, 0.0f, 0.0f, st0);
            const float ir = 1.0f / st0.rho;
            xin[0] = st0.rho - 1.0f;
            xin[1] = st0.k4 * ir;
            xin[2] = st0.n.m210 * ir;
            xin[3] = st0.n.m120 * ir;
            xin[4] = st0.n.m201 * ir;
            xin[5] = st0.n.m102 * ir;
            xin[6] = st0.n.m021 * ir;
            xin[7] = st0.n.m012 * ir;
            xin[8] = st0.n.m220 * ir;
            xin[9] = st0.n.m202 * ir;
            xin[10] = st0.n.m022 * ir;
        }
        // the network, staged in LDS once per work-group, is re-read every
        // tile rather than held in registers across the loop (hoisting its
        // loads costs ~70 registers): an offset the compiler cannot see
        // keeps the reads inside the loop, and LDS reads
        int zoff = 0;
        asm volatile("" : "+s"(zoff));
        mlp_forward_regs(*reinterpret_cast<const MlpPacked*>(reinterpret_cast<const char*>(net_lds) + zoff), xin, zout);
        const bool fb = mlp_fallback(zout);
        // recomputed rather than kept live across the network: with the tile
        // loop's own state, keeping it would spill at four waves per SIMD;
        // kept at three waves per SIMD (15 % fewer VALU instructions) the
        // step measured the same
#pragma unroll
        for (int i = 0; i < 19; ++i) asm volatile("" : "+v"(s[i]));
        CMState<float> st;
        pre_collide<float, true>(s, rho0, 0.0f, 0.0f, 0.0f, st);
        Rates<float> rt;
        rt.omega = (float)bd.omega;
        rt.omega_bulk = 1.0f;
        RawMoments<float> p;
        if (fb)
            relax<float, false>(st, rt, p);
        else
            relax_learned(st, rt, zout, p);
        if constexpr (Codec<S>::increment)
            post_collide_increment(st, p, s);
        else
            post_collide(st, p, s);
        if (valid) scatter<LatD3Q19, S, AB, false, true, O32>(dst_all + bd.off, g.stride, d, s);
        my_fb += (valid && fb) ? 1u : 0u;
    }
    // per-block fallback count (no atomics: one slot per block)
    uint32_t c = my_fb;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) wave_fb[w] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) tot += wave_fb[i];
        fb_counts[blockIdx.x] += tot;
    }
}

// Per-tile FP64 kinetic energy 1/2 sum rho |u|^2 (no force) and mass; the
// per-box sums follow in k_ens_box_sums in tile order (deterministic).
template <class L, class S>
__global__ __launch_bounds__(256) void k_ens_tile_energy(const S* __restrict__ buf, const BoxDesc* __restrict__ boxes,
                                                         const int* __restrict__ tile_box, int ntiles, double rho0,
                                                         double* __restrict__ tile_out)
{
    using R = typename Codec<S>::R;
    __shared__ double red[2][4];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BoxDesc bd = boxes[tile_box[t]];
        const int n = (t - bd.tile0) * ENS_TILE + threadIdx.x;
        double ke = 0.0, mass = 0.0;
        if (n < bd.N) {
            int x, y, z;
            box_node(bd, n, x, y, z);
            const Geom g = box_geom(bd);
            NodeIdx d;
            node_idx(g, x, y, z, d);
            R s[L::Q];
            gather<L, S, AB, false>(buf + bd.off, g.stride, d, s);
            double m0 = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                const double si = (double)s[i];
                m0 += si;
                if (L::cx(i)) jx += L::cx(i) * si;
                if (L::cy(i)) jy += L::cy(i) * si;
                if (L::cz(i)) jz += L::cz(i) * si;
            }
            const double rho = rho0 + m0;
            ke = 0.5 * (jx * jx + jy * jy + jz * jz) / rho;
            mass = rho;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            ke += __shfl_xor(ke, o, 64);
            mass += __shfl_xor(mass, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            red[0][threadIdx.x >> 6] = ke;
            red[1][threadIdx.x >> 6] = mass;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, b = 0.0;
            for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) {
                a += red[0][i];
                b += red[1][i];
            }
            tile_out[2 * (int64_t)t] = a;
            tile_out[2 * (int64_t)t + 1] = b;
        }
        __syncthreads();
    }
}

// One work-group per box: each thread sums a fixed strided subset of the
// box's tile partials, then a fixed-order tree in LDS (deterministic).
__global__ __launch_bounds__(256) void k_ens_box_sums(const double* __restrict__ tile_out,
                                                      const BoxDesc* __restrict__ boxes, int nboxes,
                                                      const int* __restrict__ tile_count, double* __restrict__ box_out)
{
    __shared__ double red[2][256];
    const int b = blockIdx.x;
    const BoxDesc bd = boxes[b];
    double ke = 0.0, mass = 0.0;
    for (int t = bd.tile0 + threadIdx.x; t < bd.tile0 + tile_count[b]; t += blockDim.x) {
        ke += tile_out[2 * (int64_t)t];
        mass += tile_out[2 * (int64_t)t + 1];
    }
    red[0][threadIdx.x] = ke;
    red[1][threadIdx.x] = mass;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        box_out[2 * b] = red[0][0];
        box_out[2 * b + 1] = red[1][0];
    }
}

// ---------------------------------------------------------------------------
// lds_pad: dynamic LDS of the plain step's work-groups (a cap on resident
// wavefronts per SIMD, as for the single lattice); the learned step runs at
// four wavefronts per SIMD by its registers and takes none
template <bool O32>
static void ens_step_o(int q, int precision, bool mlp, const void* src, void* dst, const BoxDesc* bd, const int* tile_box,
                       int ntiles, float rho0, const void* net, uint32_t* fb, int grid, int block, unsigned lds_pad,
                       hipStream_t st)
{
    if (mlp) {
        hipLaunchKernelGGL((k_ens_step_mlp<float, O32>), dim3(grid), dim3(block), 0, st, (const float*)src, (float*)dst,
                           bd, tile_box, ntiles, rho0, (const MlpPacked*)net, fb);
        return;
    }
    if (q == 27) {
        if (precision == PREC_FP64)
            hipLaunchKernelGGL((k_ens_step<LatD3Q27, double, O32>), dim3(grid), dim3(block), lds_pad, st, (const double*)src,
                               (double*)dst, bd, tile_box, ntiles, rho0);
        else
            hipLaunchKernelGGL((k_ens_step<LatD3Q27, float, O32>), dim3(grid), dim3(block), lds_pad, st, (const float*)src,
                               (float*)dst, bd, tile_box, ntiles, rho0);
    } else {
        if (precision == PREC_FP64)
            hipLaunchKernelGGL((k_ens_step<LatD3Q19, double, O32>), dim3(grid), dim3(block), lds_pad, st, (const double*)src,
                               (double*)dst, bd, tile_box, ntiles, rho0);
        else
            hipLaunchKernelGGL((k_ens_step<LatD3Q19, float, O32>), dim3(grid), dim3(block), lds_pad, st, (const float*)src,
                               (float*)dst, bd, tile_box, ntiles, rho0);
    }
}

void launch_ens_step(int q, int precision, bool mlp, bool off32, const void* src, void* dst, const void* boxes,
                     const int* tile_box, int ntiles, float rho0, const void* net, uint32_t* fb, int grid, int block,
                     int occ_waves, int lds_per_cu, hipStream_t st)
{
    const BoxDesc* bd = (const BoxDesc*)boxes;
    const unsigned pad = occ_pad(occ_waves, lds_per_cu, 0, dim3(block));
    if (off32)
        ens_step_o<true>(q, precision, mlp, src, dst, bd, tile_box, ntiles, rho0, net, fb, grid, block, pad, st);
    else
        ens_step_o<false>(q, precision, mlp, src, dst, bd, tile_box, ntiles, rho0, net, fb, grid, block, pad, st);
}

void launch_ens_energy(int q, int precision, const void* buf, const void* boxes, const int* tile_box, int ntiles,
                       int nboxes, const int* tile_count, double rho0, double* tile_out, double* box_out, int grid,
                       hipStream_t st)
{
    const BoxDesc* bd = (const BoxDesc*)boxes;
#define LBM_ENS_E(LAT, S_)                                                                                       \
    hipLaunchKernelGGL((k_ens_tile_energy<LAT, S_>), dim3(grid), dim3(ENS_TILE), 0, st, (const S_*)buf, bd, tile_box, \
                       ntiles, rho0, tile_out)
    if (q == 27) {
        if (precision == PREC_FP64) LBM_ENS_E(LatD3Q27, double);
        else LBM_ENS_E(LatD3Q27, float);
    } else {
        if (precision == PREC_FP64) LBM_ENS_E(LatD3Q19, double);
        else LBM_ENS_E(LatD3Q19, float);
    }
#undef LBM_ENS_E
    hipLaunchKernelGGL(k_ens_box_sums, dim3(nboxes), dim3(256), 0, st, tile_out, bd, nboxes, tile_count, box_out);
}

size_t ens_box_desc_bytes() { return sizeof(BoxDesc); }

void ens_fill_box_desc(void* out, int L, int tile0, int64_t off, int64_t stride, double omega)
{
    BoxDesc* b = (BoxDesc*)out;
    b->L = L;
    b->N = L * L * L;
    b->tile0 = tile0;
    b->pad_ = 0;
    b->off = off;
    b->stride = stride;
    b->omega = omega;
}

} // namespace lbm
