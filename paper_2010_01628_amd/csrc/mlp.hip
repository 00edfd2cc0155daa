// Learned-rate D3Q19 step, its training kernels, and the D3Q27 -> D3Q19
// projection that produces training data.
#include "dual.hpp"
#include "lattice_kernels.hpp"
#include "mlp_device.hpp"

namespace lbm {

// Raw features of reading L1 from the pre-collision state (the kernels scale
// them by MlpPacked::inv_scale).
template <class R> __device__ inline void mlp_features(const CMState<R>& st, R x[MLP_NIN])
{
    const R ir = R(1) / st.rho;
    const RawMoments<R>& n = st.n;
    x[0] = st.rho - R(1);
    x[1] = st.k4 * ir;
    x[2] = n.m210 * ir;
    x[3] = n.m120 * ir;
    x[4] = n.m201 * ir;
    x[5] = n.m102 * ir;
    x[6] = n.m021 * ir;
    x[7] = n.m012 * ir;
    x[8] = n.m220 * ir;
    x[9] = n.m202 * ir;
    x[10] = n.m022 * ir;
}

// ---------------------------------------------------------------------------
// Step with learned rates (FP32 collision; FP32/FP16/BF16 storage).  Every
// lane of every wavefront takes part in the network (lanes past the lattice
// edge work on a clamped node and store nothing).  The number of nodes that
// fell back is added to fb_partials[block].
// ---------------------------------------------------------------------------
// ROWS (A-B, periodic, work-groups of whole x rows, blockDim.x == nx <= 256):
// the populations that move along x are staged through LDS as in
// k_step_ab_rows (each source row read aligned, once); the network copy's
// barrier serves both.  Same values as the direct reads, bit for bit.
template <class S, Pattern P, bool WALLS, bool NT, bool O32 = false, bool ROWS = false>
__device__ inline void step_mlp_body(const S* src, S* dst, const Geom& g, const Phys& ph,
                                     const MlpPacked* __restrict__ net, uint32_t* __restrict__ fb_partials)
{
    static_assert(!ROWS || (P == AB && !WALLS), "row staging: periodic A-B only");
    // the inference part of the network, once per work-group in LDS: each
    // wavefront reads its MFMA weight operands and bias accumulators from
    // there instead of from memory (~17 KB per wavefront).  Its loads are
    // issued first, the populations' next, so both are in flight together.
    __shared__ __align__(16) uint32_t net_lds[MLP_INFER_WORDS];
    const NetCopy netcopy = net_copy_begin(net, MLP_INFER_WORDS);
    const MlpPacked* snet = reinterpret_cast<const MlpPacked*>(net_lds);
    const int xr = blockIdx.x * blockDim.x + threadIdx.x;
    const int yr = blockIdx.y * blockDim.y + threadIdx.y;
    const bool valid = xr < g.nx && yr < g.ny;
    const int x = xr < g.nx ? xr : g.nx - 1;
    const int y = yr < g.ny ? yr : g.ny - 1;
    const int z = blockIdx.z;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    // the force's loads next, then the populations' (ahead of them for every
    // storage type here: learned FP16 +2-3 %, FP32 within noise)
    const ForceRaw fr = force_load(ph, g, nb(d, 0, 0, 0), y);
    float s[19];
    if constexpr (ROWS) {
        using L = LatD3Q19;
        __shared__ S rows[moving_x_count<L>()][256];
        const int row0 = threadIdx.y * blockDim.x;
        S direct[L::Q];
        {
            int k = 0;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                const S v = ld<S, NT>(pop_at<S, O32, true>(src, g.stride, i, nb(d, 0, -L::cy(i), -L::cz(i))));
                if (L::cx(i) != 0) {
                    rows[k][row0 + x] = v;
                    ++k;
                } else {
                    direct[i] = v;
                }
            }
        }
        net_copy_finish(netcopy, net, MLP_INFER_WORDS, net_lds);
        int k = 0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            if (L::cx(i) != 0) {
                int xs = x - L::cx(i);
                xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
                s[i] = Codec<S>::dec(rows[k][row0 + xs]);
                ++k;
            } else {
                s[i] = Codec<S>::dec(direct[i]);
            }
        }
    } else {
        gather<LatD3Q19, S, P, WALLS, NT, O32>(src, g.stride, d, s);
        net_copy_finish(netcopy, net, MLP_INFER_WORDS, net_lds);
    }
    float Fx, Fy, Fz;
    force_value(ph, fr, Fx, Fy, Fz);
    float xin[MLP_NIN], zout[MLP_NOUT];
    CMState<float> st;
    pre_collide<float, true>(s, (float)ph.rho0, Fx, Fy, Fz, st);
    mlp_features(st, xin);
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    mlp_forward_regs(*snet, xin, zout);
    const bool fb = mlp_fallback(zout);
    const Rates<float> rt = rates_of<float>(ph);
    RawMoments<float> p;
    if (fb && ph.omega_bulk == 1.0)
        relax<float, false>(st, rt, p); // the paper's rates: the plain step's arithmetic, bit for bit
    else
        relax_learned(st, rt, zout, p);
    if constexpr (Codec<S>::increment)
        post_collide_increment(st, p, s);
    else
        post_collide(st, p, s);
    if (valid) scatter<LatD3Q19, S, P, WALLS, NT, O32>(dst, g.stride, d, s);
    // fallback count: one atomic add per wavefront that has fallen-back
    // nodes (none in normal operation), so a wavefront neither waits for the
    // others of its block nor for a read before it retires
    const uint64_t ballot = __ballot(valid && fb);
    if (ballot != 0 && (tid & 63) == 0) {
        const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        atomicAdd(&fb_partials[bid], (uint32_t)__popcll(ballot));
    }
}

// A-B fits four waves per SIMD without spilling (~125 VGPRs, the collision
// state kept live across the network); the AA variants would spill under
// that limit and keep the compiler's choice.
template <class S, bool WALLS, bool NT, bool O32, bool ROWS = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_step_mlp_ab(
    const S* src, S* dst, Geom g, Phys ph, const MlpPacked* __restrict__ net, uint32_t* __restrict__ fb_partials)
{
    step_mlp_body<S, AB, WALLS, NT, O32, ROWS>(src, dst, g, ph, net, fb_partials);
}

template <class S, Pattern P, bool WALLS, bool NT>
__global__ __launch_bounds__(256) void k_step_mlp(const S* src, S* dst, Geom g, Phys ph,
                                                  const MlpPacked* __restrict__ net, uint32_t* __restrict__ fb_partials)
{
    step_mlp_body<S, P, WALLS, NT>(src, dst, g, ph, net, fb_partials);
}

// ---------------------------------------------------------------------------
// Training, reading L5: loss on the 10 raw moments of f(t+1) after one A-B
// step from f(t) (periodic, no force).  post: post-collision buffer written by
// k_step_mlp (A-B).  Writes dL/df_i(y, t+1) to gbuf (SoA floats, stride N) and
// one FP64 loss partial per block; with `accumulate` the gradient is added to
// what gbuf holds (the adjoint carried back from later steps of a rollout).
// ---------------------------------------------------------------------------
// Energy term (rollouts, `energy` != nullptr): the gradient of
// ew ((E - E_t) / E_t)^2, with the kinetic energies E = 1/2 sum |j|^2 / rho of
// the populations and E_t of the target moments (energy[0] = E, energy[1] =
// E_t, from k_train_energy), is added per node: 2 ew (E - E_t) / E_t^2
// (c_i . u - |u|^2 / 2).  The term's value is formed by the host.
__global__ __launch_bounds__(256) void k_train_loss(const float* __restrict__ post, Geom g, float rho0,
                                                    const float* __restrict__ target, const float* __restrict__ inv_sigma,
                                                    float* __restrict__ gbuf, double* __restrict__ loss_partials,
                                                    int accumulate, const double* __restrict__ energy, float ew)
{
    __shared__ double red[4];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double l2 = 0.0;
    if (x < g.nx && y < g.ny) {
        NodeIdx d;
        node_idx(g, x, y, z, d);
        const int n = nb(d, 0, 0, 0);
        float s[19];
        gather<LatD3Q19, float, AB, false>(post, g.stride, d, s);
        // moments of f = w rho0 + s: rest part (1, 0,0,0, 1/3 x3, 0 x3) rho0
        float m[10] = {rho0, 0, 0, 0, rho0 / 3.0f, rho0 / 3.0f, rho0 / 3.0f, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const float cx = LatD3Q19::cx(i), cy = LatD3Q19::cy(i), cz = LatD3Q19::cz(i);
            m[0] += s[i];
            m[1] += cx * s[i];
            m[2] += cy * s[i];
            m[3] += cz * s[i];
            m[4] += cx * cx * s[i];
            m[5] += cy * cy * s[i];
            m[6] += cz * cz * s[i];
            m[7] += cx * cy * s[i];
            m[8] += cx * cz * s[i];
            m[9] += cy * cz * s[i];
        }
        float dm[10];
        const float two_over_n = 2.0f / (float)g.N;
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const float r = (m[k] - target[(int64_t)k * g.N + n]) * inv_sigma[k];
            l2 += (double)r * (double)r;
            dm[k] = two_over_n * r * inv_sigma[k];
        }
        float ce = 0.0f, ux = 0.0f, uy = 0.0f, uz = 0.0f, u2 = 0.0f;
        if (energy) {
            ce = (float)(2.0 * ew * (energy[0] - energy[1]) / (energy[1] * energy[1]));
            const float ir = 1.0f / m[0];
            ux = m[1] * ir;
            uy = m[2] * ir;
            uz = m[3] * ir;
            u2 = 0.5f * (ux * ux + uy * uy + uz * uz);
        }
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const float cx = LatD3Q19::cx(i), cy = LatD3Q19::cy(i), cz = LatD3Q19::cz(i);
            float gi = dm[0] + cx * dm[1] + cy * dm[2] + cz * dm[3] + cx * cx * dm[4] + cy * cy * dm[5] +
                       cz * cz * dm[6] + cx * cy * dm[7] + cx * cz * dm[8] + cy * cz * dm[9];
            if (energy) gi += ce * (cx * ux + cy * uy + cz * uz - u2);
            float* gp = gbuf + (int64_t)i * g.N + n;
            *gp = accumulate ? *gp + gi : gi;
        }
    }
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    double v = l2;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)((blockDim.x * blockDim.y + 63) / 64); ++i) t += red[i];
        loss_partials[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = t / (double)g.N;
    }
}

// Per-block FP64 partial kinetic energies 1/2 |j|^2 / rho of the populations
// pulled from post (no force) and of the target moments (rho, j): out[b] and
// out[nblocks + b].
__global__ __launch_bounds__(256) void k_train_energy(const float* __restrict__ post, Geom g, float rho0,
                                                      const float* __restrict__ target, double* __restrict__ out)
{
    __shared__ double red[2][4];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double e = 0.0, et = 0.0;
    if (x < g.nx && y < g.ny) {
        NodeIdx d;
        node_idx(g, x, y, z, d);
        const int n = nb(d, 0, 0, 0);
        float s[19];
        gather<LatD3Q19, float, AB, false>(post, g.stride, d, s);
        double r = rho0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            r += s[i];
            jx += LatD3Q19::cx(i) * (double)s[i];
            jy += LatD3Q19::cy(i) * (double)s[i];
            jz += LatD3Q19::cz(i) * (double)s[i];
        }
        e = 0.5 * (jx * jx + jy * jy + jz * jz) / r;
        const double rt = target[n], tx = target[(int64_t)g.N + n], ty = target[2 * (int64_t)g.N + n],
                     tz = target[3 * (int64_t)g.N + n];
        et = 0.5 * (tx * tx + ty * ty + tz * tz) / rt;
    }
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        e += __shfl_xor(e, o, 64);
        et += __shfl_xor(et, o, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = e;
        red[1][tid >> 6] = et;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < (int)((blockDim.x * blockDim.y + 63) / 64); ++i) {
            a += red[0][i];
            b += red[1][i];
        }
        const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        const int nb_ = gridDim.x * gridDim.y * gridDim.z;
        out[bid] = a;
        out[nb_ + bid] = b;
    }
}

// Backward pass, one wavefront per block (64 nodes): recompute the forward
// state from f(t), pull dL/df*_i(x) = dL/df_i(x + c_i, t+1), form
// dL/domega_j = kbar_{10+j} (-(k_{10+j} - k_eq) - R_{10+j}/2) with
// kbar = S(+u)^T M^-T gbar, then back-propagate through the network.  Writes
// this wavefront's 1737 gradient entries to grad_partials[wave].
//
// PROP (rollouts): also dL/df_j(x, t), written to gout[j N + x].  It has two
// parts: the collision's own dependence on the populations at fixed rates,
// and the dependence through the rates (features -> network -> rates).  The
// first is the directional derivative of the collision along each of the 19
// unit vectors, by evaluating it on dual numbers, contracted with gbar; the
// second contracts the same directional derivatives of the 11 raw features
// with xbar = dL/dx, which the network's backward pass gives (ReLU masks,
// W1^T, the input scales).  Nodes that fall back use rates 1 that do not
// depend on the state, and take only the first part.
template <bool PROP>
__global__ __launch_bounds__(64) void k_train_backward(const float* __restrict__ state, const float* __restrict__ gbuf,
                                                       Geom g, Phys ph, const MlpPacked* __restrict__ net,
                                                       float* __restrict__ grad_partials, float* __restrict__ gout,
                                                       int accumulate)
{
    const float rho0 = (float)ph.rho0;
    __shared__ MlpPacked snet;
    __shared__ uint16_t tx[MLP_TILE], th1[MLP_TILE], th2[MLP_TILE], tdz[MLP_TILE], tdh[MLP_TILE];
    __shared__ float tz[64 * MLP_NOUT];
    load_net(reinterpret_cast<uint32_t*>(&snet), net, (int)(sizeof(MlpPacked) / 4));
    const int l = threadIdx.x;
    const int xr = blockIdx.x * 64 + l;
    const int yr = blockIdx.y;
    const bool valid = xr < g.nx;
    const int x = valid ? xr : g.nx - 1;
    const int y = yr, z = blockIdx.z;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    float s[19];
    gather<LatD3Q19, float, AB, false>(state, g.stride, d, s);
    CMState<float> st;
    pre_collide<float, true>(s, rho0, 0.0f, 0.0f, 0.0f, st);
    float xin[MLP_NIN], zout[MLP_NOUT], rates[MLP_NOUT];
    mlp_features(st, xin);
    mlp_forward_wave(snet, tx, th1, th2, tz, xin, zout);
    const bool fb = mlp_rates(zout, rates);
    // adjoint of the streaming
    float gbar[19];
#pragma unroll
    for (int i = 0; i < 19; ++i)
        gbar[i] = gbuf[(int64_t)i * g.N + nb(d, LatD3Q19::cx(i), LatD3Q19::cy(i), LatD3Q19::cz(i))];
    RawMoments<float> kb;
    pops_from_raw_T(gbar, kb);
    shift_all_T(kb, st.ux, st.uy, st.uz);
    const RawMoments<float>& n = st.n;
    // no force in training: R = 0 on rows 10..18
    float dz[MLP_NOUT] = {-kb.m210 * n.m210, -kb.m120 * n.m120, -kb.m201 * n.m201, -kb.m102 * n.m102, -kb.m021 * n.m021,
                          -kb.m012 * n.m012, -kb.m220 * n.m220, -kb.m202 * n.m202, -kb.m022 * n.m022};
    const bool active = valid && !fb;
#pragma unroll
    for (int k = 0; k < 32; ++k) tdz[l * MLP_LDS_STRIDE + k] = (k < MLP_NOUT && active) ? f32_to_bf16(dz[k]) : 0;
    __syncthreads();
    float* gp = grad_partials + (int64_t)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)) * MLP_NPARAM;
    // accumulate: add to the partials of earlier steps of a rollout
    auto put = [accumulate](float* q, float v) { *q = accumulate ? *q + v : v; };
    // dW3[o][h] = sum_n dz[n][o] h2[n][h]
    {
        const f32x16_t acc = mfma_AtB(tdz, th2);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int o = 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
            if (o < MLP_NOUT) put(gp + MLP_OFF_W3 + o * 32 + (l & 31), acc[r]);
        }
    }
    // db3, and dh2 = (dz W3) * relu'(h2)
    if (l < MLP_NOUT) {
        float sb = 0.0f;
        for (int q = 0; q < 64; ++q) sb += bf16_to_f32(tdz[q * MLP_LDS_STRIDE + l]);
        put(gp + MLP_OFF_B3 + l, sb);
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        const f32x16_t acc = mfma_xwT<32>(tdz, rb, snet.w3t, 32);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = acc_row(rb, r), h = l & 31;
            const float a2 = bf16_to_f32(th2[row * MLP_LDS_STRIDE + h]);
            tdh[row * MLP_LDS_STRIDE + h] = f32_to_bf16(a2 > 0.0f ? acc[r] : 0.0f);
        }
    }
    __syncthreads();
    // dW2, db2, dh1 = (dh2 W2) * relu'(h1) written over tdz
    {
        const f32x16_t acc = mfma_AtB(tdh, th1);
#pragma unroll
        for (int r = 0; r < 16; ++r) put(gp + MLP_OFF_W2 + (8 * (r >> 2) + 4 * (l >> 5) + (r & 3)) * 32 + (l & 31), acc[r]);
    }
    if (l < 32) {
        float sb = 0.0f;
        for (int q = 0; q < 64; ++q) sb += bf16_to_f32(tdh[q * MLP_LDS_STRIDE + l]);
        put(gp + MLP_OFF_B2 + l, sb);
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        const f32x16_t acc = mfma_xwT<32>(tdh, rb, snet.w2t, 32);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = acc_row(rb, r), h = l & 31;
            const float a1 = bf16_to_f32(th1[row * MLP_LDS_STRIDE + h]);
            tdz[row * MLP_LDS_STRIDE + h] = f32_to_bf16(a1 > 0.0f ? acc[r] : 0.0f);
        }
    }
    __syncthreads();
    // dW1[o][i] = sum_n dh1[n][o] x[n][i], db1
    {
        const f32x16_t acc = mfma_AtB(tdz, tx);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = l & 31;
            if (i < MLP_NIN) put(gp + MLP_OFF_W1 + (8 * (r >> 2) + 4 * (l >> 5) + (r & 3)) * MLP_NIN + i, acc[r]);
        }
    }
    if (l < 32) {
        float sb = 0.0f;
        for (int q = 0; q < 64; ++q) sb += bf16_to_f32(tdz[q * MLP_LDS_STRIDE + l]);
        put(gp + MLP_OFF_B1 + l, sb);
    }
    if constexpr (PROP) {
        // xbar = (W1^T dh1) * inv_scale: dh1 of this lane's node is row l of tdz
        float xbar[MLP_NIN];
#pragma unroll
        for (int i = 0; i < MLP_NIN; ++i) xbar[i] = 0.0f;
        for (int o = 0; o < 32; ++o) {
            const float dh = bf16_to_f32(tdz[l * MLP_LDS_STRIDE + o]);
#pragma unroll
            for (int i = 0; i < MLP_NIN; ++i) xbar[i] += dh * bf16_to_f32(snet.w1[o * 16 + i]);
        }
#pragma unroll
        for (int i = 0; i < MLP_NIN; ++i) xbar[i] *= snet.inv_scale[i];
        Rates<Dual> rt = rates_of<Dual>(ph);
#pragma unroll
        for (int j = 0; j < MLP_NOUT; ++j) rt.omega_hi[j] = Dual(rates[j], 0.0f);
#pragma unroll 1
        for (int j = 0; j < 19; ++j) {
            Dual sd[19];
#pragma unroll
            for (int i = 0; i < 19; ++i) sd[i] = Dual(s[i], i == j ? 1.0f : 0.0f);
            CMState<Dual> sdt;
            pre_collide<Dual, true>(sd, Dual(rho0, 0.0f), Dual(0.0), Dual(0.0), Dual(0.0), sdt);
            Dual xd[MLP_NIN];
            mlp_features(sdt, xd);
            RawMoments<Dual> pd;
            relax<Dual, true>(sdt, rt, pd);
            post_collide_increment(sdt, pd, sd);
            float acc = 0.0f;
#pragma unroll
            for (int i = 0; i < 19; ++i) acc += gbar[i] * sd[i].d;
#pragma unroll
            for (int k = 0; k < MLP_NIN; ++k) acc += xbar[k] * xd[k].d;
            if (valid) gout[(int64_t)j * g.N + nb(d, 0, 0, 0)] = acc;
        }
    }
}

// grad[p] += sum over the per-wavefront partials, in FP64 and a fixed order
// (repeatable bit for bit).  Stage 1: block (x, y) sums slice y of the
// partials for 64 parameters, four lanes per parameter over interleaved
// partials (each wavefront reads 64 consecutive floats per partial), into
// tmp[y][p]; stage 2 adds the slices.
constexpr int MLP_RED_SLICES = 32;
__global__ __launch_bounds__(256) void k_reduce_grad_slices(const float* __restrict__ partials, int nparts,
                                                            double* __restrict__ tmp)
{
    __shared__ double red[4][64];
    const int l = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + l;
    const int chunk = (nparts + MLP_RED_SLICES - 1) / MLP_RED_SLICES;
    const int w0 = blockIdx.y * chunk, w1 = min(nparts, w0 + chunk);
    double s = 0.0;
    if (p < MLP_NPARAM)
        for (int w = w0 + sub; w < w1; w += 4) s += (double)partials[(int64_t)w * MLP_NPARAM + p];
    red[sub][l] = s;
    __syncthreads();
    if (sub == 0 && p < MLP_NPARAM) tmp[(int64_t)blockIdx.y * MLP_NPARAM + p] = (red[0][l] + red[1][l]) + (red[2][l] + red[3][l]);
}
__global__ __launch_bounds__(256) void k_reduce_grad(const double* __restrict__ tmp, double* __restrict__ grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    double s = 0.0;
    for (int y = 0; y < MLP_RED_SLICES; ++y) s += tmp[(int64_t)y * MLP_NPARAM + p];
    grad[p] += s;
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partials, int n, double* __restrict__ out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Adam on the FP32 master parameters (FP64 gradient).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ theta, float* __restrict__ m1, float* __restrict__ m2,
                                              const double* __restrict__ grad, float lr, float b1, float b2, float eps,
                                              float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float gr = (float)grad[p];
    const float a = b1 * m1[p] + (1.0f - b1) * gr;
    const float b = b2 * m2[p] + (1.0f - b2) * gr * gr;
    m1[p] = a;
    m2[p] = b;
    theta[p] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// FP32 master parameters + inverse feature scales -> packed bf16 network.
__global__ __launch_bounds__(256) void k_mlp_pack(const float* __restrict__ theta, const float* __restrict__ inv_scale,
                                                  MlpPacked* __restrict__ out)
{
    const int t = threadIdx.x;
    for (int i = t; i < 32 * 16; i += 256) {
        const int o = i / 16, k = i % 16;
        out->w1[i] = k < MLP_NIN ? f32_to_bf16(theta[MLP_OFF_W1 + o * MLP_NIN + k]) : 0;
    }
    for (int i = t; i < 32 * 32; i += 256) {
        const int o = i / 32, k = i % 32;
        const uint16_t v2 = f32_to_bf16(theta[MLP_OFF_W2 + o * 32 + k]);
        out->w2[i] = v2;
        out->w2t[k * 32 + o] = v2;
        const uint16_t v3 = o < MLP_NOUT ? f32_to_bf16(theta[MLP_OFF_W3 + o * 32 + k]) : 0;
        out->w3[i] = v3;
        out->w3t[k * 32 + o] = v3;
    }
    if (t < 32) {
        out->b1[t] = theta[MLP_OFF_B1 + t];
        out->b2[t] = theta[MLP_OFF_B2 + t];
        out->b3[t] = t < MLP_NOUT ? theta[MLP_OFF_B3 + t] : 0.0f;
    }
    if (t < 16) out->inv_scale[t] = t < MLP_NIN ? inv_scale[t] : 0.0f;
}

// D3Q27 populations (canonical, double) -> D3Q19 populations with the same 19
// raw moments, and the 10 moments (rho, j, Pi) of the D3Q27 state.
__global__ __launch_bounds__(256) void k_project_q27(const double* __restrict__ f27, int64_t N, double* __restrict__ f19,
                                                     float* __restrict__ mom)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    RawMoments<double> m = {};
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const double v = f27[(int64_t)i * N + n];
        const int a = cx27(i), b = cy27(i), c = cz27(i);
        const int a2 = a * a, b2 = b * b, c2 = c * c;
        m.m000 += v;
        m.m100 += a * v;
        m.m010 += b * v;
        m.m001 += c * v;
        m.m200 += a2 * v;
        m.m020 += b2 * v;
        m.m002 += c2 * v;
        m.m110 += a * b * v;
        m.m101 += a * c * v;
        m.m011 += b * c * v;
        m.m210 += a2 * b * v;
        m.m120 += a * b2 * v;
        m.m201 += a2 * c * v;
        m.m102 += a * c2 * v;
        m.m021 += b2 * c * v;
        m.m012 += b * c2 * v;
        m.m220 += a2 * b2 * v;
        m.m202 += a2 * c2 * v;
        m.m022 += b2 * c2 * v;
    }
    if (f19) {
        double s[19];
        pops_from_raw(m, s);
#pragma unroll
        for (int i = 0; i < 19; ++i) f19[(int64_t)i * N + n] = s[i];
    }
    if (mom) {
        const double v[10] = {m.m000, m.m100, m.m010, m.m001, m.m200, m.m020, m.m002, m.m110, m.m101, m.m011};
#pragma unroll
        for (int k = 0; k < 10; ++k) mom[(int64_t)k * N + n] = (float)v[k];
    }
}

// Per-block FP64 sums of squares of the 11 raw network inputs of the current
// state (to fit the input scales); partials[block][11].
template <class S, Pattern P, bool WALLS>
__global__ __launch_bounds__(256) void k_feature_sumsq(const S* __restrict__ buf, Geom g, Phys ph, double* __restrict__ partials)
{
    __shared__ double red[4][MLP_NIN];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double v[MLP_NIN] = {};
    if (x < g.nx && y < g.ny) {
        NodeIdx d;
        node_idx(g, x, y, z, d);
        float s[19];
        gather<LatD3Q19, S, P, WALLS>(buf, g.stride, d, s);
        float Fx, Fy, Fz;
        node_force(ph, g, nb(d, 0, 0, 0), y, Fx, Fy, Fz);
        CMState<float> st;
        pre_collide<float, true>(s, (float)ph.rho0, Fx, Fy, Fz, st);
        float xin[MLP_NIN];
        mlp_features(st, xin);
#pragma unroll
        for (int k = 0; k < MLP_NIN; ++k) v[k] = (double)xin[k] * (double)xin[k];
    }
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
#pragma unroll
    for (int k = 0; k < MLP_NIN; ++k) {
        double a = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        if ((tid & 63) == 0) red[tid >> 6][k] = a;
    }
    __syncthreads();
    if (tid < MLP_NIN) {
        double t = 0.0;
        for (int i = 0; i < (int)((blockDim.x * blockDim.y + 63) / 64); ++i) t += red[i][tid];
        partials[(int64_t)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)) * MLP_NIN + tid] = t;
    }
}

// out[k] = sum over blocks of partials[block][k], k < 11 (FP64, fixed order)
__global__ void k_sum_features(const double* __restrict__ partials, int nblocks, double* __restrict__ out)
{
    const int k = threadIdx.x;
    if (k >= MLP_NIN) return;
    double t = 0.0;
    for (int b = 0; b < nblocks; ++b) t += partials[(int64_t)b * MLP_NIN + k];
    out[k] = t;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_feature_sumsq(int precision, int pattern, bool walls, const void* buf, const Geom& g, const Phys& ph,
                          double* partials, double* out, int nblocks, dim3 grid, dim3 block, hipStream_t st)
{
#define LBM_FEAT(S_)                                                                                              \
    switch (pattern) {                                                                                            \
    case AB:                                                                                                      \
        if (walls) hipLaunchKernelGGL((k_feature_sumsq<S_, AB, true>), grid, block, 0, st, (const S_*)buf, g, ph, partials); \
        else hipLaunchKernelGGL((k_feature_sumsq<S_, AB, false>), grid, block, 0, st, (const S_*)buf, g, ph, partials); \
        break;                                                                                                    \
    case AA_EVEN:                                                                                                 \
        if (walls) hipLaunchKernelGGL((k_feature_sumsq<S_, AA_EVEN, true>), grid, block, 0, st, (const S_*)buf, g, ph, partials); \
        else hipLaunchKernelGGL((k_feature_sumsq<S_, AA_EVEN, false>), grid, block, 0, st, (const S_*)buf, g, ph, partials); \
        break;                                                                                                    \
    default:                                                                                                      \
        if (walls) hipLaunchKernelGGL((k_feature_sumsq<S_, AA_ODD, true>), grid, block, 0, st, (const S_*)buf, g, ph, partials); \
        else hipLaunchKernelGGL((k_feature_sumsq<S_, AA_ODD, false>), grid, block, 0, st, (const S_*)buf, g, ph, partials); \
    }
    switch (precision) {
    case PREC_FP32: LBM_FEAT(float); break;
    case PREC_FP16: LBM_FEAT(_Float16); break;
    default: LBM_FEAT(bf16_t); break;
    }
#undef LBM_FEAT
    hipLaunchKernelGGL(k_sum_features, dim3(1), dim3(64), 0, st, partials, nblocks, out);
}

template <class S>
static void step_mlp_s(int pattern, bool walls, bool nt, const void* src, void* dst, const Geom& g, const Phys& ph,
                       const void* net, uint32_t* fb, dim3 grid, dim3 block, hipStream_t st)
{
    const S* a = (const S*)src;
    S* b = (S*)dst;
    const MlpPacked* w = (const MlpPacked*)net;
    // row staging: a periodic A-B lattice whose work-groups span whole rows,
    // FP32 storage (at 256^3 staged 0.683 -> 0.702 of 8 TB/s; FP16 storage
    // read directly 0.474, staged 0.462)
    const bool rows = sizeof(S) >= 4 && g.row_stage && (int)block.x == g.nx && grid.x == 1 && block.x * block.y <= 256;
#define LBM_MLP_STEP(P, W, NT_)                                                                       \
    do {                                                                                              \
        if constexpr (P == AB && !W && sizeof(S) >= 4) {                                              \
            if (rows && g.off32) hipLaunchKernelGGL((k_step_mlp_ab<S, W, NT_, true, true>), grid, block, 0, st, a, b, g, ph, w, fb); \
            else if (rows) hipLaunchKernelGGL((k_step_mlp_ab<S, W, NT_, false, true>), grid, block, 0, st, a, b, g, ph, w, fb); \
            else if (g.off32) hipLaunchKernelGGL((k_step_mlp_ab<S, W, NT_, true>), grid, block, 0, st, a, b, g, ph, w, fb); \
            else hipLaunchKernelGGL((k_step_mlp_ab<S, W, NT_, false>), grid, block, 0, st, a, b, g, ph, w, fb); \
        }                                                                                             \
        else if constexpr (P == AB) {                                                                 \
            if (g.off32) hipLaunchKernelGGL((k_step_mlp_ab<S, W, NT_, true>), grid, block, 0, st, a, b, g, ph, w, fb); \
            else hipLaunchKernelGGL((k_step_mlp_ab<S, W, NT_, false>), grid, block, 0, st, a, b, g, ph, w, fb); \
        }                                                                                             \
        else hipLaunchKernelGGL((k_step_mlp<S, P, W, NT_>), grid, block, 0, st, a, b, g, ph, w, fb);    \
    } while (0)
#define LBM_MLP_NT(P, W) \
    if (nt) LBM_MLP_STEP(P, W, true); else LBM_MLP_STEP(P, W, false)
#define LBM_MLP_W(P) \
    if (walls) { LBM_MLP_NT(P, true); } else { LBM_MLP_NT(P, false); }
    switch (pattern) {
    case AB: LBM_MLP_W(AB); break;
    case AA_EVEN: LBM_MLP_W(AA_EVEN); break;
    default: LBM_MLP_W(AA_ODD); break;
    }
#undef LBM_MLP_W
#undef LBM_MLP_NT
#undef LBM_MLP_STEP
}

void launch_step_mlp(int precision, int pattern, bool walls, bool nt, const void* src, void* dst, const Geom& g,
                     const Phys& ph, const void* net, uint32_t* fb_partials, dim3 grid, dim3 block, hipStream_t st)
{
    switch (precision) {
    case PREC_FP32: step_mlp_s<float>(pattern, walls, nt, src, dst, g, ph, net, fb_partials, grid, block, st); break;
    case PREC_FP16: step_mlp_s<_Float16>(pattern, walls, nt, src, dst, g, ph, net, fb_partials, grid, block, st); break;
    default: step_mlp_s<bf16_t>(pattern, walls, nt, src, dst, g, ph, net, fb_partials, grid, block, st); break;
    }
}

void launch_train_loss(const float* post, const Geom& g, float rho0, const float* target, const float* inv_sigma,
                       float* gbuf, double* loss_partials, bool accumulate, const double* energy, float ew, dim3 grid,
                       dim3 block, hipStream_t st)
{
    hipLaunchKernelGGL(k_train_loss, grid, block, 0, st, post, g, rho0, target, inv_sigma, gbuf, loss_partials,
                       (int)accumulate, energy, ew);
}

void launch_train_energy(const float* post, const Geom& g, float rho0, const float* target, double* partials,
                         dim3 grid, dim3 block, hipStream_t st)
{
    hipLaunchKernelGGL(k_train_energy, grid, block, 0, st, post, g, rho0, target, partials);
}

void launch_train_backward(const float* state, const float* gbuf, const Geom& g, const Phys& ph, const void* net,
                           float* grad_partials, float* gout, bool accumulate, hipStream_t st)
{
    const dim3 grid((g.nx + 63) / 64, g.ny, g.nz);
    if (gout)
        hipLaunchKernelGGL(k_train_backward<true>, grid, dim3(64), 0, st, state, gbuf, g, ph, (const MlpPacked*)net,
                           grad_partials, gout, (int)accumulate);
    else
        hipLaunchKernelGGL(k_train_backward<false>, grid, dim3(64), 0, st, state, gbuf, g, ph, (const MlpPacked*)net,
                           grad_partials, gout, (int)accumulate);
}

size_t reduce_grad_tmp_bytes() { return sizeof(double) * MLP_RED_SLICES * MLP_NPARAM; }

void launch_reduce_grad(const float* partials, int nparts, double* grad, double* tmp, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_grad_slices, dim3((MLP_NPARAM + 63) / 64, MLP_RED_SLICES), dim3(256), 0, st, partials,
                       nparts, tmp);
    hipLaunchKernelGGL(k_reduce_grad, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, tmp, grad);
}

void launch_sum_partials(const double* partials, int n, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partials, n, out);
}

void launch_adam(float* theta, float* m1, float* m2, const double* grad, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t st)
{
    hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, theta, m1, m2, grad, lr, b1, b2, eps, c1,
                       c2);
}

void launch_mlp_pack(const float* theta, const float* inv_scale, void* packed, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(256), 0, st, theta, inv_scale, (MlpPacked*)packed);
}

void launch_project_q27(const double* f27, int64_t N, double* f19, float* mom, hipStream_t st)
{
    hipLaunchKernelGGL(k_project_q27, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, f27, N, f19, mom);
}

size_t mlp_packed_bytes() { return sizeof(MlpPacked); }

} // namespace lbm
