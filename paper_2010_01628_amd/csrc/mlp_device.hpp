// Learned higher-order relaxation rates: a per-node MLP on BF16 MFMA.
//
// Network (not in the paper; it replaces the fixed rate 1 of the CMs k10..k18
// of Sec. II.B): 11 inputs -> 32 ReLU -> 32 ReLU -> 9 linear outputs z,
// omega_hi = 1 + z; any rate outside (0, 2) sends the node back to the
// paper's rates.  Inputs: rho - 1, (k4 - rho)/rho, k10..k15/rho and
// (k16..k18 - rho/9)/rho, each times a fixed inverse scale.
//
// One wavefront evaluates the network for its 64 nodes (one per lane) on
// 32 x 32 MFMA products.  Inference (the step kernels, mlp_forward_regs)
// keeps the activations in registers and uses the 16-deep
// v_mfma_f32_32x32x16bf16 (its layout is described there); training
// (mlp_forward_wave) moves them through per-wavefront LDS tiles (rows =
// nodes, bf16), which its weight-gradient products need, and uses the 8-deep
// v_mfma_f32_32x32x8bf16_1k, operand layout (lane l, v = 0..3):
//   A[l % 32][4 (l / 32) + v],  B[4 (l / 32) + v][l % 32],
//   D: acc[r] = D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
// (the same D layout for both depths).  Products take BF16 operands and
// accumulate in FP32; biases and the rates are FP32; ReLU is applied to the
// bf16 activations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "d3q19_cm.hpp"

namespace lbm {

constexpr int MLP_NIN = 11, MLP_NH = 32, MLP_NOUT = 9;
constexpr int MLP_NPARAM = MLP_NH * MLP_NIN + MLP_NH + MLP_NH * MLP_NH + MLP_NH + MLP_NOUT * MLP_NH + MLP_NOUT;
// offsets of the flat FP32 parameter vector: W1[32][11] b1[32] W2[32][32] b2[32] W3[9][32] b3[9]
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = 352, MLP_OFF_W2 = 384, MLP_OFF_B2 = 1408, MLP_OFF_W3 = 1440,
              MLP_OFF_B3 = 1728;
static_assert(MLP_OFF_B3 + MLP_NOUT == MLP_NPARAM, "parameter layout");

// Packed network as the kernels read it (built by k_mlp_pack from the FP32
// master parameters).  Matrices are bf16 [row][col], zero padded to 32 x 32
// (W1 to 32 x 16); the transposed copies serve the backward products.
struct alignas(16) MlpPacked {
    // inference part (what the step kernels read)
    uint16_t w1[32 * 16]; // [out][in]
    uint16_t w2[32 * 32]; // [out][in]
    uint16_t w3[32 * 32]; // [out (9 used)][in]
    float b1[32], b2[32], b3[32];
    float inv_scale[16];
    // transposed copies for the backward pass
    uint16_t w2t[32 * 32]; // [in][out]
    uint16_t w3t[32 * 32]; // [in][out (9 used)]
};
constexpr int MLP_INFER_WORDS = (int)(__builtin_offsetof(MlpPacked, w2t) / 4);
static_assert(MLP_INFER_WORDS % 4 == 0 && sizeof(MlpPacked) % 16 == 0, "16-byte network copies");

// Cooperative copy of the first `words` 32-bit words (a multiple of four) of
// the packed network into 16-byte aligned LDS, in two parts so that a kernel
// can issue its own memory reads in between: net_copy_begin issues each
// thread's two 16-byte loads, net_copy_finish writes them, copies what is
// left (work-groups of fewer than words / 8 threads) and waits for the
// work-group.  All threads of the block take part.  The loads and stores
// are unconditional, so that the compiler keeps the loads where they are
// issued: a thread with no chunk of its own copies chunk min(tid, n4 - 1)
// again (the same value to the same place as the thread that owns it).
struct NetCopy {
    uint4 r0, r1;
    int i0, i1;
};
__device__ __attribute__((always_inline)) inline NetCopy net_copy_begin(const MlpPacked* __restrict__ src, int words)
{
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int nthr = blockDim.x * blockDim.y;
    const int n4 = words / 4;
    const uint4* s = reinterpret_cast<const uint4*>(src);
    NetCopy c;
    c.i0 = tid < n4 ? tid : n4 - 1;
    c.i1 = tid + nthr < n4 ? tid + nthr : c.i0;
    c.r0 = s[c.i0];
    c.r1 = s[c.i1];
    return c;
}
__device__ __attribute__((always_inline)) inline void net_copy_finish(const NetCopy& c, const MlpPacked* __restrict__ src,
                                                                      int words, uint32_t* d)
{
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int nthr = blockDim.x * blockDim.y;
    const int n4 = words / 4;
    uint4* d4 = reinterpret_cast<uint4*>(d);
    d4[c.i0] = c.r0;
    d4[c.i1] = c.r1;
    const uint4* s = reinterpret_cast<const uint4*>(src);
    for (int i = tid + 2 * nthr; i < n4; i += nthr) d4[i] = s[i];
    __syncthreads();
}

__device__ inline void load_net(uint32_t* d, const MlpPacked* __restrict__ src, int words)
{
    net_copy_finish(net_copy_begin(src, words), src, words, d);
}

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__host__ __device__ inline uint16_t f32_to_bf16(float f)
{
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t b)
{
    const uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// ReLU of a value that is rounded to bf16 next: max(x, 0).  Rounding keeps
// the sign and zero, so ReLU then round equals round then ReLU.
__device__ inline float relu(float x) { return x > 0.0f ? x : 0.0f; }

// LDS tile of 64 rows (nodes) of bf16; stride 36 keeps 8-byte alignment and
// halves bank conflicts of column-parallel reads.
constexpr int MLP_LDS_STRIDE = 36;
constexpr int MLP_TILE = 64 * MLP_LDS_STRIDE; // uint16 elements per tile

__device__ inline bf16x4_t lds4(const uint16_t* p) { return *reinterpret_cast<const bf16x4_t*>(p); }

__device__ inline int lane_id() { return __lane_id(); }

// Y = X W^T over one 32-row block: X rows [rb*32, rb*32+32) of a tile (K
// columns), W [32][kw] bf16 row-major (rows = outputs).  K multiple of 8.
template <int K>
__device__ inline f32x16_t mfma_xwT(const uint16_t* xtile, int rb, const uint16_t* w, int kw)
{
    const int l = lane_id();
    f32x16_t acc = {0};
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += 8) {
        const bf16x4_t a = lds4(xtile + (rb * 32 + (l & 31)) * MLP_LDS_STRIDE + k0 + 4 * (l >> 5));
        const bf16x4_t b = lds4(w + (l & 31) * kw + k0 + 4 * (l >> 5));
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// Row (node) index within the 64-row tile of accumulator register r.
__device__ inline int acc_row(int rb, int r) { return rb * 32 + 8 * (r >> 2) + 4 * (lane_id() >> 5) + (r & 3); }

// Forward pass for the 64 nodes of this wavefront.  x: this lane's 11 raw
// features.  Tiles: tx (inputs), th1, th2 (hidden activations, kept for the
// backward pass), tz (outputs as floats, 64 x 9).  On return z holds this
// lane's 9 outputs.  Must be called by all 64 lanes.
__device__ inline void mlp_forward_wave(const MlpPacked& W, uint16_t* tx, uint16_t* th1, uint16_t* th2, float* tz,
                                        const float x[MLP_NIN], float z[MLP_NOUT])
{
    const int l = lane_id();
#pragma unroll
    for (int k = 0; k < 16; ++k) tx[l * MLP_LDS_STRIDE + k] = k < MLP_NIN ? f32_to_bf16(x[k] * W.inv_scale[k]) : 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        const f32x16_t acc = mfma_xwT<16>(tx, rb, W.w1, 16);
        const float bias = W.b1[l & 31];
#pragma unroll
        for (int r = 0; r < 16; ++r) th1[acc_row(rb, r) * MLP_LDS_STRIDE + (l & 31)] = f32_to_bf16(relu(acc[r] + bias));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        const f32x16_t acc = mfma_xwT<32>(th1, rb, W.w2, 32);
        const float bias = W.b2[l & 31];
#pragma unroll
        for (int r = 0; r < 16; ++r) th2[acc_row(rb, r) * MLP_LDS_STRIDE + (l & 31)] = f32_to_bf16(relu(acc[r] + bias));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        const f32x16_t acc = mfma_xwT<32>(th2, rb, W.w3, 32);
        if ((l & 31) < MLP_NOUT) {
            const float bias = W.b3[l & 31];
#pragma unroll
            for (int r = 0; r < 16; ++r) tz[acc_row(rb, r) * MLP_NOUT + (l & 31)] = acc[r] + bias;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int j = 0; j < MLP_NOUT; ++j) z[j] = tz[l * MLP_NOUT + j];
}

// ---------------------------------------------------------------------------
// Inference with the activations kept in registers, on the 16-deep product
// v_mfma_f32_32x32x16bf16 (lane l holds eight k of each operand: A[l % 32][k],
// B[k][l % 32] for the k of slots v = 0..7).  Each layer is computed
// transposed, Y^T[out][node] = W[out][k] X^T[k][node], as two 32-node column
// blocks.  The contraction pairs the slots of A and B, so any assignment of
// k to (half-wave, slot) that both operands share is valid; this one takes
// what the previous layer's accumulator already holds, acc[r] =
// Y^T[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]: for k-step m (16 hidden
// units) slots 0..3 are units 16 m + 4 (l / 32) + 0..3 and slots 4..7 units
// 16 m + 8 + 4 (l / 32) + 0..3, i.e. acc[8m .. 8m+7].  Hidden layers chain
// without data movement; the weight operand reads the two matching 8-byte
// runs of the row.  The input layer takes features 8 (l / 32) + v (one
// 16-byte run of the zero-padded W1 row).  Only the input (lane = node,
// features split over the two half-waves) and the output (rates back to the
// node's lane) cross half-waves, by v_permlane32_swap.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Round to nearest even, two floats per conversion instruction.
__device__ inline uint32_t pack2_bf16(float a, float b)
{
    typedef float f32x2_t __attribute__((ext_vector_type(2)));
    typedef __bf16 b16x2_t __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, b16x2_t));
}

// swap: a <- [a.lo | b.lo], b <- [a.hi | b.hi] (half-waves of 32 lanes)
__device__ inline void swap_halves(uint32_t& a, uint32_t& b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}
__device__ inline void swap_halves(float& a, float& b)
{
    uint32_t ua = __builtin_bit_cast(uint32_t, a), ub = __builtin_bit_cast(uint32_t, b);
    swap_halves(ua, ub);
    a = __builtin_bit_cast(float, ua);
    b = __builtin_bit_cast(float, ub);
}

// bias in accumulator layout: acc[4m + v] = b[8m + 4 (l / 32) + v].  b holds
// 32 floats, zero past the layer's rows (the packed layout), 16-byte aligned:
// four unguarded 16-byte loads per lane.
__device__ inline f32x16_t bias_acc(const float* b)
{
    const float4* p = reinterpret_cast<const float4*>(b + 4 * (lane_id() >> 5));
    f32x16_t acc;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const float4 q = p[2 * m];
        acc[4 * m] = q.x;
        acc[4 * m + 1] = q.y;
        acc[4 * m + 2] = q.z;
        acc[4 * m + 3] = q.w;
    }
    return acc;
}

// ReLU of a pair of bf16 values packed in 32 bits: as 16-bit integers a bf16
// pattern is negative exactly when its sign bit is set, so an integer max
// with 0 zeroes the negative values (and -0) and keeps the others
// (one v_pk_max_i16 per two activations).
__device__ inline uint32_t relu_bf16x2(uint32_t p)
{
    typedef short s16x2_t __attribute__((ext_vector_type(2)));
    const s16x2_t v = __builtin_bit_cast(s16x2_t, p);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, (s16x2_t){0, 0}));
}

// bf16 and ReLU of an accumulator: the next layer's two B operands
// (k-step m from acc[8m .. 8m+7])
__device__ inline void act_to_operands(const f32x16_t& acc, bf16x8_t op[2])
{
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        u32x4_t w;
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = relu_bf16x2(pack2_bf16(acc[8 * m + 2 * q], acc[8 * m + 2 * q + 1]));
        op[m] = __builtin_bit_cast(bf16x8_t, w);
    }
}

// weight operand of a hidden layer's k-step m: row l % 32 of the 32 x 32
// matrix, units 16 m + 4 (l / 32) + 0..3 and 16 m + 8 + 4 (l / 32) + 0..3
__device__ inline bf16x8_t w_hidden(const uint16_t* w, int row, int kh, int m)
{
    typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
    const u32x2_t a = *reinterpret_cast<const u32x2_t*>(w + row * 32 + 16 * m + kh);
    const u32x2_t b = *reinterpret_cast<const u32x2_t*>(w + row * 32 + 16 * m + 8 + kh);
    return __builtin_bit_cast(bf16x8_t, (u32x4_t){a[0], a[1], b[0], b[1]});
}

// One 32-node column block through the three layers; o[q] = accumulator
// rows q (q < 5) of the output layer.
__device__ inline void mlp_block_regs(const MlpPacked& W, const bf16x8_t in, float o[5])
{
    const int l = lane_id();
    const int row = l & 31, kh = 4 * (l >> 5);
    f32x16_t acc = bias_acc(W.b1);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
        __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(W.w1 + row * 16 + 2 * kh)), in, acc, 0, 0, 0);
    bf16x8_t h[2];
    act_to_operands(acc, h);
    acc = bias_acc(W.b2);
#pragma unroll
    for (int m = 0; m < 2; ++m) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w_hidden(W.w2, row, kh, m), h[m], acc, 0, 0, 0);
    act_to_operands(acc, h);
    acc = bias_acc(W.b3);
#pragma unroll
    for (int m = 0; m < 2; ++m) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w_hidden(W.w3, row, kh, m), h[m], acc, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 5; ++q) o[q] = acc[q];
}

// Forward pass for the 64 nodes of this wavefront (node = lane), network W in
// global or LDS memory.  x: this lane's 11 raw features; z: its 9 outputs.
// Must be called by all 64 lanes.
__device__ inline void mlp_forward_regs(const MlpPacked& W, const float x[MLP_NIN], float z[MLP_NOUT])
{
    // input operands: features scaled and rounded, lo = features 0..7 and
    // hi = 8..15 of this lane's node; after the swap lo feeds block 0
    // (nodes 0..31: features 0..7 in lanes < 32, 8..15 in lanes >= 32) and
    // hi block 1 (nodes 32..63)
    float xs[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) xs[k] = k < MLP_NIN ? x[k] * W.inv_scale[k] : 0.0f;
    u32x4_t lo, hi;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        lo[q] = pack2_bf16(xs[2 * q], xs[2 * q + 1]);
        hi[q] = pack2_bf16(xs[8 + 2 * q], xs[8 + 2 * q + 1]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t a = lo[q], b = hi[q];
        swap_halves(a, b);
        lo[q] = a;
        hi[q] = b;
    }
    // o_b[q]: output q (lanes < 32) or 4 + q (lanes >= 32) of node 32 b + l % 32;
    // o_b[4]: output 8 (lanes < 32)
    float o0[5], o1[5];
    mlp_block_regs(W, __builtin_bit_cast(bf16x8_t, lo), o0);
    mlp_block_regs(W, __builtin_bit_cast(bf16x8_t, hi), o1);
#pragma unroll
    for (int q = 0; q < 5; ++q) swap_halves(o0[q], o1[q]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        z[q] = o0[q];
        z[4 + q] = o1[q];
    }
    z[8] = o0[4];
}

// rates 1 + z, or the paper's rates (all 1) when any leaves (0, 2); returns
// true on fallback.  As unsigned integers the FP32 patterns of (0, 2) are
// exactly 1 .. 0x3fffffff (+0 is 0, negative values and NaNs have the sign
// bit or lie above 2.0 = 0x40000000), so one unsigned maximum of pattern - 1
// tests all nine rates, NaN included.  The rates are reset only in
// wavefronts that hold a fallen-back node.
__device__ inline bool mlp_rates(const float z[MLP_NOUT], float rates[MLP_NOUT])
{
    uint32_t worst = 0;
#pragma unroll
    for (int j = 0; j < MLP_NOUT; ++j) {
        const float w = 1.0f + z[j];
        rates[j] = w;
        const uint32_t k = __builtin_bit_cast(uint32_t, w) - 1u;
        worst = k > worst ? k : worst;
    }
    const bool bad = worst >= 0x3fffffffu;
    if (__builtin_amdgcn_ballot_w64(bad) != 0)
#pragma unroll
        for (int j = 0; j < MLP_NOUT; ++j) rates[j] = bad ? 1.0f : rates[j];
    return bad;
}

// The step kernels' form of the same test and of the relaxation, on the
// outputs z = omega_hi - 1 themselves: omega = 1 + z lies in (0, 2) exactly
// when |z| < 1, and as unsigned integers the FP32 patterns with the sign bit
// cleared are below 0x3f800000 (1.0) exactly for |z| < 1 (NaNs lie above),
// so one unsigned maximum tests the nine.  A fallen-back node's z are set to
// 0 (rates 1), in wavefronts that hold one.  Returns true on fallback.
__device__ inline bool mlp_fallback(float z[MLP_NOUT])
{
    uint32_t worst = 0;
#pragma unroll
    for (int j = 0; j < MLP_NOUT; ++j) {
        const uint32_t k = __builtin_bit_cast(uint32_t, z[j]) & 0x7fffffffu;
        worst = k > worst ? k : worst;
    }
    const bool bad = worst >= 0x3f800000u;
    if (__builtin_amdgcn_ballot_w64(bad) != 0)
#pragma unroll
        for (int j = 0; j < MLP_NOUT; ++j) z[j] = bad ? 0.0f : z[j];
    return bad;
}

// Post-collision non-equilibrium CMs with the learned higher-order rates
// omega_hi = 1 + z (eq. posColl0, as relax<R, true>): 1 - omega = -z and
// 1 - omega / 2 = (1 - z) / 2 are formed from z directly, without rounding
// 1 + z first.
__device__ inline void relax_learned(const CMState<float>& st, const Rates<float>& rt, const float z[MLP_NOUT],
                                     RawMoments<float>& p)
{
    const float third = 1.0f / 3.0f, cs2 = third;
    const RawMoments<float>& n = st.n;
    const float Fx = st.Fx, Fy = st.Fy, Fz = st.Fz;
    const float w1 = 1.0f - rt.omega;
    const float s5 = w1 * st.k5, s6 = w1 * st.k6;
    const float s4 = (1.0f - rt.omega_bulk) * st.k4;
    const float hx = 0.5f * cs2 * Fx, hy = 0.5f * cs2 * Fy, hz = 0.5f * cs2 * Fz;
    p.m000 = 0.0f;
    p.m100 = 0.5f * Fx;
    p.m010 = 0.5f * Fy;
    p.m001 = 0.5f * Fz;
    p.m110 = w1 * n.m110;
    p.m101 = w1 * n.m101;
    p.m011 = w1 * n.m011;
    p.m210 = (1.0f - z[0]) * hy - z[0] * n.m210;
    p.m120 = (1.0f - z[1]) * hx - z[1] * n.m120;
    p.m201 = (1.0f - z[2]) * hz - z[2] * n.m201;
    p.m102 = (1.0f - z[3]) * hx - z[3] * n.m102;
    p.m021 = (1.0f - z[4]) * hz - z[4] * n.m021;
    p.m012 = (1.0f - z[5]) * hy - z[5] * n.m012;
    p.m220 = -z[6] * n.m220;
    p.m202 = -z[7] * n.m202;
    p.m022 = -z[8] * n.m022;
    p.m200 = third * (s4 + 2.0f * s5 + s6);
    p.m020 = third * (s4 - s5 + s6);
    p.m002 = third * (s4 - s5 - 2.0f * s6);
}

// Weight-gradient product over the 64 nodes of the wavefront:
// G[i][j] += sum_n A[n][i] B[n][j], A and B tiles (rows = nodes), i, j < 32.
// Returns the accumulator (D layout: row i = 8(r/4) + 4(l/32) + r%4, col j = l%32).
__device__ inline f32x16_t mfma_AtB(const uint16_t* ta, const uint16_t* tb)
{
    const int l = lane_id();
    f32x16_t acc = {0};
#pragma unroll
    for (int n0 = 0; n0 < 64; n0 += 8) {
        bf16x4_t a, b;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int n = n0 + 4 * (l >> 5) + v;
            a[v] = (short)ta[n * MLP_LDS_STRIDE + (l & 31)];
            b[v] = (short)tb[n * MLP_LDS_STRIDE + (l & 31)];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

} // namespace lbm
