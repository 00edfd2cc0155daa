// Lattice-generic kernels for gfx950: fused gather + collide + store, init,
// macroscopic moments with FP64 reductions, population import/export.
//
// Data layout in HBM: populations are structure of arrays, one array per
// direction, stored as deviations s_i = f_i - w_i rho0 in the storage type S.
// Element (i, n) sits at buf[i * stride + n], n = x + nx (y + ny z); stride >=
// N is padded so that the streams of a step do not start on the same HBM
// channel.
//
// Streaming patterns (Sec. II.B eq. "streaming_f", f_i(x + c_i, t+1) = f_i*(x, t)):
//   A-B pull:  src holds post-collision values of the previous step at their
//              own nodes.  Node x gathers f_i(x) = src_i(x - c_i) (or, when
//              x - c_i lies beyond a wall, src_opp(i)(x): halfway bounce-back),
//              collides and writes f_i*(x) to dst_i(x): reads shifted, writes
//              aligned and coalesced.
//   AA even:   node x reads slot i at x (= f_i(x)), writes f_i* to slot opp(i)
//              at x.  All accesses local.
//   AA odd:    node x reads slot opp(i) at x - c_i (wall: slot i at x) and
//              writes f_i* to slot i at x + c_i (wall: slot opp(i) at x).  Each
//              node writes exactly the locations it read, so the update is in
//              place and race free.
#pragma once

#include "d3q19_cm.hpp"
#include "d3q27_cm.hpp"
#include "lbm_internal.hpp"

namespace lbm {

enum Pattern { AB = 0, AA_EVEN = 1, AA_ODD = 2 };

template <class R> __device__ inline Rates<R> rates_of(const Phys& ph)
{
    Rates<R> rt;
    rt.omega = (R)ph.omega;
    rt.omega_bulk = (R)ph.omega_bulk;
#pragma unroll
    for (int j = 0; j < 9; ++j) rt.omega_hi[j] = (R)ph.omega_hi[j];
    return rt;
}

// Lattice traits ------------------------------------------------------------
struct LatD3Q19 {
    static constexpr int Q = 19;
    __host__ __device__ static constexpr int cx(int i) { return cx19(i); }
    __host__ __device__ static constexpr int cy(int i) { return cy19(i); }
    __host__ __device__ static constexpr int cz(int i) { return cz19(i); }
    __host__ __device__ static constexpr int opp(int i) { return opp19(i); }
    __host__ __device__ static constexpr double w(int i) { return w19(i); }
    template <class R, bool GENERAL, bool INC = false>
    __device__ static void collide(R* s, R rho0, R Fx, R Fy, R Fz, const Phys& ph, NodeMacro<R>& mac)
    {
        collide_cm<R, GENERAL, INC>(s, rho0, Fx, Fy, Fz, rates_of<R>(ph), mac);
    }
    template <class R> __device__ static void eq(R rho, R rho0, R ux, R uy, R uz, R* s)
    {
        equilibrium_deviation<R>(rho, rho0, ux, uy, uz, s);
    }
};

// Same lattice, raw-moment collision (App. C with N = I).
struct LatD3Q19RM : LatD3Q19 {
    template <class R, bool GENERAL, bool INC = false>
    __device__ static void collide(R* s, R rho0, R Fx, R Fy, R Fz, const Phys& ph, NodeMacro<R>& mac)
    {
        collide_rm<R, GENERAL>(s, rho0, Fx, Fy, Fz, rates_of<R>(ph), mac);
    }
};

struct LatD3Q27 {
    static constexpr int Q = 27;
    __host__ __device__ static constexpr int cx(int i) { return cx27(i); }
    __host__ __device__ static constexpr int cy(int i) { return cy27(i); }
    __host__ __device__ static constexpr int cz(int i) { return cz27(i); }
    __host__ __device__ static constexpr int opp(int i) { return opp27(i); }
    __host__ __device__ static constexpr double w(int i) { return w27(i); }
    template <class R, bool GENERAL, bool INC = false>
    __device__ static void collide(R* s, R rho0, R Fx, R Fy, R Fz, const Phys& ph, NodeMacro<R>& mac)
    {
        collide_cm27<R>(s, rho0, Fx, Fy, Fz, (R)ph.omega, mac);
    }
    template <class R> __device__ static void eq(R rho, R rho0, R ux, R uy, R uz, R* s)
    {
        equilibrium_deviation27<R>(rho, rho0, ux, uy, uz, s);
    }
};

// Same lattice, raw-moment collision (N = I).
struct LatD3Q27RM : LatD3Q27 {
    template <class R, bool GENERAL, bool INC = false>
    __device__ static void collide(R* s, R rho0, R Fx, R Fy, R Fz, const Phys& ph, NodeMacro<R>& mac)
    {
        collide_rm27<R>(s, rho0, Fx, Fy, Fz, (R)ph.omega, mac);
    }
};

// Node indexing -------------------------------------------------------------
struct NodeIdx {
    int x, y, z;
    int ox[3], oy[3], oz[3]; // offsets of x-1,x,x+1 (and y, z rows/planes)
    bool ylo, yhi;           // y-1 / y+1 beyond a wall
};

__device__ inline void node_idx(const Geom& g, int x, int y, int z, NodeIdx& d)
{
    d.x = x;
    d.y = y;
    d.z = z;
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
    d.ox[0] = xm;
    d.ox[1] = x;
    d.ox[2] = xp;
    d.oy[0] = ym * g.nx;
    d.oy[1] = y * g.nx;
    d.oy[2] = yp * g.nx;
    d.oz[0] = zm * g.nxy;
    d.oz[1] = z * g.nxy;
    d.oz[2] = zp * g.nxy;
    d.ylo = y == 0;
    d.yhi = y == g.ny - 1;
}

// Node of this thread: a 3-D grid of (bx, by) work-groups over x rows and z
// planes, or (g.flat) a 1-D grid over all N nodes in index order, which
// leaves no lane idle when nx is not a multiple of the work-group width.
__device__ inline bool thread_node(const Geom& g, int& x, int& y, int& z)
{
    if (g.flat) {
        const int n = blockIdx.x * blockDim.x + threadIdx.x;
        if (n >= g.N) return false;
        const int t = n / g.nx;
        x = n - t * g.nx;
        y = t % g.ny;
        z = t / g.ny;
        return true;
    }
    x = blockIdx.x * blockDim.x + threadIdx.x;
    y = blockIdx.y * blockDim.y + threadIdx.y;
    z = blockIdx.z;
    return x < g.nx && y < g.ny;
}

// index of node x + (dx, dy, dz), dx etc. in {-1, 0, 1}
__device__ inline int nb(const NodeIdx& d, int dx, int dy, int dz) { return d.ox[1 + dx] + d.oy[1 + dy] + d.oz[1 + dz]; }

// Is x + (0, dy, 0) beyond a y wall?
template <bool WALLS> __device__ inline bool beyond(const NodeIdx& d, int dy)
{
    if constexpr (!WALLS) return false;
    return (dy < 0 && d.ylo) || (dy > 0 && d.yhi);
}

// Population loads and stores, with or without the non-temporal (streaming)
// hint.  Each population value is touched once per step, so the hint keeps it
// from displacing reusable lines.
//
// The AA even step with 16-bit storage may read without the hint while its
// stores keep it (Geom::even_cached, set by the host for lattices of up to
// 2^25 nodes).  Measured, FP16 / BF16 AA against the hint on both: +4-7 % at
// 128^3, 256^3 and 512x256x128 (0.72 -> 0.75-0.76 of 8 TB/s), within 1 % at
// 192^3, 256x256x512 and 512x512x128, -3 to -4 % at 256x256x1024 and 512^3.
template <class S, bool NT> __device__ inline S ld(const S* p)
{
    if constexpr (!NT) {
        return *p;
    } else if constexpr (sizeof(S) == 2) {
        const uint16_t v = __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p));
        S out;
        __builtin_memcpy(&out, &v, 2);
        return out;
    } else {
        return __builtin_nontemporal_load(p);
    }
}
template <class S, bool NT> __device__ inline void st(S* p, S v)
{
    if constexpr (!NT) {
        *p = v;
    } else if constexpr (sizeof(S) == 2) {
        uint16_t u;
        __builtin_memcpy(&u, &v, 2);
        __builtin_nontemporal_store(u, reinterpret_cast<uint16_t*>(p));
    } else {
        __builtin_nontemporal_store(v, p);
    }
}

// Element `idx` of population array `slot`.  O32: every population array is
// below 4 GiB, so the element's byte offset is formed in 32 bits and added to
// the array base, which is the same for the whole wavefront when the slot is a
// constant: the access then takes a scalar base and a 32-bit vector offset
// instead of a 64-bit address per lane.  UNIFORM (the slot is the same for
// every lane: a constant of the unrolled loop, not a per-node bounce-back
// choice; buf and stride are kernel arguments): the empty asm pins the base
// in scalar registers.  Without it the compiler hoists the offset that the 19
// stores share into one 64-bit vector pointer and rebuilds every store
// address from it with 64-bit vector multiply-adds.
template <class S, bool O32, bool UNIFORM = false>
__device__ inline const S* pop_at(const S* buf, int64_t stride, int slot, int idx)
{
    const S* base = buf + (int64_t)slot * stride;
    if constexpr (O32) {
        const uint32_t off = (uint32_t)idx * (uint32_t)sizeof(S);
        if constexpr (UNIFORM) {
            // pinned as a global-address-space pointer, so accesses stay
            // global (not flat) instructions
            typedef __attribute__((address_space(1))) const char gchar;
            gchar* gb = (gchar*)base;
            asm("" : "+s"(gb));
            // the offset passes through an asm, so its 64-bit extension is
            // formed beside the access; not volatile, and not tied to the
            // array: accesses with the same offset share one asm (and one
            // register), where one asm per (array, offset) pair cost a register
            // copy per access (~20 VALU instructions per wavefront, 5 % of the
            // 16-bit step's; the 16-bit steps ran 4-6 % faster without them)
            uint32_t o;
            asm("" : "=v"(o) : "0"(off));
            return reinterpret_cast<const S*>((const char*)(gb + o));
        }
        return reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + off);
    } else
        return base + idx;
}
template <class S, bool O32, bool UNIFORM = false> __device__ inline S* pop_at(S* buf, int64_t stride, int slot, int idx)
{
    return const_cast<S*>(pop_at<S, O32, UNIFORM>(static_cast<const S*>(buf), stride, slot, idx));
}

// Where f_i(x, t) lives in the buffer for pattern P (slot, node index).
template <class L, Pattern P, bool WALLS>
__device__ inline void state_loc(const NodeIdx& d, int i, int& slot, int& idx)
{
    const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    if constexpr (P == AA_EVEN) {
        slot = i;
        idx = nb(d, 0, 0, 0);
    } else {
        if (beyond<WALLS>(d, -cy)) {
            // population i arriving from beyond a wall: bounce-back of opp(i)
            slot = (P == AB) ? L::opp(i) : i;
            idx = nb(d, 0, 0, 0);
        } else {
            slot = (P == AB) ? i : L::opp(i);
            idx = nb(d, -cx, -cy, -cz);
        }
    }
}

// Load f_i(x, t) (as deviations) for the current pattern.
template <class L, class S, Pattern P, bool WALLS, bool NT = false, bool O32 = false>
__device__ inline void gather(const S* __restrict__ buf, int64_t stride, const NodeIdx& d, typename Codec<S>::R* s)
{
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int slot, idx;
        state_loc<L, P, WALLS>(d, i, slot, idx);
        // the slot depends on the node only where a wall bounces it back
        constexpr bool U = !WALLS || P == AA_EVEN;
        s[i] = Codec<S>::dec(ld<S, NT>(pop_at<S, O32, U>(buf, stride, slot, idx)));
    }
}

// Store f_i*(x, t) (deviations) for the current pattern.
template <class L, class S, Pattern P, bool WALLS, bool NT, bool O32 = false>
__device__ inline void scatter(S* __restrict__ buf, int64_t stride, const NodeIdx& d, const typename Codec<S>::R* s)
{
    const int n = nb(d, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
        int slot, idx;
        if constexpr (P == AB) {
            slot = i;
            idx = n;
        } else if constexpr (P == AA_EVEN) {
            slot = L::opp(i);
            idx = n;
        } else {
            if (beyond<WALLS>(d, cy)) {
                slot = L::opp(i);
                idx = n;
            } else {
                slot = i;
                idx = nb(d, cx, cy, cz);
            }
        }
        constexpr bool U = !WALLS || P != AA_ODD;
        st<S, NT>(pop_at<S, O32, U>(buf, stride, slot, idx), Codec<S>::enc(s[i]));
    }
}

// Write given deviations s_i(x) where the next step of pattern P reads them as
// f_i(x, t) (the locations of state_loc; a bijection over all (node, i)).
template <class L, class S, Pattern P, bool WALLS>
__device__ inline void place_state(S* __restrict__ buf, int64_t stride, const NodeIdx& d, const typename Codec<S>::R* s)
{
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int slot, idx;
        state_loc<L, P, WALLS>(d, i, slot, idx);
        buf[(int64_t)slot * stride + idx] = Codec<S>::enc(s[i]);
    }
}

// The force at a node in two parts: force_load issues the loads a node's
// force needs (a row table or field entry; issued ahead of the population
// loads), force_value converts where the collision needs it, so that the
// conversion does not make the wavefront wait for the load early (the
// components force_load does not read stay 0 and are not used).
struct ForceRaw {
    double x, y, z;
};
__device__ inline ForceRaw force_load(const Phys& ph, const Geom& g, int n, int y)
{
    ForceRaw f{0.0, 0.0, 0.0};
    if (ph.force_mode == FORCE_FIELD) {
        f.x = ph.force_field[n];
        f.y = ph.force_field[g.N + n];
        f.z = ph.force_field[2 * (int64_t)g.N + n];
    } else if (ph.force_mode == FORCE_ROW_TABLE) {
        f.x = ph.row_table[y];
    }
    return f;
}
template <class R> __device__ inline void force_value(const Phys& ph, const ForceRaw& f, R& Fx, R& Fy, R& Fz)
{
    switch (ph.force_mode) {
    case FORCE_UNIFORM:
        Fx = (R)ph.force[0];
        Fy = (R)ph.force[1];
        Fz = (R)ph.force[2];
        break;
    case FORCE_FIELD:
        Fx = (R)f.x;
        Fy = (R)f.y;
        Fz = (R)f.z;
        break;
    case FORCE_ROW_TABLE:
        Fx = (R)f.x;
        Fy = R(0);
        Fz = R(0);
        break;
    default:
        Fx = Fy = Fz = R(0);
    }
}
// The same in one part, converted where it is read.
template <class R> __device__ inline void node_force(const Phys& ph, const Geom& g, int n, int y, R& Fx, R& Fy, R& Fz)
{
    switch (ph.force_mode) {
    case FORCE_UNIFORM:
        Fx = (R)ph.force[0];
        Fy = (R)ph.force[1];
        Fz = (R)ph.force[2];
        break;
    case FORCE_FIELD:
        Fx = (R)ph.force_field[n];
        Fy = (R)ph.force_field[g.N + n];
        Fz = (R)ph.force_field[2 * (int64_t)g.N + n];
        break;
    case FORCE_ROW_TABLE:
        Fx = (R)ph.row_table[y];
        Fy = R(0);
        Fz = R(0);
        break;
    default:
        Fx = Fy = Fz = R(0);
    }
}

// Whether a step issues the force's load ahead of the population loads
// (force_load / force_value) or reads it after them (node_force).  Ahead
// measured faster for the AA steps with 2- and 8-byte storage (FP16 / BF16
// AA +1.5-2 %, FP64 AA within noise) and slower with 4-byte storage (FP32
// AA -0.5 %); the staged A-B step keeps its load after the barrier for
// every storage type (ahead: FP32 -0.7 %, FP16 / BF16 -1 to -2 %).
template <class S> constexpr bool early_force() { return sizeof(S) != 4; }

// One fused step at one node.  Block (bx, by, 1) covers bx x-values of by
// rows; blockIdx.z is the z plane.
// Block coordinates of this work-group.  A 3-D grid (ceil(nx/bx), ceil(ny/by),
// nz) maps directly.  A 1-D grid of all those blocks (T of them, a multiple of
// 8 * chunk) is read in the same x-then-y-then-z order after an XCD-aware
// permutation: work-groups go to the eight XCDs round-robin by launch index
// L, so XCD L % 8 takes its k-th block (k = L / 8) from block
// (k / chunk) * 8 chunk + (L % 8) chunk + k % chunk, i.e. each XCD sweeps runs
// of `chunk` consecutive blocks (rows), interleaved with the other XCDs'.
__device__ inline void block_coords(const Geom& g, int chunk, int& bxi, int& byi, int& bz)
{
    if (gridDim.y == 1 && gridDim.z == 1) {
        int L = blockIdx.x;
        if (chunk > 1) {
            const int k = L >> 3;
            L = (k / chunk) * (8 * chunk) + (L & 7) * chunk + k % chunk;
        }
        const int gx = (g.nx + blockDim.x - 1) / blockDim.x;
        const int gy = (g.ny + blockDim.y - 1) / blockDim.y;
        bxi = L % gx;
        const int t = L / gx;
        byi = t % gy;
        bz = t / gy;
    } else {
        bxi = blockIdx.x;
        byi = blockIdx.y;
        bz = blockIdx.z;
    }
}

// NTL: the streaming hint on the loads (NT: on the stores)
template <class L, class S, Pattern P, bool WALLS, bool GENERAL, bool NT, bool O32, bool NTL = NT>
__device__ inline void step_node(const S* src, S* dst, const Geom& g, const Phys& ph)
{
    using R = typename Codec<S>::R;
    int bxi, byi, z;
    block_coords(g, g.xcd_chunk, bxi, byi, z);
    const int x = bxi * blockDim.x + threadIdx.x;
    const int y = byi * blockDim.y + threadIdx.y;
    if (x >= g.nx || y >= g.ny) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    ForceRaw fr{0.0, 0.0, 0.0};
    if constexpr (early_force<S>()) fr = force_load(ph, g, nb(d, 0, 0, 0), y);
    R s[L::Q];
    gather<L, S, P, WALLS, NTL, O32>(src, g.stride, d, s);
    R Fx, Fy, Fz;
    if constexpr (early_force<S>())
        force_value(ph, fr, Fx, Fy, Fz);
    else
        node_force(ph, g, nb(d, 0, 0, 0), y, Fx, Fy, Fz);
    NodeMacro<R> mac;
    L::template collide<R, GENERAL, Codec<S>::increment>(s, (R)ph.rho0, Fx, Fy, Fz, ph, mac);
    if constexpr (Codec<S>::stochastic) dither_bf16(s, ph.sr_key, (uint32_t)nb(d, 0, 0, 0));
    scatter<L, S, P, WALLS, NT, O32>(dst, g.stride, d, s);
}

// A-B: two distinct buffers.
template <class L, class S, bool WALLS, bool GENERAL, bool NT, bool O32>
__global__ __launch_bounds__(256) void k_step_ab(const S* __restrict__ src, S* __restrict__ dst, Geom g, Phys ph)
{
    step_node<L, S, AB, WALLS, GENERAL, NT, O32>(src, dst, g, ph);
}

// Dynamic LDS for a step launch that caps the resident wavefronts per SIMD at
// g.occ_waves (0: no cap): a work-group of T threads places ceil(T / 64)
// wavefronts spread over the compute unit's four SIMDs, so at most
// 4 occ_waves / ceil(T / 64) work-groups may share the unit's LDS; each one
// is given that share (at most 64 KB) less the static LDS it already uses.
inline unsigned occ_pad(int occ_waves, int lds_per_cu, unsigned static_lds, dim3 b)
{
    const unsigned waves = (b.x * b.y * b.z + 63) / 64;
    if (occ_waves <= 0 || waves == 0) return 0; // no cap, or no launch (an empty block shape)
    unsigned wgs = 4u * (unsigned)occ_waves / waves;
    if (wgs < 1) wgs = 1;
    unsigned total = (unsigned)lds_per_cu / wgs;
    if (total > 65536u) total = 65536u;
    return total > static_lds ? total - static_lds : 0;
}
inline unsigned occ_pad(const Geom& g, unsigned static_lds, dim3 b)
{
    return occ_pad(g.occ_waves, g.lds_per_cu, static_lds, b);
}

// A-B, periodic, with work-groups of whole x rows (blockDim.x == nx): the
// populations that move along x are staged through LDS.  Each such
// population's source row (y - c_y, z - c_z) is read aligned, each element
// once, into LDS, and node x takes element x - c_x (wrapped) from there;
// reading it straight from memory would start each wavefront's load four
// bytes off a line boundary.  Same values as k_step_ab, bit for bit.
template <class L> __host__ __device__ constexpr int moving_x_count()
{
    int k = 0;
    for (int i = 0; i < L::Q; ++i) k += L::cx(i) != 0;
    return k;
}

// W: the widest row a work-group may span (256; 512 or 1024 for rows of
// 257..512 or 513..1024 nodes with one work-group of nx threads per row).
template <class L, class S, bool GENERAL, bool NT, bool O32, int W = 256>
__global__ __launch_bounds__(W) void k_step_ab_rows(const S* __restrict__ src, S* __restrict__ dst, Geom g, Phys ph)
{
    using R = typename Codec<S>::R;
    constexpr int QX = moving_x_count<L>();
    __shared__ S rows[QX][W];
    int bxi, byi, z;
    block_coords(g, g.xcd_chunk, bxi, byi, z);
    const int x = threadIdx.x; // bxi == 0: one work-group spans the row
    const int yr = byi * blockDim.y + threadIdx.y;
    const bool valid = yr < g.ny;
    const int y = valid ? yr : g.ny - 1;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    const int row0 = threadIdx.y * blockDim.x;
    // every population load is issued before the barrier: the populations
    // that stay in x go straight to registers, the others to LDS (the
    // force's load follows the barrier; see early_force)
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
    __syncthreads();
    R s[L::Q];
    {
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
    }
    R Fx, Fy, Fz;
    node_force(ph, g, nb(d, 0, 0, 0), y, Fx, Fy, Fz);
    NodeMacro<R> mac;
    L::template collide<R, GENERAL, Codec<S>::increment>(s, (R)ph.rho0, Fx, Fy, Fz, ph, mac);
    if constexpr (Codec<S>::stochastic) dither_bf16(s, ph.sr_key, (uint32_t)nb(d, 0, 0, 0));
    if (valid) scatter<L, S, AB, false, NT, O32>(dst, g.stride, d, s);
}

// AA: one buffer, each node rewrites exactly the locations it read.
template <class L, class S, Pattern P, bool WALLS, bool GENERAL, bool NT, bool O32, bool NTL = NT>
__global__ __launch_bounds__(256) void k_step_aa(S* buf, Geom g, Phys ph)
{
    step_node<L, S, P, WALLS, GENERAL, NT, O32, NTL>(buf, buf, g, ph);
}

// AA odd step, periodic, with work-groups of whole x rows (blockDim.x == nx).
// Node x reads slot opp(i) at x - c_i and writes slot i at x + c_i; for the
// populations that move along x both accesses are staged through LDS so that
// every global access is aligned: thread x reads element x of the source row
// (y - c_y, z - c_z) of array opp(i) into LDS and takes element x - c_x;
// after the collision it puts its value at x + c_x of an LDS row, and thread
// x stores element x of the destination row (y + c_y, z + c_z) of array i.
// In place and race free as the plain kernel: location (i, m) is read only
// by node m - c_i, which lies in the same x row, and a thread stores only
// elements it loaded itself earlier.  Same values as k_step_aa, bit for bit.
template <class L, class S, bool GENERAL, bool NT, bool O32, int W = 256>
__global__ __launch_bounds__(W) void k_step_aa_odd_rows(S* __restrict__ buf, Geom g, Phys ph)
{
    using R = typename Codec<S>::R;
    constexpr int QX = moving_x_count<L>();
    __shared__ S rows[QX][W];
    int bxi, byi, z;
    block_coords(g, g.xcd_chunk, bxi, byi, z);
    const int x = threadIdx.x; // bxi == 0: one work-group spans the row
    const int yr = byi * blockDim.y + threadIdx.y;
    const bool valid = yr < g.ny;
    const int y = valid ? yr : g.ny - 1;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    const int row0 = threadIdx.y * blockDim.x;
    // every population load is issued before the barrier (as in
    // k_step_ab_rows), the force's ahead of them where early_force says so
    ForceRaw fr{0.0, 0.0, 0.0};
    if constexpr (early_force<S>()) fr = force_load(ph, g, nb(d, 0, 0, 0), y);
    S direct[L::Q];
    {
        int k = 0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const S v = ld<S, NT>(pop_at<S, O32, true>(buf, g.stride, L::opp(i), nb(d, 0, -L::cy(i), -L::cz(i))));
            if (L::cx(i) != 0) {
                rows[k][row0 + x] = v;
                ++k;
            } else {
                direct[i] = v;
            }
        }
    }
    __syncthreads();
    R s[L::Q];
    {
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
    }
    R Fx, Fy, Fz;
    if constexpr (early_force<S>())
        force_value(ph, fr, Fx, Fy, Fz);
    else
        node_force(ph, g, nb(d, 0, 0, 0), y, Fx, Fy, Fz);
    NodeMacro<R> mac;
    L::template collide<R, GENERAL, Codec<S>::increment>(s, (R)ph.rho0, Fx, Fy, Fz, ph, mac);
    if constexpr (Codec<S>::stochastic) dither_bf16(s, ph.sr_key, (uint32_t)nb(d, 0, 0, 0));
    __syncthreads(); // every staged value has been taken out of LDS
    {
        int k = 0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            if (L::cx(i) != 0) {
                int xd = x + L::cx(i);
                xd = xd < 0 ? xd + g.nx : (xd >= g.nx ? xd - g.nx : xd);
                rows[k][row0 + xd] = Codec<S>::enc(s[i]);
                ++k;
            } else if (valid) {
                st<S, NT>(pop_at<S, O32, true>(buf, g.stride, i, nb(d, 0, L::cy(i), L::cz(i))), Codec<S>::enc(s[i]));
            }
        }
    }
    __syncthreads();
    if (valid) {
        int k = 0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            if (L::cx(i) != 0) {
                st<S, NT>(pop_at<S, O32, true>(buf, g.stride, i, nb(d, 0, L::cy(i), L::cz(i))), rows[k][row0 + x]);
                ++k;
            }
    }
}

// Initialisation at equilibrium from rho, u (double, device).
template <class L, class S, Pattern P, bool WALLS>
__global__ __launch_bounds__(256) void k_init(S* __restrict__ buf, Geom g, double rho0, const double* __restrict__ rho,
                                             const double* __restrict__ u)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    const int n = nb(d, 0, 0, 0);
    R s[L::Q];
    L::template eq<R>((R)rho[n], (R)rho0, (R)u[n], (R)u[g.N + n], (R)u[2 * (int64_t)g.N + n], s);
    place_state<L, S, P, WALLS>(buf, g.stride, d, s);
}

// Populations f = w rho0 + s from double[Q N] (device) into the state.
template <class L, class S, Pattern P, bool WALLS>
__global__ __launch_bounds__(256) void k_set_pops(S* __restrict__ buf, Geom g, double rho0, const double* __restrict__ f)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    const int n = nb(d, 0, 0, 0);
    R s[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) s[i] = (R)(f[(int64_t)i * g.N + n] - L::w(i) * rho0);
    place_state<L, S, P, WALLS>(buf, g.stride, d, s);
}

template <class L, class S, Pattern P, bool WALLS>
__global__ __launch_bounds__(256) void k_get_pops(const S* __restrict__ buf, Geom g, double rho0, double* __restrict__ f)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    NodeIdx d;
    node_idx(g, x, y, z, d);
    const int n = nb(d, 0, 0, 0);
    R s[L::Q];
    gather<L, S, P, WALLS>(buf, g.stride, d, s);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) f[(int64_t)i * g.N + n] = L::w(i) * rho0 + (double)s[i];
}

// ---------------------------------------------------------------------------
// Macroscopic fields and FP64 diagnostics.  Each block reduces its nodes with
// wavefront shuffles then LDS, and writes one partial; k_reduce_partials sums
// the partials in a fixed order (deterministic).
// partial layout: [sum rho, sum rho ux, sum rho uy, sum rho uz, KE, max|u|,
//                  bad count, min rho]
// ---------------------------------------------------------------------------
constexpr int NDIAG = 8;

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline double combine(int k, double a, double b) { return k == 5 ? fmax(a, b) : (k == 7 ? fmin(a, b) : a + b); }

__device__ inline void block_reduce_store(double v[NDIAG], double* __restrict__ out)
{
    __shared__ double lds[NDIAG][16];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int nthreads = blockDim.x * blockDim.y;
    const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int k = 0; k < NDIAG; ++k) {
        double r = (k == 5) ? wave_max(v[k]) : (k == 7 ? wave_min(v[k]) : wave_sum(v[k]));
        if (lane == 0) lds[k][wid] = r;
    }
    __syncthreads();
    if (tid == 0) {
        const int nw = (nthreads + 63) / 64;
        for (int k = 0; k < NDIAG; ++k) {
            double r = lds[k][0];
            for (int w = 1; w < nw; ++w) r = combine(k, r, lds[k][w]);
            out[k] = r;
        }
    }
}

// One work-group per (x-block, y-block) covers the planes z = blockIdx.z,
// blockIdx.z + gridDim.z, ... (one plane when the grid spans all nz planes).
template <class L, class S, Pattern P, bool WALLS>
__global__ __launch_bounds__(256) void k_moments(const S* __restrict__ buf, Geom g, Phys ph, double* __restrict__ rho_out,
                                                double* __restrict__ u_out, double* __restrict__ partials)
{
    using R = typename Codec<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    double v[NDIAG] = {0, 0, 0, 0, 0, 0, 0, 1e300};
    bool first = true;
    for (int z = blockIdx.z; z < g.nz; z += gridDim.z) {
        if (!(x < g.nx && y < g.ny)) break;
        NodeIdx d;
        node_idx(g, x, y, z, d);
        const int n = nb(d, 0, 0, 0);
        R s[L::Q];
        gather<L, S, P, WALLS>(buf, g.stride, d, s);
        double m0 = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const double si = (double)s[i];
            m0 += si;
            if (L::cx(i)) jx += L::cx(i) * si;
            if (L::cy(i)) jy += L::cy(i) * si;
            if (L::cz(i)) jz += L::cz(i) * si;
        }
        R Fx, Fy, Fz;
        node_force(ph, g, n, y, Fx, Fy, Fz);
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
        double w[NDIAG];
        w[0] = rho;
        w[1] = rho * ux;
        w[2] = rho * uy;
        w[3] = rho * uz;
        w[4] = 0.5 * rho * u2;
        w[5] = sqrt(u2);
        w[6] = (isfinite(rho) && isfinite(u2) && rho > 0.0) ? 0.0 : 1.0;
        w[7] = rho;
#pragma unroll
        for (int k = 0; k < NDIAG; ++k) v[k] = first ? w[k] : combine(k, v[k], w[k]);
        first = false;
    }
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    block_reduce_store(v, partials + (int64_t)bid * NDIAG);
}

// ---------------------------------------------------------------------------
// Host-side launchers for one lattice and storage type.
// ---------------------------------------------------------------------------
template <class L, class S> struct Launch {
    static void step(int pattern, bool walls, bool general, bool nt, const void* src, void* dst, const Geom& g,
                     const Phys& ph, dim3 grid, dim3 block, hipStream_t st)
    {
        const S* a = (const S*)src;
        S* b = (S*)dst;
        if (nt)
            step_nt<true>(pattern, walls, general, a, b, g, ph, grid, block, st);
        else
            step_nt<false>(pattern, walls, general, a, b, g, ph, grid, block, st);
    }
    template <bool NT>
    static void step_nt(int pattern, bool walls, bool general, const S* a, S* b, const Geom& g, const Phys& ph,
                        dim3 grid, dim3 block, hipStream_t st)
    {
        // D3Q27 has fixed rates: no general-rate variant
        if (L::Q == 27) general = false;
        // wide work-groups (one per row of 257..1024 nodes; kernels for rows
        // up to 512 or up to 1024) exist only for the staged kernels; every
        // other step kernel of such a launch (the AA even step, and any kernel
        // whose staging rows would not fit in 64 KB of LDS) runs on 256-thread
        // work-groups over the same rows
        const bool wide = block.x > 256;
        constexpr bool wide_fits = moving_x_count<L>() * 512 * sizeof(S) <= 65536;
        constexpr bool fits1024 = moving_x_count<L>() * 1024 * sizeof(S) <= 65536;
        // those 256-thread work-groups take an x width that divides the row
        // where one does (256, 128, 64 or 32 x-values by 1, 2, 4 or 8 rows)
        const int wx = row_width(g.nx);
        const dim3 block256(wide ? wx : block.x, wide ? 256 / wx : block.y, 1);
        const dim3 grid256(wide ? (g.nx + wx - 1) / wx : grid.x, wide ? (g.ny + 256 / wx - 1) / (256 / wx) : grid.y,
                           grid.z);
        // dynamic LDS that caps the resident wavefronts per SIMD (g.occ_waves)
        constexpr unsigned rows256 = moving_x_count<L>() * 256 * sizeof(S);
        constexpr unsigned rows512 = moving_x_count<L>() * 512 * sizeof(S);
        constexpr unsigned rows1024 = moving_x_count<L>() * 1024 * sizeof(S);
        const unsigned pad_r = occ_pad(g, rows256, block), pad_0 = occ_pad(g, 0, block);
        const unsigned pad_w512 = occ_pad(g, rows512, block), pad_w1024 = occ_pad(g, rows1024, block);
        const unsigned pad_256 = occ_pad(g, 0, block256);
#define LBM_STEP_O(P, W, G, O)                                                                                      \
    do {                                                                                                            \
        if constexpr (P == AB && !W) {                                                                              \
            if (g.row_stage && wide) {                                                                              \
                if (block.x > 512) {                                                                                \
                    if constexpr (fits1024) hipLaunchKernelGGL((k_step_ab_rows<L, S, G, NT, O, 1024>), grid, block, pad_w1024, st, a, b, g, ph); \
                    else hipLaunchKernelGGL((k_step_ab<L, S, W, G, NT, O>), grid256, block256, pad_256, st, a, b, g, ph); \
                } else if constexpr (wide_fits) hipLaunchKernelGGL((k_step_ab_rows<L, S, G, NT, O, 512>), grid, block, pad_w512, st, a, b, g, ph); \
                else hipLaunchKernelGGL((k_step_ab<L, S, W, G, NT, O>), grid256, block256, pad_256, st, a, b, g, ph);     \
            } else if (g.row_stage) hipLaunchKernelGGL((k_step_ab_rows<L, S, G, NT, O>), grid, block, pad_r, st, a, b, g, ph); \
            else hipLaunchKernelGGL((k_step_ab<L, S, W, G, NT, O>), grid, block, pad_0, st, a, b, g, ph);              \
        } else if constexpr (P == AB) hipLaunchKernelGGL((k_step_ab<L, S, W, G, NT, O>), grid, block, pad_0, st, a, b, g, ph); \
        else if constexpr (P == AA_ODD && !W) {                                                                     \
            if (g.row_stage && wide) {                                                                              \
                if (block.x > 512) {                                                                                \
                    if constexpr (fits1024) hipLaunchKernelGGL((k_step_aa_odd_rows<L, S, G, NT, O, 1024>), grid, block, pad_w1024, st, b, g, ph); \
                    else hipLaunchKernelGGL((k_step_aa<L, S, P, W, G, NT, O>), grid256, block256, pad_256, st, b, g, ph); \
                } else if constexpr (wide_fits) hipLaunchKernelGGL((k_step_aa_odd_rows<L, S, G, NT, O, 512>), grid, block, pad_w512, st, b, g, ph); \
                else hipLaunchKernelGGL((k_step_aa<L, S, P, W, G, NT, O>), grid256, block256, pad_256, st, b, g, ph);     \
            } else if (g.row_stage) hipLaunchKernelGGL((k_step_aa_odd_rows<L, S, G, NT, O>), grid, block, pad_r, st, b, g, ph); \
            else hipLaunchKernelGGL((k_step_aa<L, S, P, W, G, NT, O>), grid, block, pad_0, st, b, g, ph);               \
        } else if constexpr (P == AA_EVEN && sizeof(S) == 2 && NT) {                                       \
            const dim3 gr = wide ? grid256 : grid, bl = wide ? block256 : block;                            \
            if (g.even_cached) hipLaunchKernelGGL((k_step_aa<L, S, P, W, G, NT, O, false>), gr, bl, wide ? pad_256 : pad_0, st, b, g, ph); \
            else hipLaunchKernelGGL((k_step_aa<L, S, P, W, G, NT, O>), gr, bl, wide ? pad_256 : pad_0, st, b, g, ph);              \
        } else if (wide) hipLaunchKernelGGL((k_step_aa<L, S, P, W, G, NT, O>), grid256, block256, pad_256, st, b, g, ph); \
        else hipLaunchKernelGGL((k_step_aa<L, S, P, W, G, NT, O>), grid, block, pad_0, st, b, g, ph);                   \
    } while (0)
#define LBM_STEP(P, W, G)                        \
    do {                                         \
        if (g.off32) LBM_STEP_O(P, W, G, true);  \
        else LBM_STEP_O(P, W, G, false);         \
    } while (0)
#define LBM_STEP_G(P, W)                                 \
    if constexpr (L::Q == 19) {                          \
        if (general) LBM_STEP(P, W, true);               \
        else LBM_STEP(P, W, false);                      \
    } else {                                             \
        LBM_STEP(P, W, false);                           \
    }
#define LBM_STEP_W(P) \
    if (walls) { LBM_STEP_G(P, true); } else { LBM_STEP_G(P, false); }
        switch (pattern) {
        case AB: LBM_STEP_W(AB); break;
        case AA_EVEN: LBM_STEP_W(AA_EVEN); break;
        default: LBM_STEP_W(AA_ODD); break;
        }
#undef LBM_STEP_W
#undef LBM_STEP_G
#undef LBM_STEP
#undef LBM_STEP_O
    }

#define LBM_DISPATCH_PW(KERNEL, ...)                                                                     \
    switch (pattern) {                                                                                   \
    case AB:                                                                                             \
        if (walls) hipLaunchKernelGGL((KERNEL<L, S, AB, true>), grid, block, 0, st, __VA_ARGS__);          \
        else hipLaunchKernelGGL((KERNEL<L, S, AB, false>), grid, block, 0, st, __VA_ARGS__);               \
        break;                                                                                           \
    case AA_EVEN:                                                                                        \
        if (walls) hipLaunchKernelGGL((KERNEL<L, S, AA_EVEN, true>), grid, block, 0, st, __VA_ARGS__);     \
        else hipLaunchKernelGGL((KERNEL<L, S, AA_EVEN, false>), grid, block, 0, st, __VA_ARGS__);          \
        break;                                                                                           \
    default:                                                                                             \
        if (walls) hipLaunchKernelGGL((KERNEL<L, S, AA_ODD, true>), grid, block, 0, st, __VA_ARGS__);      \
        else hipLaunchKernelGGL((KERNEL<L, S, AA_ODD, false>), grid, block, 0, st, __VA_ARGS__);           \
    }

    static void init(int pattern, bool walls, void* buf, const Geom& g, double rho0, const double* rho, const double* u,
                     dim3 grid, dim3 block, hipStream_t st)
    {
        LBM_DISPATCH_PW(k_init, (S*)buf, g, rho0, rho, u);
    }
    static void set_pops(int pattern, bool walls, void* buf, const Geom& g, double rho0, const double* f, dim3 grid,
                         dim3 block, hipStream_t st)
    {
        LBM_DISPATCH_PW(k_set_pops, (S*)buf, g, rho0, f);
    }
    static void get_pops(int pattern, bool walls, const void* buf, const Geom& g, double rho0, double* f, dim3 grid,
                         dim3 block, hipStream_t st)
    {
        LBM_DISPATCH_PW(k_get_pops, (const S*)buf, g, rho0, f);
    }
    static void moments(int pattern, bool walls, const void* buf, const Geom& g, const Phys& ph, double* rho, double* u,
                        double* partials, dim3 grid, dim3 block, hipStream_t st)
    {
        LBM_DISPATCH_PW(k_moments, (const S*)buf, g, ph, rho, u, partials);
    }
#undef LBM_DISPATCH_PW
};

} // namespace lbm
