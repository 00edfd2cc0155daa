// D3Q19 central-moment collision for gfx950 -- device functions.
//
// The method is the D3Q19-CM-LBM of De Rosis & Coreixas (arXiv 2010.01628),
// Sec. II.B: k = T(u) f, k* = (I - K) k + K k_eq + (I - K/2) R, f* = T(u)^-1 k*.
// This file evaluates that map in a form chosen for FP32 accuracy and low
// operation count, not the paper's closed forms:
//
//   * every quantity is carried as a deviation: populations are stored as
//     s_i = f_i - w_i rho0, raw moments as m - rho0 W (W the raw moments of the
//     rest weights), and the collision works on non-equilibrium moments
//     m - m_eq(rho, u), so no step subtracts two O(1) numbers;
//   * raw moments come from +-1 sums over the three face-diagonal groups and
//     the three axes (the monomial set of the paper's basis is closed under
//     lowering any exponent, so each central moment is reached by three 1-D
//     binomial sweeps, one per axis: T = N M of App. C with N applied as
//     x-, y- and z-shifts);
//   * relaxation happens in the paper's basis rows (trace k4, deviators
//     k5..k9, third order k10..k15, fourth order k16..k18) and the result is
//     swept back with +u and mapped to populations by the inverse of M written
//     per velocity group.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q19 = 19;

// Sec. II.A velocity order.
__host__ __device__ constexpr int cx19(int i)
{
    constexpr int v[19] = {0, -1, 0, 0, -1, -1, -1, -1, 0, 0, 1, 0, 0, 1, 1, 1, 1, 0, 0};
    return v[i];
}
__host__ __device__ constexpr int cy19(int i)
{
    constexpr int v[19] = {0, 0, -1, 0, -1, 1, 0, 0, -1, -1, 0, 1, 0, 1, -1, 0, 0, 1, 1};
    return v[i];
}
__host__ __device__ constexpr int cz19(int i)
{
    constexpr int v[19] = {0, 0, 0, -1, 0, 0, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int opp19(int i) { return i == 0 ? 0 : (i <= 9 ? i + 9 : i - 9); }
__host__ __device__ constexpr double w19(int i)
{
    return i == 0 ? 1.0 / 3.0 : (((i >= 1 && i <= 3) || (i >= 10 && i <= 12)) ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ---------------------------------------------------------------------------
// Storage codecs.  FP16 and BF16 use the hardware round-to-nearest-even
// conversions.
// ---------------------------------------------------------------------------
struct bf16_t {
    uint16_t bits;
};

template <class S> struct Codec;
// increment: the collision returns s + (f* - f), the change computed from the
// non-equilibrium moments alone (post_collide_increment), rather than f*
// rebuilt from its moments (post_collide).  Used for FP32 storage, whose
// long-run error it keeps at the storage rounding's; the rebuilt form's
// roundings, relative to the equilibrium-sized moments, add ~100 times that.
template <> struct Codec<double> {
    static constexpr bool stochastic = false;
    static constexpr bool increment = false;
    using R = double;
    __device__ static inline double dec(double v) { return v; }
    __device__ static inline double enc(double v) { return v; }
};
template <> struct Codec<float> {
    static constexpr bool stochastic = false;
    static constexpr bool increment = true;
    using R = float;
    __device__ static inline float dec(float v) { return v; }
    __device__ static inline float enc(float v) { return v; }
};
template <> struct Codec<_Float16> {
    static constexpr bool stochastic = false;
    static constexpr bool increment = false;
    using R = float;
    __device__ static inline float dec(_Float16 v) { return (float)v; }
    // the empty asm keeps the last FP32 operation of the collision from being
    // fused into a mixed-precision FMA with the conversion: the value is
    // rounded to FP32 first, then RNE to FP16 (and the plain conversion timed
    // ~1.5 % faster in the 16-bit step)
    __device__ static inline _Float16 enc(float v)
    {
        asm("" : "+v"(v));
        return (_Float16)v;
    }
};
template <> struct Codec<bf16_t> {
    static constexpr bool stochastic = false;
    static constexpr bool increment = false;
    using R = float;
    __device__ static inline float dec(bf16_t v) { return __uint_as_float((uint32_t)v.bits << 16); }
    // gfx950's conversion instruction (v_cvt_pk_bf16_f32): round to nearest
    // even, one instruction instead of the bit-pattern rounding's six
    __device__ static inline bf16_t enc(float v)
    {
        const __bf16 b = (__bf16)v;
        return bf16_t{__builtin_bit_cast(uint16_t, b)};
    }
};

// BF16 storage with stochastic rounding: after the collision the step kernels
// round each population to a BF16 value themselves (dither_bf16): uniform
// random bits are added below the 16 kept ones of its FP32 pattern and the
// low 16 bits are cut, so it rounds up with probability equal to the fraction
// it lies above the lower BF16 neighbour.  The stored value is then exact in
// BF16 and enc (nearest even, as for bf16_t, which init and
// lbm_set_populations also use) keeps it.  Same layout and decoding as bf16_t.
struct bf16sr_t {
    uint16_t bits;
};
template <> struct Codec<bf16sr_t> {
    static constexpr bool stochastic = true;
    static constexpr bool increment = false;
    using R = float;
    __device__ static inline float dec(bf16sr_t v) { return __uint_as_float((uint32_t)v.bits << 16); }
    __device__ static inline bf16sr_t enc(float v) { return bf16sr_t{Codec<bf16_t>::enc(v).bits}; }
};

// 32-bit integer hash "lowbias32" (C. Wellons, hash prospector; public
// domain): xor-shift / multiply rounds, a bijection of 32-bit integers.
__host__ __device__ inline uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Stochastic rounding to BF16, counter-based: the post-collision populations
// of node n in the step whose key is `key` (a hash of the seed and the step
// count) take 16 random bits each from hash32(10 n + j + key), j = i / 2 (low
// half for even i, high half for odd i), added to their FP32 patterns before
// the low 16 bits are cut.  NaN and infinity are left alone.  The bits depend
// on (seed, step, node, population) only: A-B and AA steps store the same
// values.
template <class R> __device__ inline void dither_bf16(R s[19], uint32_t key, uint32_t n)
{
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        const uint32_t h = hash32(10u * n + (uint32_t)j + key);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int i = 2 * j + k;
            if (i < 19) {
                const uint32_t u = __float_as_uint(s[i]);
                const uint32_t r = k ? (h >> 16) : (h & 0xffffu);
                // finite: the exponent field is not all ones (one class test)
                if (__builtin_isfinite(s[i])) s[i] = __uint_as_float((u + r) & 0xffff0000u);
            }
        }
    }
}

// Relaxation rates of the non-conserved rows of K (Sec. II.B).
template <class R> struct Rates {
    R omega;      // k5..k9
    R omega_bulk; // k4
    R omega_hi[9];// k10..k18
};

// Output of a collision besides the new populations.
template <class R> struct NodeMacro {
    R rho, ux, uy, uz;
};

// Deviation raw moments S_pqr = sum_i s_i cx^p cy^q cz^r in the monomial set of
// the paper's basis.
template <class R> struct RawMoments {
    R m000, m100, m010, m001;
    R m200, m020, m002, m110, m101, m011;
    R m210, m120, m201, m102, m021, m012;
    R m220, m202, m022;
};

template <class R> __host__ __device__ inline void raw_from_pops(const R s[19], RawMoments<R>& m)
{
    // xy face diagonals 4(-,-) 5(-,+) 13(+,+) 14(+,-)
    m.m220 = (s[4] + s[5]) + (s[13] + s[14]);
    m.m110 = (s[4] - s[5]) + (s[13] - s[14]);
    m.m210 = (s[5] - s[4]) + (s[13] - s[14]);
    m.m120 = (s[13] + s[14]) - (s[4] + s[5]);
    // xz face diagonals 6(-,-) 7(-,+) 15(+,+) 16(+,-)
    m.m202 = (s[6] + s[7]) + (s[15] + s[16]);
    m.m101 = (s[6] - s[7]) + (s[15] - s[16]);
    m.m201 = (s[7] - s[6]) + (s[15] - s[16]);
    m.m102 = (s[15] + s[16]) - (s[6] + s[7]);
    // yz face diagonals 8(-,-) 9(-,+) 17(+,+) 18(+,-)
    m.m022 = (s[8] + s[9]) + (s[17] + s[18]);
    m.m011 = (s[8] - s[9]) + (s[17] - s[18]);
    m.m021 = (s[9] - s[8]) + (s[17] - s[18]);
    m.m012 = (s[17] + s[18]) - (s[8] + s[9]);
    // axes
    const R ax = s[1] + s[10], ay = s[2] + s[11], az = s[3] + s[12];
    m.m200 = ax + m.m220 + m.m202;
    m.m020 = ay + m.m220 + m.m022;
    m.m002 = az + m.m202 + m.m022;
    m.m100 = (s[10] - s[1]) + m.m120 + m.m102;
    m.m010 = (s[11] - s[2]) + m.m210 + m.m012;
    m.m001 = (s[12] - s[3]) + m.m201 + m.m021;
    m.m000 = s[0] + (ax + ay + az) + (m.m220 + m.m202 + m.m022);
}

// Populations from deviation raw moments (inverse of raw_from_pops).
template <class R> __host__ __device__ inline void pops_from_raw(const RawMoments<R>& m, R s[19])
{
    const R q = R(0.25), h = R(0.5);
    s[13] = q * ((m.m220 + m.m110) + (m.m210 + m.m120));
    s[4] = q * ((m.m220 + m.m110) - (m.m210 + m.m120));
    s[5] = q * ((m.m220 - m.m110) + (m.m210 - m.m120));
    s[14] = q * ((m.m220 - m.m110) - (m.m210 - m.m120));
    s[15] = q * ((m.m202 + m.m101) + (m.m201 + m.m102));
    s[6] = q * ((m.m202 + m.m101) - (m.m201 + m.m102));
    s[7] = q * ((m.m202 - m.m101) + (m.m201 - m.m102));
    s[16] = q * ((m.m202 - m.m101) - (m.m201 - m.m102));
    s[17] = q * ((m.m022 + m.m011) + (m.m021 + m.m012));
    s[8] = q * ((m.m022 + m.m011) - (m.m021 + m.m012));
    s[9] = q * ((m.m022 - m.m011) + (m.m021 - m.m012));
    s[18] = q * ((m.m022 - m.m011) - (m.m021 - m.m012));
    const R ax = m.m200 - (m.m220 + m.m202), dx = m.m100 - (m.m120 + m.m102);
    const R ay = m.m020 - (m.m220 + m.m022), dy = m.m010 - (m.m210 + m.m012);
    const R az = m.m002 - (m.m202 + m.m022), dz = m.m001 - (m.m201 + m.m021);
    s[10] = h * (ax + dx);
    s[1] = h * (ax - dx);
    s[11] = h * (ay + dy);
    s[2] = h * (ay - dy);
    s[12] = h * (az + dz);
    s[3] = h * (az - dz);
    s[0] = m.m000 - (ax + ay + az) - (m.m220 + m.m202 + m.m022);
}

// Equilibrium raw moments minus the rest ones: m_eq(rho, u) - rho0 W, with
// m_eq the raw moments of the extended equilibrium (those of T^-1 k_eq).
template <class R>
__host__ __device__ inline void eq_raw_deviation(R drho, R rho, R ux, R uy, R uz, RawMoments<R>& d)
{
    const R t = R(1) / R(3), n = R(1) / R(9);
    const R x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
    const R rx = rho * ux, ry = rho * uy, rz = rho * uz;
    d.m000 = drho;
    d.m100 = rx;
    d.m010 = ry;
    d.m001 = rz;
    d.m200 = drho * t + rho * x2;
    d.m020 = drho * t + rho * y2;
    d.m002 = drho * t + rho * z2;
    d.m110 = rx * uy;
    d.m101 = rx * uz;
    d.m011 = ry * uz;
    d.m210 = ry * (x2 + t);
    d.m120 = rx * (y2 + t);
    d.m201 = rz * (x2 + t);
    d.m102 = rx * (z2 + t);
    d.m021 = rz * (y2 + t);
    d.m012 = ry * (z2 + t);
    d.m220 = drho * n + rho * (x2 * y2 + (x2 + y2) * t);
    d.m202 = drho * n + rho * (x2 * z2 + (x2 + z2) * t);
    d.m022 = drho * n + rho * (y2 * z2 + (y2 + z2) * t);
}

// 1-D binomial shift of a chain (v0, v1, v2) of moments with exponents 0,1,2
// along one axis by a: v_p <- sum_k C(p,k) a^(p-k) v_k.
template <class R> __host__ __device__ inline void shift3(R v0, R& v1, R& v2, R a)
{
    const R n2 = v2 + a * (R(2) * v1 + a * v0);
    v1 = v1 + a * v0;
    v2 = n2;
}
template <class R> __host__ __device__ inline void shift2(R v0, R& v1, R a) { v1 = v1 + a * v0; }

// Shift every moment of the monomial set by (a, b, c): central moments from raw
// ones with (a,b,c) = -u, raw from central with +u.  m000 is left unchanged.
template <class R> __host__ __device__ inline void shift_all(RawMoments<R>& m, R a, R b, R c)
{
    // x sweeps along chains with fixed (q, r)
    shift3(m.m000, m.m100, m.m200, a);
    shift3(m.m010, m.m110, m.m210, a);
    shift3(m.m001, m.m101, m.m201, a);
    shift3(m.m020, m.m120, m.m220, a);
    shift3(m.m002, m.m102, m.m202, a);
    // y sweeps along chains with fixed (p, r)
    shift3(m.m000, m.m010, m.m020, b);
    shift3(m.m100, m.m110, m.m120, b);
    shift3(m.m200, m.m210, m.m220, b);
    shift3(m.m001, m.m011, m.m021, b);
    shift3(m.m002, m.m012, m.m022, b);
    // z sweeps along chains with fixed (p, q)
    shift3(m.m000, m.m001, m.m002, c);
    shift3(m.m100, m.m101, m.m102, c);
    shift3(m.m010, m.m011, m.m012, c);
    shift3(m.m200, m.m201, m.m202, c);
    shift3(m.m020, m.m021, m.m022, c);
}

// State between the two halves of a collision: macroscopic fields, the
// equilibrium raw-moment deviation and the pre-collision non-equilibrium
// central moments (monomial form; k4 trace and k5, k6 deviators of the paper's
// rows precomputed).
template <class R> struct CMState {
    R rho, drho, ux, uy, uz, Fx, Fy, Fz;
    RawMoments<R> e; // m_eq(rho, u) - rho0 W
    RawMoments<R> n; // non-equilibrium central moments (n.m000 = 0, n.m100 = -Fx/2, ...)
    R k4, k5, k6;
};

// First half of the collision of Sec. II.B: moments, equilibrium and the
// pre-collision non-equilibrium CMs.  GENERAL = false skips the third- and
// fourth-order CMs (not needed when their rates are 1).
template <class R, bool GENERAL>
__host__ __device__ inline void pre_collide(const R s[19], R rho0, R Fx, R Fy, R Fz, CMState<R>& st)
{
    RawMoments<R> m;
    raw_from_pops(s, m);
    st.drho = m.m000;
    st.rho = rho0 + st.drho;
    const R irho = R(1) / st.rho;
    st.ux = (m.m100 + R(0.5) * Fx) * irho;
    st.uy = (m.m010 + R(0.5) * Fy) * irho;
    st.uz = (m.m001 + R(0.5) * Fz) * irho;
    st.Fx = Fx;
    st.Fy = Fy;
    st.Fz = Fz;
    eq_raw_deviation(st.drho, st.rho, st.ux, st.uy, st.uz, st.e);
    RawMoments<R>& n = st.n;
    const RawMoments<R>& e = st.e;
    n.m000 = R(0);
    n.m100 = R(-0.5) * Fx;
    n.m010 = R(-0.5) * Fy;
    n.m001 = R(-0.5) * Fz;
    n.m200 = m.m200 - e.m200;
    n.m020 = m.m020 - e.m020;
    n.m002 = m.m002 - e.m002;
    n.m110 = m.m110 - e.m110;
    n.m101 = m.m101 - e.m101;
    n.m011 = m.m011 - e.m011;
    if constexpr (GENERAL) {
        n.m210 = m.m210 - e.m210;
        n.m120 = m.m120 - e.m120;
        n.m201 = m.m201 - e.m201;
        n.m102 = m.m102 - e.m102;
        n.m021 = m.m021 - e.m021;
        n.m012 = m.m012 - e.m012;
        n.m220 = m.m220 - e.m220;
        n.m202 = m.m202 - e.m202;
        n.m022 = m.m022 - e.m022;
    } else {
        n.m210 = n.m120 = n.m201 = n.m102 = n.m021 = n.m012 = n.m220 = n.m202 = n.m022 = R(0);
    }
    // central non-equilibrium moments (shift by -u)
    shift_all(n, -st.ux, -st.uy, -st.uz);
    st.k4 = n.m200 + n.m020 + n.m002;
    st.k5 = n.m200 - n.m020;
    st.k6 = n.m020 - n.m002;
}

// Post-collision non-equilibrium CMs, k* - k_eq = (I - K)(k - k_eq) + (I - K/2) R
// (eq. posColl0), in monomial form.
template <class R, bool GENERAL>
__host__ __device__ inline void relax(const CMState<R>& st, const Rates<R>& rt, RawMoments<R>& p)
{
    const R third = R(1) / R(3), cs2 = third;
    const RawMoments<R>& n = st.n;
    const R Fx = st.Fx, Fy = st.Fy, Fz = st.Fz;
    const R w1 = R(1) - rt.omega;
    const R s5 = w1 * st.k5, s6 = w1 * st.k6;
    R s4 = R(0);
    p.m000 = R(0);
    p.m100 = R(0.5) * Fx;
    p.m010 = R(0.5) * Fy;
    p.m001 = R(0.5) * Fz;
    p.m110 = w1 * n.m110;
    p.m101 = w1 * n.m101;
    p.m011 = w1 * n.m011;
    if constexpr (GENERAL) {
        s4 = (R(1) - rt.omega_bulk) * st.k4;
        const R* oh = rt.omega_hi;
        p.m210 = (R(1) - oh[0]) * n.m210 + (R(1) - R(0.5) * oh[0]) * cs2 * Fy;
        p.m120 = (R(1) - oh[1]) * n.m120 + (R(1) - R(0.5) * oh[1]) * cs2 * Fx;
        p.m201 = (R(1) - oh[2]) * n.m201 + (R(1) - R(0.5) * oh[2]) * cs2 * Fz;
        p.m102 = (R(1) - oh[3]) * n.m102 + (R(1) - R(0.5) * oh[3]) * cs2 * Fx;
        p.m021 = (R(1) - oh[4]) * n.m021 + (R(1) - R(0.5) * oh[4]) * cs2 * Fz;
        p.m012 = (R(1) - oh[5]) * n.m012 + (R(1) - R(0.5) * oh[5]) * cs2 * Fy;
        p.m220 = (R(1) - oh[6]) * n.m220;
        p.m202 = (R(1) - oh[7]) * n.m202;
        p.m022 = (R(1) - oh[8]) * n.m022;
    } else {
        const R hf = R(0.5) * cs2;
        p.m210 = hf * Fy;
        p.m120 = hf * Fx;
        p.m201 = hf * Fz;
        p.m102 = hf * Fx;
        p.m021 = hf * Fz;
        p.m012 = hf * Fy;
        p.m220 = p.m202 = p.m022 = R(0);
    }
    p.m200 = third * (s4 + R(2) * s5 + s6);
    p.m020 = third * (s4 - s5 + s6);
    p.m002 = third * (s4 - s5 - R(2) * s6);
}

// Second half: back to raw moments (shift by +u), add the equilibrium
// deviation, populations by M^-1.
template <class R> __host__ __device__ inline void post_collide(const CMState<R>& st, RawMoments<R>& p, R s[19])
{
    const RawMoments<R>& e = st.e;
    shift_all(p, st.ux, st.uy, st.uz);
    p.m000 = e.m000;
    p.m100 += e.m100;
    p.m010 += e.m010;
    p.m001 += e.m001;
    p.m200 += e.m200;
    p.m020 += e.m020;
    p.m002 += e.m002;
    p.m110 += e.m110;
    p.m101 += e.m101;
    p.m011 += e.m011;
    p.m210 += e.m210;
    p.m120 += e.m120;
    p.m201 += e.m201;
    p.m102 += e.m102;
    p.m021 += e.m021;
    p.m012 += e.m012;
    p.m220 += e.m220;
    p.m202 += e.m202;
    p.m022 += e.m022;
    pops_from_raw(p, s);
}

// Second half in increment form: f* - f = T(u)^-1 (k* - k), where k* - k =
// -K (k - k_eq) + (I - K/2) R is formed from the non-equilibrium CMs, then
// shifted back with +u and mapped to populations; s += that change.  Every
// term is of the size of the non-equilibrium part, so the only rounding of
// equilibrium size is the final addition.  st.n must hold all non-equilibrium
// CMs (pre_collide with GENERAL = true).
template <class R> __host__ __device__ inline void post_collide_increment(const CMState<R>& st, RawMoments<R>& p, R s[19])
{
    const RawMoments<R>& n = st.n;
    p.m000 = R(0);
    p.m100 -= n.m100;
    p.m010 -= n.m010;
    p.m001 -= n.m001;
    p.m200 -= n.m200;
    p.m020 -= n.m020;
    p.m002 -= n.m002;
    p.m110 -= n.m110;
    p.m101 -= n.m101;
    p.m011 -= n.m011;
    p.m210 -= n.m210;
    p.m120 -= n.m120;
    p.m201 -= n.m201;
    p.m102 -= n.m102;
    p.m021 -= n.m021;
    p.m012 -= n.m012;
    p.m220 -= n.m220;
    p.m202 -= n.m202;
    p.m022 -= n.m022;
    shift_all(p, st.ux, st.uy, st.uz);
    R d[19];
    pops_from_raw(p, d);
#pragma unroll
    for (int i = 0; i < 19; ++i) s[i] += d[i];
}

// The collision of Sec. II.B eq. (posColl0) applied to deviations s (in place).
// GENERAL = false assumes the paper's rates (omega_bulk = 1, omega_hi = 1);
// INC selects the increment form of the second half.
template <class R, bool GENERAL, bool INC = false>
__host__ __device__ inline void collide_cm(R s[19], R rho0, R Fx, R Fy, R Fz, const Rates<R>& rt, NodeMacro<R>& mac)
{
    CMState<R> st;
    pre_collide<R, GENERAL || INC>(s, rho0, Fx, Fy, Fz, st);
    mac.rho = st.rho;
    mac.ux = st.ux;
    mac.uy = st.uy;
    mac.uz = st.uz;
    RawMoments<R> p;
    relax<R, GENERAL>(st, rt, p);
    if constexpr (INC)
        post_collide_increment(st, p, s);
    else
        post_collide(st, p, s);
}

// Raw-moment variant (App. C with N = I, the classical MRT in the paper's
// basis): the same relaxation applied to un-shifted moments, towards the raw
// equilibrium, with the raw moments of the forcing term of App. B (eq. RMQ19).
// No binomial shifts.  GENERAL = false assumes the paper's rates.
template <class R, bool GENERAL>
__host__ __device__ inline void collide_rm(R s[19], R rho0, R Fx, R Fy, R Fz, const Rates<R>& rt, NodeMacro<R>& mac)
{
    RawMoments<R> m;
    raw_from_pops(s, m);
    const R drho = m.m000, rho = rho0 + drho, irho = R(1) / rho;
    const R ux = (m.m100 + R(0.5) * Fx) * irho;
    const R uy = (m.m010 + R(0.5) * Fy) * irho;
    const R uz = (m.m001 + R(0.5) * Fz) * irho;
    mac.rho = rho;
    mac.ux = ux;
    mac.uy = uy;
    mac.uz = uz;
    RawMoments<R> e;
    eq_raw_deviation(drho, rho, ux, uy, uz, e);
    const R third = R(1) / R(3), cs2 = third;
    // second-order forcing moments: 2 u_a F_a on the diagonal, u_a F_b + u_b F_a off it
    const R fxx = R(2) * ux * Fx, fyy = R(2) * uy * Fy, fzz = R(2) * uz * Fz;
    const R w1 = R(1) - rt.omega, h1 = R(1) - R(0.5) * rt.omega;
    const R n5 = (m.m200 - e.m200) - (m.m020 - e.m020);
    const R n6 = (m.m020 - e.m020) - (m.m002 - e.m002);
    const R p5 = w1 * n5 + h1 * (fxx - fyy);
    const R p6 = w1 * n6 + h1 * (fyy - fzz);
    R p4;
    if constexpr (GENERAL) {
        const R n4 = (m.m200 - e.m200) + (m.m020 - e.m020) + (m.m002 - e.m002);
        p4 = (R(1) - rt.omega_bulk) * n4 + (R(1) - R(0.5) * rt.omega_bulk) * (fxx + fyy + fzz);
    } else {
        p4 = R(0.5) * (fxx + fyy + fzz);
    }
    RawMoments<R> p;
    p.m000 = e.m000;
    p.m100 = e.m100 + R(0.5) * Fx;
    p.m010 = e.m010 + R(0.5) * Fy;
    p.m001 = e.m001 + R(0.5) * Fz;
    p.m200 = e.m200 + third * (p4 + R(2) * p5 + p6);
    p.m020 = e.m020 + third * (p4 - p5 + p6);
    p.m002 = e.m002 + third * (p4 - p5 - R(2) * p6);
    p.m110 = e.m110 + w1 * (m.m110 - e.m110) + h1 * (ux * Fy + uy * Fx);
    p.m101 = e.m101 + w1 * (m.m101 - e.m101) + h1 * (ux * Fz + uz * Fx);
    p.m011 = e.m011 + w1 * (m.m011 - e.m011) + h1 * (uy * Fz + uz * Fy);
    // third- and fourth-order forcing moments
    const R f210 = cs2 * Fy + ux * (ux * Fy + R(2) * uy * Fx);
    const R f120 = cs2 * Fx + uy * (uy * Fx + R(2) * ux * Fy);
    const R f201 = cs2 * Fz + ux * (ux * Fz + R(2) * uz * Fx);
    const R f102 = cs2 * Fx + uz * (uz * Fx + R(2) * ux * Fz);
    const R f021 = cs2 * Fz + uy * (uy * Fz + R(2) * uz * Fy);
    const R f012 = cs2 * Fy + uz * (uz * Fy + R(2) * uy * Fz);
    const R f220 = R(2) * (ux * uy * (ux * Fy + uy * Fx) + cs2 * (ux * Fx + uy * Fy));
    const R f202 = R(2) * (ux * uz * (ux * Fz + uz * Fx) + cs2 * (ux * Fx + uz * Fz));
    const R f022 = R(2) * (uy * uz * (uy * Fz + uz * Fy) + cs2 * (uy * Fy + uz * Fz));
    if constexpr (GENERAL) {
        const R* oh = rt.omega_hi;
        auto rel = [](R mm, R ee, R ff, R w) { return ee + (R(1) - w) * (mm - ee) + (R(1) - R(0.5) * w) * ff; };
        p.m210 = rel(m.m210, e.m210, f210, oh[0]);
        p.m120 = rel(m.m120, e.m120, f120, oh[1]);
        p.m201 = rel(m.m201, e.m201, f201, oh[2]);
        p.m102 = rel(m.m102, e.m102, f102, oh[3]);
        p.m021 = rel(m.m021, e.m021, f021, oh[4]);
        p.m012 = rel(m.m012, e.m012, f012, oh[5]);
        p.m220 = rel(m.m220, e.m220, f220, oh[6]);
        p.m202 = rel(m.m202, e.m202, f202, oh[7]);
        p.m022 = rel(m.m022, e.m022, f022, oh[8]);
    } else {
        p.m210 = e.m210 + R(0.5) * f210;
        p.m120 = e.m120 + R(0.5) * f120;
        p.m201 = e.m201 + R(0.5) * f201;
        p.m102 = e.m102 + R(0.5) * f102;
        p.m021 = e.m021 + R(0.5) * f021;
        p.m012 = e.m012 + R(0.5) * f012;
        p.m220 = e.m220 + R(0.5) * f220;
        p.m202 = e.m202 + R(0.5) * f202;
        p.m022 = e.m022 + R(0.5) * f022;
    }
    pops_from_raw(p, s);
}

// ---------------------------------------------------------------------------
// Adjoints (transposes) of the linear maps of the back-transform, for the
// gradient of a loss on post-collision populations with respect to the
// post-collision CMs: s* = M^-1 (S(+u) k* + e) gives kbar = S(+u)^T M^-T sbar.
// ---------------------------------------------------------------------------
template <class R> __host__ __device__ inline void pops_from_raw_T(const R g[19], RawMoments<R>& m)
{
    const R q = R(0.25), h = R(0.5);
    const R ax = h * (g[10] + g[1]) - g[0], dx = h * (g[10] - g[1]);
    const R ay = h * (g[11] + g[2]) - g[0], dy = h * (g[11] - g[2]);
    const R az = h * (g[12] + g[3]) - g[0], dz = h * (g[12] - g[3]);
    m.m000 = g[0];
    m.m200 = ax;
    m.m020 = ay;
    m.m002 = az;
    m.m100 = dx;
    m.m010 = dy;
    m.m001 = dz;
    m.m220 = q * ((g[13] + g[4]) + (g[5] + g[14])) - ax - ay - g[0];
    m.m110 = q * ((g[13] + g[4]) - (g[5] + g[14]));
    m.m210 = q * ((g[13] - g[4]) + (g[5] - g[14])) - dy;
    m.m120 = q * ((g[13] - g[4]) - (g[5] - g[14])) - dx;
    m.m202 = q * ((g[15] + g[6]) + (g[7] + g[16])) - ax - az - g[0];
    m.m101 = q * ((g[15] + g[6]) - (g[7] + g[16]));
    m.m201 = q * ((g[15] - g[6]) + (g[7] - g[16])) - dz;
    m.m102 = q * ((g[15] - g[6]) - (g[7] - g[16])) - dx;
    m.m022 = q * ((g[17] + g[8]) + (g[9] + g[18])) - ay - az - g[0];
    m.m011 = q * ((g[17] + g[8]) - (g[9] + g[18]));
    m.m021 = q * ((g[17] - g[8]) + (g[9] - g[18])) - dz;
    m.m012 = q * ((g[17] - g[8]) - (g[9] - g[18])) - dy;
}

// transpose of shift3: (g0, g1, g2) <- (g0 + a g1 + a^2 g2, g1 + 2 a g2, g2)
template <class R> __host__ __device__ inline void shift3_T(R& g0, R& g1, R g2, R a)
{
    g0 = g0 + a * (g1 + a * g2);
    g1 = g1 + R(2) * a * g2;
}

// transpose of shift_all: the sweeps in reverse order
template <class R> __host__ __device__ inline void shift_all_T(RawMoments<R>& m, R a, R b, R c)
{
    shift3_T(m.m000, m.m001, m.m002, c);
    shift3_T(m.m100, m.m101, m.m102, c);
    shift3_T(m.m010, m.m011, m.m012, c);
    shift3_T(m.m200, m.m201, m.m202, c);
    shift3_T(m.m020, m.m021, m.m022, c);
    shift3_T(m.m000, m.m010, m.m020, b);
    shift3_T(m.m100, m.m110, m.m120, b);
    shift3_T(m.m200, m.m210, m.m220, b);
    shift3_T(m.m001, m.m011, m.m021, b);
    shift3_T(m.m002, m.m012, m.m022, b);
    shift3_T(m.m000, m.m100, m.m200, a);
    shift3_T(m.m010, m.m110, m.m210, a);
    shift3_T(m.m001, m.m101, m.m201, a);
    shift3_T(m.m020, m.m120, m.m220, a);
    shift3_T(m.m002, m.m102, m.m202, a);
}

// Deviations of the extended equilibrium f_eq(rho, u) - w rho0 (eq. EqQ19RM),
// through its raw moments.
template <class R> __host__ __device__ inline void equilibrium_deviation(R rho, R rho0, R ux, R uy, R uz, R s[19])
{
    RawMoments<R> e;
    eq_raw_deviation(rho - rho0, rho, ux, uy, uz, e);
    pops_from_raw(e, s);
}

} // namespace lbm
