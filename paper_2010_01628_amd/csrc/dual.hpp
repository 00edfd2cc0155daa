// First-order dual numbers: a value and its derivative along one direction.
// The collision's device functions are templates on their real type and use
// only + - * / and constants, so evaluating them on Dual gives the
// directional derivative of the post-collision populations (forward-mode
// differentiation) without a second, hand-differentiated copy of the scheme.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

struct Dual {
    float v, d;
    Dual() = default;
    __host__ __device__ constexpr Dual(double c) : v((float)c), d(0.0f) {}
    __host__ __device__ constexpr Dual(float a, float b) : v(a), d(b) {}
};

__host__ __device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__host__ __device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__host__ __device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__host__ __device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__host__ __device__ inline Dual operator/(Dual a, Dual b)
{
    const float q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
__host__ __device__ inline Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
__host__ __device__ inline Dual& operator-=(Dual& a, Dual b) { return a = a - b; }

} // namespace lbm
