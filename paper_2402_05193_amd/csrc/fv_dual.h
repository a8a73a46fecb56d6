// fv_dual.h -- first-order forward-mode differentiation of the point-wise
// device functions of fv_physics.h.
//
// Dual<T> carries a value and one directional derivative.  The templated
// point-wise functions (U->W map, WENO5-Z, HLLC) instantiated with Dual<double>
// return the derivative of exactly the arithmetic the stage kernel performs.
// Non-differentiable points take the conventions of the adjoint's reference:
// |x|' = sgn(x) with sgn(0) = 0; min/max at a tie split the derivative evenly;
// the upwind switch of the HLLC flux is piecewise constant (derivative 0).
// The hardware-estimate helpers (rcp, rsqrt, sqrt_fast) are differentiated
// exactly (d(1/x) = -dx/x^2, ...), not through their Newton refinement.
#pragma once

#include "fv_physics.h"

namespace fv {

template <typename T>
struct Dual {
    T v, d;
    __device__ __forceinline__ Dual() = default;
    __device__ __forceinline__ constexpr Dual(T x) : v(x), d(T(0)) {}
    __device__ __forceinline__ constexpr Dual(T x, T dx) : v(x), d(dx) {}
};

template <typename T>
__device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator/(Dual<T> a, Dual<T> b)
{
    const T q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
template <typename T>
__device__ __forceinline__ Dual<T>& operator+=(Dual<T>& a, Dual<T> b) { return a = a + b; }
template <typename T>
__device__ __forceinline__ Dual<T>& operator-=(Dual<T>& a, Dual<T> b) { return a = a - b; }

template <typename T>
__device__ __forceinline__ bool operator<(Dual<T> a, Dual<T> b) { return a.v < b.v; }
template <typename T>
__device__ __forceinline__ bool operator>(Dual<T> a, Dual<T> b) { return a.v > b.v; }
template <typename T>
__device__ __forceinline__ bool operator<=(Dual<T> a, Dual<T> b) { return a.v <= b.v; }
template <typename T>
__device__ __forceinline__ bool operator>=(Dual<T> a, Dual<T> b) { return a.v >= b.v; }
template <typename T>
__device__ __forceinline__ bool operator==(Dual<T> a, Dual<T> b) { return a.v == b.v; }

template <typename T>
__device__ __forceinline__ Dual<T> fma(Dual<T> a, Dual<T> b, Dual<T> c)
{
    return {a.v * b.v + c.v, a.d * b.v + a.v * b.d + c.d};
}
template <typename T>
__device__ __forceinline__ Dual<T> fabs(Dual<T> a)
{
    const T s = a.v > T(0) ? T(1) : (a.v < T(0) ? T(-1) : T(0));
    return {a.v < T(0) ? -a.v : a.v, s * a.d};
}
template <typename T>
__device__ __forceinline__ Dual<T> fmin(Dual<T> a, Dual<T> b)
{
    if (a.v < b.v) return a;
    if (b.v < a.v) return b;
    return {a.v, T(0.5) * (a.d + b.d)};
}
template <typename T>
__device__ __forceinline__ Dual<T> fmax(Dual<T> a, Dual<T> b)
{
    if (a.v > b.v) return a;
    if (b.v > a.v) return b;
    return {a.v, T(0.5) * (a.d + b.d)};
}
template <typename T>
__device__ __forceinline__ Dual<T> rcp(Dual<T> x)
{
    const T r = rcp(x.v);
    return {r, -x.d * r * r};
}
template <typename T>
__device__ __forceinline__ Dual<T> rsqrt(Dual<T> x)
{
    const T y = rsqrt(x.v);
    return {y, T(-0.5) * x.d * y * y * y};
}
template <typename T>
__device__ __forceinline__ Dual<T> sqrt_fast(Dual<T> x)
{
    const T y = rsqrt(x.v);
    return {sqrt_fast(x.v), T(0.5) * x.d * y};
}

template <typename T>
__device__ __forceinline__ Material<Dual<T>> dual_material(const Material<T>& m)
{
    Material<Dual<T>> r;
    r.gamma = m.gamma;
    r.pinf = m.pinf;
    r.gm1 = m.gm1;
    r.gpinf = m.gpinf;
    r.iG1 = m.iG1;
    r.PI1 = m.PI1;
    r.iG2 = m.iG2;
    r.PI2 = m.PI2;
    return r;
}

}  // namespace fv
