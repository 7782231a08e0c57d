// Forward-mode tangent numbers for the mode-Z adjoint: a value and N directional
// derivatives, propagated through every arithmetic operation by the chain rule.
// Running a small local map (a WENO-Z line, the full flux at one Gauss point) on
// Tan<N> with unit seeds gives N columns of its Jacobian exactly (to rounding);
// the adjoint kernel multiplies their transpose into the output cotangents.
// |x| takes the derivative sign(x) with sign(0) = +1, the one-sided choice of
// the branch x >= 0.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace hgks {

// the scalar functions stay visible beside the overloads below
using ::erf;
using ::exp;
using ::fabs;
using ::log;
using ::pow;
using ::sqrt;

template <int N>
struct Tan {
  double v;
  double d[N];
  __host__ __device__ __forceinline__ Tan() : v(0.0) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
  __host__ __device__ __forceinline__ Tan(double x) : v(x) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
  __host__ __device__ __forceinline__ Tan& operator+=(const Tan& o) {
    v += o.v;
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] += o.d[i];
    return *this;
  }
  __host__ __device__ __forceinline__ Tan& operator-=(const Tan& o) {
    v -= o.v;
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] -= o.d[i];
    return *this;
  }
};

// r = a x + b y on the tangents, value set by the caller
template <int N>
__host__ __device__ __forceinline__ Tan<N> tan_lin(double value, double a, const Tan<N>& x, double b, const Tan<N>& y) {
  Tan<N> r;
  r.v = value;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a * x.d[i] + b * y.d[i];
  return r;
}

// r = a x on the tangents, value set by the caller
template <int N>
__host__ __device__ __forceinline__ Tan<N> tan_scale(double value, double a, const Tan<N>& x) {
  Tan<N> r;
  r.v = value;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a * x.d[i];
  return r;
}

template <int N>
__host__ __device__ __forceinline__ Tan<N> operator+(const Tan<N>& a, const Tan<N>& b) {
  return tan_lin(a.v + b.v, 1.0, a, 1.0, b);
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator-(const Tan<N>& a, const Tan<N>& b) {
  return tan_lin(a.v - b.v, 1.0, a, -1.0, b);
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator-(const Tan<N>& a) {
  return tan_scale(-a.v, -1.0, a);
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator*(const Tan<N>& a, const Tan<N>& b) {
  return tan_lin(a.v * b.v, b.v, a, a.v, b);
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator/(const Tan<N>& a, const Tan<N>& b) {
  const double q = a.v / b.v;
  const double ib = 1.0 / b.v;
  // d(a/b) = (da - q db) / b
  return tan_lin(q, ib, a, -q * ib, b);
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator+(const Tan<N>& a, double b) {
  Tan<N> r = a;
  r.v += b;
  return r;
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator+(double a, const Tan<N>& b) {
  return b + a;
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator-(const Tan<N>& a, double b) {
  Tan<N> r = a;
  r.v -= b;
  return r;
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator-(double a, const Tan<N>& b) {
  return tan_scale(a - b.v, -1.0, b);
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator*(const Tan<N>& a, double b) {
  return tan_scale(a.v * b, b, a);
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator*(double a, const Tan<N>& b) {
  return tan_scale(a * b.v, a, b);
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator/(const Tan<N>& a, double b) {
  return tan_scale(a.v / b, 1.0 / b, a);
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> operator/(double a, const Tan<N>& b) {
  const double q = a / b.v;
  return tan_scale(q, -q / b.v, b);
}

template <int N>
__host__ __device__ __forceinline__ Tan<N> exp(const Tan<N>& a) {
  const double e = ::exp(a.v);
  return tan_scale(e, e, a);
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> sqrt(const Tan<N>& a) {
  const double s = ::sqrt(a.v);
  return tan_scale(s, 0.5 / s, a);
}
// d erf(x)/dx = 2/sqrt(pi) exp(-x^2)
template <int N>
__host__ __device__ __forceinline__ Tan<N> erf(const Tan<N>& a) {
  return tan_scale(::erf(a.v), 1.1283791670955125739 * ::exp(-a.v * a.v), a);
}
template <int N>
__host__ __device__ __forceinline__ Tan<N> fabs(const Tan<N>& a) {
  return a.v < 0.0 ? -a : a;
}
// a^b = exp(b log a) for a > 0
template <int N>
__host__ __device__ __forceinline__ Tan<N> pow(const Tan<N>& a, const Tan<N>& b) {
  const double y = ::pow(a.v, b.v);
  return tan_lin(y, b.v * y / a.v, a, y * ::log(a.v), b);
}

}  // namespace hgks
