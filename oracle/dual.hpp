// Forward-mode dual numbers for the oracle (test infrastructure only).
//
// A Dual carries a value and one directional derivative.  Running the oracle's
// scheme on Dual instead of double gives the exact Jacobian-vector product of a
// step (the derivative of every arithmetic operation is propagated by the chain
// rule), which is the reference the hand-written GPU adjoint is checked against.
#pragma once
#include <cmath>

namespace ref {

struct Dual {
  double v = 0.0;  // value
  double d = 0.0;  // derivative along the seeded direction
  Dual() = default;
  Dual(double value) : v(value), d(0.0) {}
  Dual(double value, double deriv) : v(value), d(deriv) {}
  Dual& operator+=(const Dual& o) { v += o.v; d += o.d; return *this; }
  Dual& operator-=(const Dual& o) { v -= o.v; d -= o.d; return *this; }
  Dual& operator*=(const Dual& o) { d = d * o.v + v * o.d; v *= o.v; return *this; }
  Dual& operator/=(const Dual& o) { *this = *this / o; return *this; }
  friend Dual operator+(Dual a, const Dual& b) { return a += b; }
  friend Dual operator-(Dual a, const Dual& b) { return a -= b; }
  friend Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
  friend Dual operator*(const Dual& a, const Dual& b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
  friend Dual operator/(const Dual& a, const Dual& b) {
    return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
  }
  friend bool operator<(const Dual& a, const Dual& b) { return a.v < b.v; }
  friend bool operator>(const Dual& a, const Dual& b) { return a.v > b.v; }
  friend bool operator<=(const Dual& a, const Dual& b) { return a.v <= b.v; }
  friend bool operator>=(const Dual& a, const Dual& b) { return a.v >= b.v; }
};

inline Dual exp(const Dual& a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
inline Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); return Dual(s, 0.5 * a.d / s); }
inline Dual erfc(const Dual& a) {
  // d/dx erfc(x) = -2/sqrt(pi) exp(-x^2)
  return Dual(std::erfc(a.v), -1.1283791670955126 * std::exp(-a.v * a.v) * a.d);
}
inline Dual pow(const Dual& a, double p) {
  double y = std::pow(a.v, p);
  return Dual(y, p * std::pow(a.v, p - 1.0) * a.d);
}
inline Dual fabs(const Dual& a) { return a.v < 0.0 ? -a : a; }
inline double value(const Dual& a) { return a.v; }
inline double value(double a) { return a; }

}  // namespace ref
