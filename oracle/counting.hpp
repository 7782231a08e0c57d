// Operation-counting scalar for the oracle (test infrastructure only).
//
// A Counted carries a double and, for every arithmetic operation it takes part
// in, increments one counter of its kind: +, -, x, /, sqrt, exp, erfc, pow.  The
// scheme run on Counted instead of double yields the operation counts of the
// algorithm as the oracle writes it (Sec. 2, in the paper's order), which is the
// per-unit algorithmic work the measurement section asks to be recorded.  Unary
// minus, |x|, comparisons and conversions are not counted.  The counters are
// shared by all threads (relaxed atomics).
#pragma once
#include <atomic>
#include <cmath>

namespace ref {

enum CountKind { kCntAdd = 0, kCntSub, kCntMul, kCntDiv, kCntSqrt, kCntExp, kCntErfc, kCntPow, kCntKinds };

inline std::atomic<long long>* op_counters() {
  static std::atomic<long long> c[kCntKinds];
  return c;
}
inline void count_op(CountKind k) { op_counters()[k].fetch_add(1, std::memory_order_relaxed); }
inline void reset_counts() {
  for (int k = 0; k < kCntKinds; ++k) op_counters()[k].store(0);
}

struct Counted {
  double v = 0.0;
  Counted() = default;
  Counted(double value) : v(value) {}
  Counted& operator+=(const Counted& o) { count_op(kCntAdd); v += o.v; return *this; }
  Counted& operator-=(const Counted& o) { count_op(kCntSub); v -= o.v; return *this; }
  Counted& operator*=(const Counted& o) { count_op(kCntMul); v *= o.v; return *this; }
  Counted& operator/=(const Counted& o) { count_op(kCntDiv); v /= o.v; return *this; }
  friend Counted operator+(Counted a, const Counted& b) { return a += b; }
  friend Counted operator-(Counted a, const Counted& b) { return a -= b; }
  friend Counted operator*(Counted a, const Counted& b) { return a *= b; }
  friend Counted operator/(Counted a, const Counted& b) { return a /= b; }
  friend Counted operator-(const Counted& a) { return Counted(-a.v); }
  friend bool operator<(const Counted& a, const Counted& b) { return a.v < b.v; }
  friend bool operator>(const Counted& a, const Counted& b) { return a.v > b.v; }
  friend bool operator<=(const Counted& a, const Counted& b) { return a.v <= b.v; }
  friend bool operator>=(const Counted& a, const Counted& b) { return a.v >= b.v; }
};

inline Counted exp(const Counted& a) { count_op(kCntExp); return Counted(std::exp(a.v)); }
inline Counted sqrt(const Counted& a) { count_op(kCntSqrt); return Counted(std::sqrt(a.v)); }
inline Counted erfc(const Counted& a) { count_op(kCntErfc); return Counted(std::erfc(a.v)); }
inline Counted pow(const Counted& a, double p) { count_op(kCntPow); return Counted(std::pow(a.v, p)); }
inline Counted fabs(const Counted& a) { return Counted(std::fabs(a.v)); }
inline double value(const Counted& a) { return a.v; }

}  // namespace ref
