// Device math of the WENO-Z / full-flux mode (mode Z) of the HGKS stage update:
// nonlinear fifth-order reconstruction with Z-type weights and the complete
// second-order gas distribution of Eq. (flux), integrated in time (Sec. 2.1).
// Host-and-device templates on the arithmetic type T (double for the FP64
// path, float for the FP32-flux form).
#pragma once

#include "device_common.hpp"

namespace hgks {

// ---------------------------------------------------------------------------
// WENO-Z on five cell averages v[0..4] (cell 2 in the middle).
//
// Sub-stencils of three cells with the Jiang-Shu smoothness indicators
//   b0 = 13/12 (v0 - 2 v1 + v2)^2 + 1/4 (v0 - 4 v1 + 3 v2)^2
//   b1 = 13/12 (v1 - 2 v2 + v3)^2 + 1/4 (v1 - v3)^2
//   b2 = 13/12 (v2 - 2 v3 + v4)^2 + 1/4 (3 v2 - 4 v3 + v4)^2
// and the Z weights alpha_k = d_k (1 + (tau5 / (b_k + eps))^p), tau5 = |b0 - b2|,
// optimal weights d = (1/10, 6/10, 3/10) towards the edge being reconstructed.
// The sub-stencil values at the right edge of cell 2 are
//   (2 v0 - 7 v1 + 11 v2)/6, (-v1 + 5 v2 + 2 v3)/6, (2 v2 + 5 v3 - v4)/6,
// and their derivatives there (per unit cell width) v0 - 3 v1 + 2 v2, v3 - v2,
// v3 - v2.  The left edge is the same construction on the reversed line, whose
// indicators are (b2, b1, b0): both edges share one set of ratios.
// ---------------------------------------------------------------------------
template <typename T>
__host__ __device__ __forceinline__ T zratio(T tau5, T b, T eps, int p) {
  T r = tau5 * recip(b + eps);
  if (p == 2) return r * r;  // the usual exponent, without a loop
  T out = r;
  for (int i = 1; i < p; ++i) out = out * r;
  return out;
}

// The three ratios (tau5 / (b_k + eps))^p.  In double one division serves all
// three (1/d0 = d1 d2 / (d0 d1 d2) and so on; the product stays far inside the
// FP64 range for any b); in float each keeps its own division, because the
// product of three denominators could leave the FP32 range on a steep line.
template <typename T>
__host__ __device__ __forceinline__ void zratios(T tau5, T b0, T b1, T b2, T eps, int p, T& r0, T& r1, T& r2) {
  if constexpr (sizeof(T) == sizeof(float)) {
    r0 = zratio(tau5, b0, eps, p);
    r1 = zratio(tau5, b1, eps, p);
    r2 = zratio(tau5, b2, eps, p);
  } else {
    const T d0 = b0 + eps, d1 = b1 + eps, d2 = b2 + eps;
    const T d01 = d0 * d1;
    const T t = tau5 * recip(d01 * d2);
    const T x0 = t * (d1 * d2), x1 = t * (d0 * d2), x2 = t * d01;
    if (p == 2) {  // the usual exponent, without a loop
      r0 = x0 * x0;
      r1 = x1 * x1;
      r2 = x2 * x2;
      return;
    }
    r0 = x0;
    r1 = x1;
    r2 = x2;
    for (int i = 1; i < p; ++i) {
      r0 = r0 * x0;
      r1 = r1 * x1;
      r2 = r2 * x2;
    }
  }
}

template <typename T>
__host__ __device__ __forceinline__ void zbeta(const T* v, T& b0, T& b1, T& b2) {
  const T c13 = T(13.0 / 12.0);
  T s0 = v[0] - T(2) * v[1] + v[2], t0 = v[0] - T(4) * v[1] + T(3) * v[2];
  T s1 = v[1] - T(2) * v[2] + v[3], t1 = v[1] - v[3];
  T s2 = v[2] - T(2) * v[3] + v[4], t2 = T(3) * v[2] - T(4) * v[3] + v[4];
  b0 = c13 * s0 * s0 + T(0.25) * t0 * t0;
  b1 = c13 * s1 * s1 + T(0.25) * t1 * t1;
  b2 = c13 * s2 * s2 + T(0.25) * t2 * t2;
}

// Value and slope (per unit width) at the right edge of the middle cell.
template <typename T>
__host__ __device__ __forceinline__ void weno_z_right(const T* v, T eps, int p, T& val, T& slope) {
  T b0, b1, b2;
  zbeta(v, b0, b1, b2);
  T tau5 = fabs(b0 - b2);
  T r0, r1, r2;
  zratios(tau5, b0, b1, b2, eps, p, r0, r1, r2);
  T a0 = T(0.1) * (T(1) + r0);
  T a1 = T(0.6) * (T(1) + r1);
  T a2 = T(0.3) * (T(1) + r2);
  const T isum = recip(a0 + a1 + a2);
  T w0 = a0 * isum, w1 = a1 * isum, w2 = a2 * isum;
  T q0 = T(1.0 / 3.0) * v[0] - T(7.0 / 6.0) * v[1] + T(11.0 / 6.0) * v[2];
  T q1 = T(-1.0 / 6.0) * v[1] + T(5.0 / 6.0) * v[2] + T(1.0 / 3.0) * v[3];
  T q2 = T(1.0 / 3.0) * v[2] + T(5.0 / 6.0) * v[3] - T(1.0 / 6.0) * v[4];
  val = w0 * q0 + w1 * q1 + w2 * q2;
  T d0 = v[0] - T(3) * v[1] + T(2) * v[2];
  T d1 = v[3] - v[2];
  slope = w0 * d0 + w1 * d1 + w2 * d1;
}

// Both edge values of the middle cell: ea at its left edge, eb at its right edge.
template <typename T>
__host__ __device__ __forceinline__ void weno_z_edges(const T* v, T eps, int p, T& ea, T& eb) {
  T b0, b1, b2;
  zbeta(v, b0, b1, b2);
  T tau5 = fabs(b0 - b2);
  T r0, r1, r2;
  zratios(tau5, b0, b1, b2, eps, p, r0, r1, r2);
  // right edge with weights (0.1, 0.6, 0.3) on (r0, r1, r2); the reversed line
  // (v4, v3, v2, v1, v0) has indicators (b2, b1, b0), so its weights take (r2, r1, r0)
  const T ab0 = T(0.1) * (T(1) + r0), ab1 = T(0.6) * (T(1) + r1), ab2 = T(0.3) * (T(1) + r2);
  const T aa0 = T(0.1) * (T(1) + r2), aa1 = T(0.6) * (T(1) + r1), aa2 = T(0.3) * (T(1) + r0);
  const T sb = ab0 + ab1 + ab2, sa = aa0 + aa1 + aa2;
  T isb, isa;
  if constexpr (sizeof(T) == sizeof(double)) {
    // one reciprocal for both sums (each lies in [1, 1 + max r], so the product
    // stays far inside the FP64 range)
    const T ip = recip(sa * sb);
    isb = sa * ip;
    isa = sb * ip;
  } else {
    isb = recip(sb);
    isa = recip(sa);
  }
  {
    T q0 = T(1.0 / 3.0) * v[0] - T(7.0 / 6.0) * v[1] + T(11.0 / 6.0) * v[2];
    T q1 = T(-1.0 / 6.0) * v[1] + T(5.0 / 6.0) * v[2] + T(1.0 / 3.0) * v[3];
    T q2 = T(1.0 / 3.0) * v[2] + T(5.0 / 6.0) * v[3] - T(1.0 / 6.0) * v[4];
    eb = (ab0 * q0 + ab1 * q1 + ab2 * q2) * isb;
  }
  {
    T q0 = T(1.0 / 3.0) * v[4] - T(7.0 / 6.0) * v[3] + T(11.0 / 6.0) * v[2];
    T q1 = T(-1.0 / 6.0) * v[3] + T(5.0 / 6.0) * v[2] + T(1.0 / 3.0) * v[1];
    T q2 = T(1.0 / 3.0) * v[2] + T(5.0 / 6.0) * v[1] - T(1.0 / 6.0) * v[0];
    ea = (aa0 * q0 + aa1 * q1 + aa2 * q2) * isa;
  }
}

// Tangential reconstruction of mode Z inside the middle face: the parabola with
// the face average m and the WENO-Z edge values ea, eb, evaluated at the Gauss
// point s = sgn / (2 sqrt 3) (value) and differentiated there (per unit width):
//   value = m + sgn (eb - ea) / (2 sqrt 3),  slope = (eb - ea) + sgn sqrt 3 (ea + eb - 2 m).
constexpr double kGauss = 0.28867513459481288225;  // 1 / (2 sqrt 3)

template <typename T>
__host__ __device__ __forceinline__ T zpar_val(T m, T ea, T eb, T sgn) {
  return m + sgn * (eb - ea) * T(kGauss);
}
template <typename T>
__host__ __device__ __forceinline__ T zpar_der(T m, T ea, T eb, T sgn) {
  return (eb - ea) + sgn * T(kS3) * (ea + eb - T(2) * m);
}

// ---------------------------------------------------------------------------
// Full gas distribution at one Gauss point (Eq. (flux)) in the local frame.
//
// f = (1 - e^{-t/tau}) g0 + ((t + tau) e^{-t/tau} - tau) (a.u) g0 + (t - tau + tau e^{-t/tau}) A g0
//     + e^{-t/tau} [ -(tau + t)(a^l.u) g_l - tau A^l g_l ]_{u>0} + [same with r]_{u<0}
// (g_l carries the Heaviside factor of u > 0, g_r that of u < 0; the zeroth-order
// half-space parts e^{-t/tau} g_{l,r} are folded in through the coefficient of
// <psi>).  Each part's psi-moments factor into one-dimensional Gaussian moments
// of u, v, w and of the internal variable xi.  Time integrals over [0, delta]
// with e = exp(-delta/tau), om = 1 - e:
//   equilibrium side:   c_eq = delta - tau om,  c_a = 2 tau^2 om - tau delta (1 + e),
//                       c_A = delta^2/2 - tau delta + tau^2 om,
//   each initial side:  c_eq = tau om,  c_a = -2 tau^2 om + tau delta e,  c_A = -tau^2 om.
// F^n and dF^n/dt follow from the integrals over [0, dt] and [0, dt/2]
// (Eq. (expansion-1)):  F = (4 I(dt/2) - I(dt)) / dt,  dF = 4 (I(dt) - 2 I(dt/2)) / dt^2.
// The Prandtl-number correction adds (1/Pr - 1) times the normal heat flux, about
// the velocity of Q0, of the integrated distribution to the energy integral.
// ---------------------------------------------------------------------------
// Moments of one side.  The normalised Maxwellian factorises into Gaussians in u,
// v, w and the internal variable xi; the u-moments M[n] = <u^n> are full-space or
// half-space, the others full-space:
//   full-space recursion  M[n] = U M[n-1] + (n-1)/(2 lambda) M[n-2],  M[0] = 1, M[1] = U;
//   half space (sign +1: u > 0, -1: u < 0) the same recursion from
//   M[0] = 1/2 + sign erf(sqrt(lambda) U)/2,
//   M[1] = U M[0] + sign exp(-lambda U^2) / (2 sqrt(pi lambda)).
// Every quantity the flux needs is <u^p P psi_k> for a polynomial P of the
// velocity, psi = (1, u, v, w, (u^2 + s)/2) with s = v^2 + w^2 + xi^2.  Writing
// P = sum_n u^n C_n(v, w, s), with C_n over the basis
// (1, v, w, v^2, vw, w^2, s, vs, ws), gives
//   <u^p P psi_0> = sum_n M[n+p] E[C_n],      <u^p P psi_1> = sum_n M[n+p+1] E[C_n],
//   <u^p P psi_2> = sum_n M[n+p] E[v C_n],    <u^p P psi_3> = sum_n M[n+p] E[w C_n],
//   <u^p P psi_4> = (sum_n M[n+p+2] E[C_n] + M[n+p] E[s C_n]) / 2,
// where E is the expectation over (v, w, xi) alone:
//   E[v^b w^c]     = V_b W_c,
//   E[v^b w^c s]   = V_{b+2} W_c + V_b W_{c+2} + V_b W_c X_1,
//   E[v^b w^c s^2] = V_{b+4} W_c + V_b W_{c+4} + V_b W_c X_2
//                    + 2 (V_{b+2} W_{c+2} + V_{b+2} W_c X_1 + V_b W_{c+2} X_1),
// with V_b = <v^b>, W_c = <w^c> (Gaussian recursions) and X_1 = <xi^2> = K/(2 lambda),
// X_2 = <xi^4> = K (K+2)/(4 lambda^2).
template <typename T>
__host__ __device__ __forceinline__ void zmom_gauss(T* M, int n, T U, T i2l) {
  M[0] = T(1);
  M[1] = U;
  for (int k = 2; k < n; ++k) M[k] = U * M[k - 1] + T(k - 1) * i2l * M[k - 2];
}

template <typename T>
__host__ __device__ __forceinline__ void zmom_half(T* M, T U, T lam, T i2l, T sign) {
  const T kInvSqrtPi = T(0.56418958354775628695);
  T sl = sqrt(lam);
  T x = sl * U;
  M[0] = T(0.5) + sign * T(0.5) * erf(x);
  M[1] = U * M[0] + sign * T(0.5) * kInvSqrtPi * exp(-x * x) / sl;
  for (int k = 2; k < 7; ++k) M[k] = U * M[k - 1] + T(k - 1) * i2l * M[k - 2];
}

template <typename T>
struct ZGauss {
  T v[6], w[6], x1, x2;
  __host__ __device__ __forceinline__ T E(int b, int c, int m) const {
    if (m == 0) return v[b] * w[c];
    if (m == 1) return v[b + 2] * w[c] + v[b] * w[c + 2] + v[b] * w[c] * x1;
    return v[b + 4] * w[c] + v[b] * w[c + 4] + v[b] * w[c] * x2 +
           T(2) * (v[b + 2] * w[c + 2] + v[b + 2] * w[c] * x1 + v[b] * w[c + 2] * x1);
  }
};

// Exponents (b, c, m) of the basis (1, v, w, v^2, vw, w^2, s, vs, ws).
__host__ __device__ constexpr int zb_b(int i) { return (i == 1 || i == 4 || i == 7) ? 1 : (i == 3 ? 2 : 0); }
__host__ __device__ constexpr int zb_c(int i) { return (i == 2 || i == 4 || i == 8) ? 1 : (i == 5 ? 2 : 0); }
__host__ __device__ constexpr int zb_m(int i) { return i >= 6 ? 1 : 0; }

// E[C], E[v C], E[w C], E[s C] of C = sum over the basis terms present in MASK
// (bit i: basis term i) with coefficients c[i].
template <int MASK, typename T>
__host__ __device__ __forceinline__ void zexpect(const T* c, const ZGauss<T>& G, T* e) {
  bool first = true;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    if (!((MASK >> i) & 1)) continue;
    const int b = zb_b(i), cc = zb_c(i), m = zb_m(i);
    T t1 = c[i] * G.E(b, cc, m), tv = c[i] * G.E(b + 1, cc, m), tw = c[i] * G.E(b, cc + 1, m),
      ts = c[i] * G.E(b, cc, m + 1);
    if (first) {
      e[0] = t1; e[1] = tv; e[2] = tw; e[3] = ts;
      first = false;
    } else {
      e[0] = e[0] + t1; e[1] = e[1] + tv; e[2] = e[2] + tw; e[3] = e[3] + ts;
    }
  }
}

// <u^p P psi> for p = 0 (r0) and, when BOTH, p = 1 (r1), from the expectations
// e[n][4] of the u-power coefficients C_n, n < NC; e[n][1] and e[n][2] are taken
// as zero for n >= NVW.
template <int NC, bool BOTH, typename T, int NVW = NC>
__host__ __device__ __forceinline__ void zrows(const T* M, const T (*e)[4], T* r0, T* r1) {
#pragma unroll
  for (int p = 0; p < (BOTH ? 2 : 1); ++p) {
    T* r = p ? r1 : r0;
    r[0] = M[p] * e[0][0];
    r[1] = M[p + 1] * e[0][0];
    r[2] = NVW > 0 ? M[p] * e[0][1] : T(0);
    r[3] = NVW > 0 ? M[p] * e[0][2] : T(0);
    T e4 = M[p + 2] * e[0][0] + M[p] * e[0][3];
#pragma unroll
    for (int n = 1; n < NC; ++n) {
      r[0] = r[0] + M[n + p] * e[n][0];
      r[1] = r[1] + M[n + p + 1] * e[n][0];
      if (n < NVW) {
        r[2] = r[2] + M[n + p] * e[n][1];
        r[3] = r[3] + M[n + p] * e[n][2];
      }
      e4 = e4 + M[n + p + 2] * e[n][0] + M[n + p] * e[n][3];
    }
    r[4] = T(0.5) * e4;
  }
}

// Expectations of the slope polynomial a_n u + a_t1 v + a_t2 w ... in the form
// u (phi_n) + v (phi_t1) + w (phi_t2), phi_X = X0 + X1 u + X2 v + X3 w + X4 (u^2 + s)/2:
//   C_0 = t0 v + t2 v^2 + (t3 + r2) vw + t4/2 vs + r0 w + r3 w^2 + r4/2 ws
//   C_1 = n0 + (n2 + t1) v + (n3 + r1) w + n4/2 s
//   C_2 = n1 + t4/2 v + r4/2 w
//   C_3 = n4/2
// (n = a_n, t = a_t1, r = a_t2).
template <typename T>
__host__ __device__ __forceinline__ void zexpect_slopes(const T (*a)[5], const ZGauss<T>& G, T (*e)[4]) {
  const T* n = a[0];
  const T* t = a[1];
  const T* r = a[2];
  {
    T c[9] = {T(0), t[0], r[0], t[2], t[3] + r[2], r[3], T(0), T(0.5) * t[4], T(0.5) * r[4]};
    zexpect<0x1BE>(c, G, e[0]);
  }
  {
    T c[9] = {n[0], n[2] + t[1], n[3] + r[1], T(0), T(0), T(0), T(0.5) * n[4], T(0), T(0)};
    zexpect<0x047>(c, G, e[1]);
  }
  {
    T c[9] = {n[1], T(0.5) * t[4], T(0.5) * r[4], T(0), T(0), T(0), T(0), T(0), T(0)};
    zexpect<0x007>(c, G, e[2]);
  }
  {
    T c[9] = {T(0.5) * n[4], T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    zexpect<0x001>(c, G, e[3]);
  }
}

// Expectations of phi_A = A0 + A1 u + A2 v + A3 w + A4 (u^2 + s)/2:
//   C_0 = A0 + A2 v + A3 w + A4/2 s,  C_1 = A1,  C_2 = A4/2.
template <typename T>
__host__ __device__ __forceinline__ void zexpect_phi(const T* A, const ZGauss<T>& G, T (*e)[4]) {
  {
    T c[9] = {A[0], A[2], A[3], T(0), T(0), T(0), T(0.5) * A[4], T(0), T(0)};
    zexpect<0x047>(c, G, e[0]);
  }
  {
    T c[9] = {A[1], T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    zexpect<0x001>(c, G, e[1]);
  }
  {
    T c[9] = {T(0.5) * A[4], T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    zexpect<0x001>(c, G, e[2]);
  }
}

// Slope polynomial a with <a psi> = b for a Maxwellian (U, V, W, lambda): the
// 5 x 5 system of Gaussian moments solved in closed form.
// The Maxwellian's factors are shared by all solves with it (zslope_coef):
// Ep = (|U|^2 + (K+3)/(2 lambda))/2 and c4 = 8 lambda^2/(K+3).
template <typename T>
struct ZSlopeCoef {
  T Ep, c4, tl;  // tl = 2 lambda
};
template <typename T>
__host__ __device__ __forceinline__ ZSlopeCoef<T> zslope_coef(T U, T V, T W, T lam, T i2l, T K) {
  ZSlopeCoef<T> c;
  c.Ep = T(0.5) * (U * U + V * V + W * W + (K + T(3)) * i2l);
  c.c4 = T(8) * lam * lam / (K + T(3));
  c.tl = T(2) * lam;
  return c;
}
template <typename T>
__host__ __device__ __forceinline__ void zslope(const T* b, T U, T V, T W, const ZSlopeCoef<T>& c, T* a) {
  T B = b[1] - U * b[0], C = b[2] - V * b[0], D = b[3] - W * b[0];
  a[4] = c.c4 * (b[4] - c.Ep * b[0] - U * B - V * C - W * D);
  a[1] = c.tl * B - U * a[4];
  a[2] = c.tl * C - V * a[4];
  a[3] = c.tl * D - W * a[4];
  a[0] = b[0] - U * a[1] - V * a[2] - W * a[3] - c.Ep * a[4];
}

// Primitive variables of a local-frame deviation state.
template <typename T>
struct ZPrim {
  T rho, U, V, W, p, lam;
};
template <typename T>
__host__ __device__ __forceinline__ ZPrim<T> zprim(const Geo& g, const T* dQ) {
  ZPrim<T> s;
  s.rho = T(g.rho_ref) + dQ[0];
  T ir = T(1) / s.rho;
  s.U = dQ[1] * ir;
  s.V = dQ[2] * ir;
  s.W = dQ[3] * ir;
  s.p = T(g.p_ref) + T(g.gm1) * (dQ[4] - T(0.5) * s.rho * (s.U * s.U + s.V * s.V + s.W * s.W));
  s.lam = T(0.5) * s.rho / s.p;
  return s;
}

// Time-integral coefficients over [0, delta]: eq[0..2] for the equilibrium side,
// in[0..2] for the two initial sides; e = exp(-delta/tau) given (ztime_e) or
// computed (ztime).
template <typename T>
__host__ __device__ __forceinline__ void ztime_e(T delta, T tau, T e, T* eq, T* in) {
  T om = T(1) - e;
  eq[0] = delta - tau * om;
  eq[1] = T(2) * tau * tau * om - tau * delta * (T(1) + e);
  eq[2] = T(0.5) * delta * delta - tau * delta + tau * tau * om;
  in[0] = tau * om;
  in[1] = T(-2) * tau * tau * om + tau * delta * e;
  in[2] = -tau * tau * om;
}
template <typename T>
__host__ __device__ __forceinline__ void ztime(T delta, T tau, T* eq, T* in) {
  ztime_e(delta, tau, T(exp(-delta / tau)), eq, in);
}

// Accumulated time integrals: I = flux moments (<u ...>), J = density moments,
// for delta = dt (suffix 1) and delta = dt/2 (suffix h).
template <typename T>
struct ZAcc {
  T I1[5], J1[5], Ih[5], Jh[5];
};

// The moment rows of one side, without rho and the time coefficients: r[0..2]
// = phi 1, a.u, A for p = 0 (density moments J), r[3..5] the same for p = 1 (flux
// moments I).
template <typename T>
__host__ __device__ __forceinline__ void zside_rows(const ZPrim<T>& s, const T (*D)[5], int half, T K, T (*r)[5]) {
  const T i2l = T(0.5) / s.lam;
  ZGauss<T> G;
  zmom_gauss(G.v, 6, s.V, i2l);
  zmom_gauss(G.w, 6, s.W, i2l);
  G.x1 = K * i2l;
  G.x2 = K * (K + T(2)) * i2l * i2l;
  T M[7];
  zmom_gauss(M, 7, s.U, i2l);
  T a[3][5];
  const ZSlopeCoef<T> sc = zslope_coef(s.U, s.V, s.W, s.lam, i2l, K);
  const T ir = T(1) / s.rho;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T b[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = D[d][k] * ir;
    zslope(b, s.U, s.V, s.W, sc, a[d]);
  }
  T ea[4][4];
  zexpect_slopes(a, G, ea);
  T ra0[5], ra1[5];
  zrows<4, false>(M, ea, ra0, ra1);  // <(a.u) psi>, full space
  T A[5];
  {
    T bt[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) bt[k] = -ra0[k];
    zslope(bt, s.U, s.V, s.W, sc, A);
  }
  if (half != 0) {
    zmom_half(M, s.U, s.lam, i2l, T(half));
    zrows<4, true>(M, ea, ra0, ra1);
  } else {
    zrows<4, true>(M, ea, ra0, ra1);
  }
  T eA[3][4];
  zexpect_phi(A, G, eA);
  T rA0[5], rA1[5];
  zrows<3, true>(M, eA, rA0, rA1);
  // phi = 1: C_0 = 1
  T r10[5], r11[5];
  {
    T e1[1][4] = {{T(1), s.V, s.W, G.E(0, 0, 1)}};
    zrows<1, true>(M, e1, r10, r11);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    r[0][k] = r10[k];
    r[1][k] = ra0[k];
    r[2][k] = rA0[k];
    r[3][k] = r11[k];
    r[4][k] = ra1[k];
    r[5][k] = rA1[k];
  }
}

// One side of the distribution: its Maxwellian (s), its spatial slopes D[3][5]
// (local frame, along n, t1, t2), half = 0 (equilibrium, full space), +1 or -1.
// Adds rho (c0 <u^p psi> + c1 <u^p (a.u) psi> + c2 <u^p A psi>) for p = 1 (I)
// and p = 0 (J) with the coefficient sets k1 (delta = dt) and kh (dt/2); the
// time slope A solves <a.u + A> = 0 over the side's full-space Maxwellian.
template <typename T>
__host__ __device__ __forceinline__ void zside(const ZPrim<T>& s, const T (*D)[5], int half, T K, const T* k1,
                                               const T* kh, ZAcc<T>& acc, bool first) {
  T r[6][5];
  zside_rows(s, D, half, K, r);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    T j1 = s.rho * (k1[0] * r[0][k] + k1[1] * r[1][k] + k1[2] * r[2][k]);
    T jh = s.rho * (kh[0] * r[0][k] + kh[1] * r[1][k] + kh[2] * r[2][k]);
    T i1 = s.rho * (k1[0] * r[3][k] + k1[1] * r[4][k] + k1[2] * r[5][k]);
    T ih = s.rho * (kh[0] * r[3][k] + kh[1] * r[4][k] + kh[2] * r[5][k]);
    acc.J1[k] = first ? j1 : acc.J1[k] + j1;
    acc.Jh[k] = first ? jh : acc.Jh[k] + jh;
    acc.I1[k] = first ? i1 : acc.I1[k] + i1;
    acc.Ih[k] = first ? ih : acc.Ih[k] + ih;
  }
}

// Normal heat flux of a perturbation with flux moments G1 and density moments G0
// about the velocity (U, V, W):  h(G1) - U h(G0),
// h(G) = G4 - (U G1 + V G2 + W G3) + |U|^2 G0 / 2.
template <typename T>
__host__ __device__ __forceinline__ T zheat(const T* G1, const T* G0, T U, T V, T W) {
  T k = T(0.5) * (U * U + V * V + W * W);
  T h1 = G1[4] - (U * G1[1] + V * G1[2] + W * G1[3]) + k * G1[0];
  T h0 = G0[4] - (U * G0[1] + V * G0[2] + W * G0[3]) + k * G0[0];
  return h1 - U * h0;
}

// Full flux at one Gauss point, in three parts so that a kernel can reconstruct
// each side's slopes just before they are used.
//   zflux_begin: primitive states, collision time
//     tau = mu(T0)/p0 + c_art |p_l - p_r| / (p_l + p_r) dt  (Sec. 3)
//     and the time-integral coefficients for dt and dt/2;
//   zside (above) for the equilibrium side and the two initial sides;
//   zflux_end: Prandtl-number correction and F^n, dF^n/dt.
// Inputs (local frame): deviations of Q0, Q_l, Q_r from the reference state and
// their derivatives along (n, t1, t2); dt is the step.  F gets F^n without the
// constant p_ref in its normal-momentum component, dF gets dF^n/dt.
template <typename T>
struct ZCoef {
  ZPrim<T> s0, sl, sr;
  T eq1[3], in1[3], eqh[3], inh[3];
};

template <bool VAR_MU, typename T>
__host__ __device__ __forceinline__ void zflux_begin(const Geo& g, const T* dQ0, const T* dQl, const T* dQr, T dt,
                                                     ZCoef<T>& c) {
  c.s0 = zprim(g, dQ0);
  c.sl = zprim(g, dQl);
  c.sr = zprim(g, dQr);
  T T0 = c.s0.p / c.s0.rho;
  T mu = T(g.mu_ref);
  if (VAR_MU) mu = mu * pow(T0 / T(g.T_ref), T(g.mu_exp));
  T tau = mu / c.s0.p + T(g.c_art) * fabs((c.sl.p - c.sr.p) / (c.sl.p + c.sr.p)) * dt;
  ztime(dt, tau, c.eq1, c.in1);
  ztime(T(0.5) * dt, tau, c.eqh, c.inh);
}

template <typename T>
__host__ __device__ __forceinline__ void zflux_end(const Geo& g, const ZCoef<T>& c, ZAcc<T>& acc, T dt, T* F, T* dF) {
  const T fix = T(g.pr_fix);
  acc.I1[4] = acc.I1[4] + fix * zheat(acc.I1, acc.J1, c.s0.U, c.s0.V, c.s0.W);
  acc.Ih[4] = acc.Ih[4] + fix * zheat(acc.Ih, acc.Jh, c.s0.U, c.s0.V, c.s0.W);
  const T idt = T(1) / dt;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    F[k] = (T(4) * acc.Ih[k] - acc.I1[k]) * idt;
    dF[k] = T(4) * (acc.I1[k] - T(2) * acc.Ih[k]) * idt * idt;
  }
  F[1] = F[1] - T(g.p_ref);
}

// ---------------------------------------------------------------------------
// The same flux with each part folded into F^n and dF^n/dt as soon as its
// moments are formed (the forward kernels).  F = (4 I(dt/2) - I(dt))/dt and
// dF = 4 (I(dt) - 2 I(dt/2))/dt^2 are linear in the time integrals, and so is the
// Prandtl correction's heat flux (zheat), so every part c_j rho <u^p P_j psi>
// goes straight into
//   F  += rho kF_j <u P_j psi>,   kF_j = (4 c_j(dt/2) - c_j(dt)) / dt,
//   dF += rho kD_j <u P_j psi>,   kD_j = 4 (c_j(dt) - 2 c_j(dt/2)) / dt^2,
// with its heat flux about U0 summed in qF, qD.  Neither the four integrals
// I, J over dt and dt/2 nor a side's six moment rows are held at once.
// ---------------------------------------------------------------------------
template <typename T>
struct ZOut {
  T F[5], D[5], qF, qD;
};

// E[C], E[v C], E[w C], E[s C] over the zero-mean Gaussian in (v, w, xi) with
// variance s2 per component, for C = c0 + cv v + cw w + cvv v^2 + cvw vw + cww w^2
// + cs s + cvs v s + cws w s and s = v^2 + w^2 + xi^2 of Nd = K + 2 components:
// E[v^2] = s2, E[s] = Nd s2, E[v^2 s] = (Nd + 2) s2^2, E[s^2] = Nd (Nd + 2) s2^2, and
// every moment odd in v or w is zero (so cvw never contributes).  The caller
// passes cq = cvv + cww + Nd cs, Ns2 = Nd s2 and N2s2 = (Nd + 2) s2.
template <typename T>
__host__ __device__ __forceinline__ void zexp0(T c0, T cv, T cw, T cq, T cvs, T cws, T s2, T Ns2, T N2s2, T* e) {
  const T q = s2 * cq;
  e[0] = c0 + q;
  e[1] = s2 * (cv + N2s2 * cvs);
  e[2] = s2 * (cw + N2s2 * cws);
  e[3] = Ns2 * c0 + N2s2 * q;
}

// kF, kD of the equilibrium side (eq = true) or of an initial side, from the
// collision time; the exponentials come from the caller (e1 = exp(-dt/tau),
// eh = exp(-dt/(2 tau))).
template <typename T>
__host__ __device__ __forceinline__ void zfd_coef(T dt, T tau, T e1, T eh, bool eq, T* kF, T* kD) {
  T k1[3], kh[3], unused[3];
  if (eq) {
    ztime_e(dt, tau, e1, k1, unused);
    ztime_e(T(0.5) * dt, tau, eh, kh, unused);
  } else {
    ztime_e(dt, tau, e1, unused, k1);
    ztime_e(T(0.5) * dt, tau, eh, unused, kh);
  }
  const T idt = T(1) / dt;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    kF[j] = (T(4) * kh[j] - k1[j]) * idt;
    kD[j] = T(4) * (k1[j] - T(2) * kh[j]) * idt * idt;
  }
}

// One part of one side: moment rows r0 (p = 0) and r1 (p = 1) with weights
// wF = rho kF_j, wD = rho kD_j.
template <typename T>
__host__ __device__ __forceinline__ void zfold(T wF, T wD, const T* r0, const T* r1, T U0, T V0, T W0, ZOut<T>& o,
                                               bool first) {
  const T h = zheat(r1, r0, U0, V0, W0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    o.F[k] = first ? wF * r1[k] : o.F[k] + wF * r1[k];
    o.D[k] = first ? wD * r1[k] : o.D[k] + wD * r1[k];
  }
  o.qF = first ? wF * h : o.qF + wF * h;
  o.qD = first ? wD * h : o.qD + wD * h;
}

// One side (as zside), folded into o; (U0, V0, W0) is the velocity of Q0.
// The side is evaluated in its own tangential rest frame, v' = v - V, w' = w - W,
// with psi' = (1, u, v', w', (u^2 + v'^2 + w'^2 + xi^2)/2); then psi = L psi' with
//   psi_2 = psi'_2 + V psi'_0,  psi_3 = psi'_3 + W psi'_0,
//   psi_4 = psi'_4 + V psi'_2 + W psi'_3 + (V^2 + W^2)/2 psi'_0,
// so moment vectors map back by L, moment data into the frame by L^-1, and a
// polynomial a.psi has coefficients a' = L^T a there.  Over the zero-mean Gaussian
// in (v', w', xi) every odd moment vanishes and the rest are closed forms in
// s2 = 1/(2 lambda) (zexp0): the expectations shrink to a few terms per u-power.
// The particle velocity of the slope term is (u, v' + V, w' + W), so the
// tangential slopes add V phi_t1 + W phi_t2 to the u^0 coefficient.
template <typename T>
__host__ __device__ __forceinline__ void zside_fold(const ZPrim<T>& s, const T (*D)[5], int half, T K, const T* kF,
                                                    const T* kD, T U0, T V0, T W0, ZOut<T>& o, bool first) {
  const T i2l = T(0.5) / s.lam;
  const T Nd = K + T(2);  // components of s' = v'^2 + w'^2 + xi^2
  const T Ns2 = Nd * i2l, N2s2 = (Nd + T(2)) * i2l;
  T M[7];
  zmom_gauss(M, 7, s.U, i2l);
  const T V = s.V, W = s.W, kVW = T(0.5) * (V * V + W * W);
  // slope solve in the rest frame: <a' psi'> = b' with b' = L^-1 b (zslope at V = W = 0)
  const T Ep = T(0.5) * (s.U * s.U + (K + T(3)) * i2l), c4 = T(8) * s.lam * s.lam / (K + T(3)), tl = T(2) * s.lam;
  auto solve = [&](const T* b, T* a) {
    const T b2 = b[2] - V * b[0], b3 = b[3] - W * b[0];
    const T b4 = b[4] - V * b2 - W * b3 - kVW * b[0];
    const T B = b[1] - s.U * b[0];
    a[4] = c4 * (b4 - Ep * b[0] - s.U * B);
    a[1] = tl * B - s.U * a[4];
    a[2] = tl * b2;
    a[3] = tl * b3;
    a[0] = b[0] - s.U * a[1] - Ep * a[4];
  };
  T ea[4][4];
  {
    T a[3][5];
    const T ir = T(1) / s.rho;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T b[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) b[k] = D[d][k] * ir;
      solve(b, a[d]);
    }
    const T* n = a[0];
    const T* t = a[1];
    const T* r = a[2];
    T X[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) X[k] = V * t[k] + W * r[k];
    zexp0(X[0], t[0] + X[2], r[0] + X[3], t[2] + r[3] + Nd * T(0.5) * X[4], T(0.5) * t[4], T(0.5) * r[4], i2l, Ns2,
          N2s2, ea[0]);
    {
      const T c0 = n[0] + X[1], q = i2l * (Nd * T(0.5) * n[4]);
      ea[1][0] = c0 + q;
      ea[1][1] = i2l * (n[2] + t[1]);
      ea[1][2] = i2l * (n[3] + r[1]);
      ea[1][3] = Ns2 * c0 + N2s2 * q;
    }
    ea[2][0] = n[1] + T(0.5) * X[4];
    ea[2][1] = i2l * T(0.5) * t[4];
    ea[2][2] = i2l * T(0.5) * r[4];
    ea[2][3] = Ns2 * ea[2][0];
    ea[3][0] = T(0.5) * n[4];
    ea[3][1] = T(0);
    ea[3][2] = T(0);
    ea[3][3] = Ns2 * ea[3][0];
  }
  // time slope: <(a.u + A) psi> = 0 over the full-space Maxwellian, solved in the
  // rest frame from the rows there (b' = -ra' directly)
  T A[5];
  {
    T ra[5], unused[5];
    zrows<4, false, T, 3>(M, ea, ra, unused);
    const T B = -ra[1] + s.U * ra[0];
    A[4] = c4 * (-ra[4] + Ep * ra[0] - s.U * B);
    A[1] = tl * B - s.U * A[4];
    A[2] = -tl * ra[2];
    A[3] = -tl * ra[3];
    A[0] = -ra[0] - s.U * A[1] - Ep * A[4];
  }
  if (half != 0) zmom_half(M, s.U, s.lam, i2l, T(half));
  // heat flux about U0 in the rest frame: relative tangential velocity of Q0
  const T dV = V0 - V, dW = W0 - W;
  auto fold = [&](T wF, T wD, T* r0, T* r1, bool f) {
    const T h = zheat(r1, r0, U0, dV, dW);
    r1[4] = r1[4] + V * r1[2] + W * r1[3] + kVW * r1[0];
    r1[2] = r1[2] + V * r1[0];
    r1[3] = r1[3] + W * r1[0];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      o.F[k] = f ? wF * r1[k] : o.F[k] + wF * r1[k];
      o.D[k] = f ? wD * r1[k] : o.D[k] + wD * r1[k];
    }
    o.qF = f ? wF * h : o.qF + wF * h;
    o.qD = f ? wD * h : o.qD + wD * h;
  };
  {
    T r0[5], r1[5];
    zrows<4, true, T, 3>(M, ea, r0, r1);  // a.u
    fold(s.rho * kF[1], s.rho * kD[1], r0, r1, first);
  }
  {
    T eA[3][4], r0[5], r1[5];
    {
      const T q = i2l * (Nd * T(0.5) * A[4]);
      eA[0][0] = A[0] + q;
      eA[0][1] = i2l * A[2];
      eA[0][2] = i2l * A[3];
      eA[0][3] = Ns2 * A[0] + N2s2 * q;
    }
    eA[1][0] = A[1];
    eA[1][1] = T(0);
    eA[1][2] = T(0);
    eA[1][3] = Ns2 * A[1];
    eA[2][0] = T(0.5) * A[4];
    eA[2][1] = T(0);
    eA[2][2] = T(0);
    eA[2][3] = Ns2 * eA[2][0];
    zrows<3, true, T, 1>(M, eA, r0, r1);  // A
    fold(s.rho * kF[2], s.rho * kD[2], r0, r1, false);
  }
  {
    T e1[1][4] = {{T(1), T(0), T(0), Ns2}};
    T r0[5], r1[5];
    zrows<1, true, T, 0>(M, e1, r0, r1);  // phi = 1
    fold(s.rho * kF[0], s.rho * kD[0], r0, r1, false);
  }
}

// F^n (without p_ref in its normal-momentum component) and dF^n/dt from o.
template <typename T>
__host__ __device__ __forceinline__ void zfold_end(const Geo& g, const ZOut<T>& o, T* F, T* dF) {
  const T fix = T(g.pr_fix);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    F[k] = o.F[k];
    dF[k] = o.D[k];
  }
  F[4] = F[4] + fix * o.qF;
  dF[4] = dF[4] + fix * o.qD;
  F[1] = F[1] - T(g.p_ref);
}

// States and collision time of zflux_begin for the folded form.
template <typename T>
struct ZFold {
  ZPrim<T> s0, sl, sr;
  T tau, e1, eh;
};

template <bool VAR_MU, typename T>
__host__ __device__ __forceinline__ void zfold_begin(const Geo& g, const T* dQ0, const T* dQl, const T* dQr, T dt,
                                                     ZFold<T>& c) {
  c.s0 = zprim(g, dQ0);
  c.sl = zprim(g, dQl);
  c.sr = zprim(g, dQr);
  T T0 = c.s0.p / c.s0.rho;
  T mu = T(g.mu_ref);
  if (VAR_MU) mu = mu * pow(T0 / T(g.T_ref), T(g.mu_exp));
  c.tau = mu / c.s0.p + T(g.c_art) * fabs((c.sl.p - c.sr.p) / (c.sl.p + c.sr.p)) * dt;
  c.e1 = exp(-dt / c.tau);
  c.eh = exp(-(T(0.5) * dt) / c.tau);
}

// side 0: equilibrium, 1: left initial state (u > 0), 2: right (u < 0)
template <typename T>
__host__ __device__ __forceinline__ void zfold_side(const ZFold<T>& c, int side, const T (*D)[5], T K, T dt,
                                                    ZOut<T>& o) {
  T kF[3], kD[3];
  zfd_coef(dt, c.tau, c.e1, c.eh, side == 0, kF, kD);
  const ZPrim<T>& s = side == 0 ? c.s0 : (side == 1 ? c.sl : c.sr);
  zside_fold(s, D, side == 0 ? 0 : (side == 1 ? +1 : -1), K, kF, kD, c.s0.U, c.s0.V, c.s0.W, o, side == 0);
}

// Full flux with a given collision time, in the folded form of the forward
// kernels (host checks of the device math).
template <typename T>
__host__ __device__ __forceinline__ void full_flux_tau(const Geo& g, const T* dQ0, const T (*D0)[5], const T* dQl,
                                                       const T (*Dl)[5], const T* dQr, const T (*Dr)[5], T tau, T dt,
                                                       T* F, T* dF) {
  const T K = T(g.K);
  ZFold<T> c;
  c.s0 = zprim(g, dQ0);
  c.sl = zprim(g, dQl);
  c.sr = zprim(g, dQr);
  c.tau = tau;
  c.e1 = exp(-dt / tau);
  c.eh = exp(-(T(0.5) * dt) / tau);
  ZOut<T> o;
  zfold_side(c, 0, D0, K, dt, o);
  zdep(c.sl.rho, o.F[4]);
  zfold_side(c, 1, Dl, K, dt, o);
  zdep(c.sr.rho, o.F[4]);
  zfold_side(c, 2, Dr, K, dt, o);
  zfold_end(g, o, F, dF);
}

}  // namespace hgks
