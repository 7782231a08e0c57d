// Building blocks of the mode-Z adjoint: the full flux at one Gauss point as a
// function of its 60 reconstructed inputs, the transpose of its Jacobian applied
// to a cotangent (by the hand-written reverse of zreverse.hpp; the columns by
// forward tangents are kept as the host tests' reference), and the Jacobians of
// the WENO-Z edge pair and of the right-edge value and slope of a five-value
// line.  Host-and-device, so the CPU tests can check them against central
// differences.
#pragma once

#include "tangent.hpp"
#include "zflux.hpp"
#include "zreverse.hpp"

namespace hgks {

// Tangent columns per pass through the Gauss-point flux.
#ifndef HGKS_ZTAN
#define HGKS_ZTAN 1
#endif
constexpr int kZTan = HGKS_ZTAN;
static_assert(15 % kZTan == 0, "the passes cover the 15 value inputs");
// Inputs of the Gauss-point flux, local frame: Q0, Q_l, Q_r (values), then the
// derivatives D0, D_l, D_r, each [3][5] along (n, t1, t2).
constexpr int kXQ0 = 0, kXQl = 5, kXQr = 10, kXD0 = 15, kXDl = 30, kXDr = 45, kXN = 60;

template <bool VAR_MU, typename T>
__host__ __device__ __forceinline__ void zgp_flux(const Geo& g, const T* X, T dt, T* F, T* dF) {
  const T K = T(g.K);
  ZCoef<T> c;
  zflux_begin<VAR_MU>(g, X + kXQ0, X + kXQl, X + kXQr, dt, c);
  ZAcc<T> acc;
  zside(c.s0, reinterpret_cast<const T(*)[5]>(X + kXD0), 0, K, c.eq1, c.eqh, acc, true);
  zside(c.sl, reinterpret_cast<const T(*)[5]>(X + kXDl), +1, K, c.in1, c.inh, acc, false);
  zside(c.sr, reinterpret_cast<const T(*)[5]>(X + kXDr), -1, K, c.in1, c.inh, acc, false);
  zflux_end(g, c, acc, dt, F, dF);
}

// The columns c0 .. c0 + kZTan - 1 of d(F, dF)/dX by forward tangents, contracted
// with the cotangents (Fb, dFb) of the Gauss point's F and dF/dt into Xb[c0 ..].
template <bool VAR_MU>
__host__ __device__ __forceinline__ void zflux_jt_columns(const Geo& g, const double* X, int c0, double dt,
                                                          const double* Fb, const double* dFb, double* Xb) {
  using TT = Tan<kZTan>;
  TT Xt[kXN];
#pragma unroll
  for (int i = 0; i < kXN; ++i) {
    Xt[i] = TT(X[i]);
#pragma unroll
    for (int j = 0; j < kZTan; ++j) Xt[i].d[j] = (i == c0 + j) ? 1.0 : 0.0;
  }
  TT F[5], dF[5];
  zgp_flux<VAR_MU>(g, Xt, TT(dt), F, dF);
#pragma unroll
  for (int j = 0; j < kZTan; ++j) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) s += Fb[k] * F[k].d[j] + dFb[k] * dF[k].d[j];
    Xb[c0 + j] = s;
  }
}

// All 60 entries of J^T (Fb, dFb) at one Gauss point, by the hand-written
// reverse sweep (zreverse.hpp).
template <bool VAR_MU>
__host__ __device__ __forceinline__ void zflux_jt_all(const Geo& g, const double* X, double dt, const double* Fb,
                                                      const double* dFb, double* Xb) {
  zflux_vjp<VAR_MU>(g, X, dt, Fb, dFb, Xb, kXQ0, kXQl, kXQr, kXD0, kXDl, kXDr);
}
// Jacobian of the WENO-Z edge pair of a five-value line:
// J[0][i] = d e_a / d v_i (left edge), J[1][i] = d e_b / d v_i (right edge).
__host__ __device__ __forceinline__ void wze_jac(const double* v, double eps, int p, double (*J)[5]) {
  Tan<5> t[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    t[i] = Tan<5>(v[i]);
    t[i].d[i] = 1.0;
  }
  Tan<5> ea, eb;
  weno_z_edges(t, Tan<5>(eps), p, ea, eb);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    J[0][i] = ea.d[i];
    J[1][i] = eb.d[i];
  }
}

// Jacobian of the WENO-Z right-edge value and slope of a five-value line.
__host__ __device__ __forceinline__ void wzr_jac(const double* v, double eps, int p, double* Jv, double* Js) {
  Tan<5> t[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    t[i] = Tan<5>(v[i]);
    t[i].d[i] = 1.0;
  }
  Tan<5> val, slope;
  weno_z_right(t, Tan<5>(eps), p, val, slope);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    Jv[i] = val.d[i];
    Js[i] = slope.d[i];
  }
}

}  // namespace hgks
