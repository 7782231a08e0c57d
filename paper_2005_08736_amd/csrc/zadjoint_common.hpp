// Building blocks of the mode-Z adjoint that run on forward tangents
// (tangent.hpp): the full flux at one Gauss point as a function of its 60
// reconstructed inputs, the transpose of its Jacobian applied to a cotangent, and
// the Jacobians of the WENO-Z edge pair and of the right-edge value and slope of a
// five-value line.  Host-and-device, so the CPU tests can check them against
// central differences.
#pragma once

#include "tangent.hpp"
#include "zflux.hpp"

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

// The 45 slope columns of J^T (Fb, dFb).  With the three Maxwellians fixed by the
// values, each side's contribution is linear in its own slopes D (15 of them) and
// the end formulas are linear in the accumulated moments, so a column is the
// linear part evaluated on a unit slope: plain double arithmetic, no tangents.
template <bool VAR_MU>
__host__ __device__ __forceinline__ void zflux_jt_slopes(const Geo& g, const double* X, double dt, const double* Fb,
                                                         const double* dFb, double* Xb) {
  ZCoef<double> c;
  zflux_begin<VAR_MU>(g, X + kXQ0, X + kXQl, X + kXQr, dt, c);
  const double K = g.K;
#pragma unroll 1
  for (int side = 0; side < 3; ++side) {
    const ZPrim<double>& s = side == 0 ? c.s0 : (side == 1 ? c.sl : c.sr);
    const double* k1 = side == 0 ? c.eq1 : c.in1;
    const double* kh = side == 0 ? c.eqh : c.inh;
    const int half = side == 0 ? 0 : (side == 1 ? +1 : -1);
    const int base = side == 0 ? kXD0 : (side == 1 ? kXDl : kXDr);
#pragma unroll 1
    for (int i = 0; i < 15; ++i) {
      double D[3][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
      D[i / 5][i % 5] = 1.0;
      ZAcc<double> acc;
      zside<true>(s, D, half, K, k1, kh, acc, true);
      double F[5], dF[5];
      zflux_end<true>(g, c, acc, dt, F, dF);
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k) sum += Fb[k] * F[k] + dFb[k] * dF[k];
      Xb[base + i] = sum;
    }
  }
}

// The 15 value columns of J^T (Fb, dFb) with one side per column.  A value input
// moves one Maxwellian (Q0 the equilibrium side, which also enters the Prandtl
// correction; Q_l, Q_r an initial side) and the collision time, which reaches
// every side only through its time-integral coefficients, linearly.  So a column
// runs the side it moves on a forward tangent, and adds the other two sides'
// moment rows (computed once, in double) times the tangents of their
// coefficients; begin and end run on the tangent as in zflux_jt_columns.
template <bool VAR_MU>
__host__ __device__ __forceinline__ void zflux_jt_values(const Geo& g, const double* X, double dt, const double* Fb,
                                                         const double* dFb, double* Xb) {
  using TT = Tan<1>;
  const double K = g.K;
  ZCoef<double> c;
  zflux_begin<VAR_MU>(g, X + kXQ0, X + kXQl, X + kXQr, dt, c);
  const ZPrim<double>* sp[3] = {&c.s0, &c.sl, &c.sr};
  double R[3][6][5];
#pragma unroll 1
  for (int side = 0; side < 3; ++side) {
    const int base = side == 0 ? kXD0 : (side == 1 ? kXDl : kXDr);
    zside_rows(*sp[side], reinterpret_cast<const double(*)[5]>(X + base), side == 0 ? 0 : (side == 1 ? +1 : -1), K,
               R[side]);
  }
  // the primal accumulators of all three sides
  ZAcc<double> a0;
#pragma unroll
  for (int k = 0; k < 5; ++k) a0.J1[k] = a0.Jh[k] = a0.I1[k] = a0.Ih[k] = 0.0;
#pragma unroll 1
  for (int side = 0; side < 3; ++side) {
    const double* k1 = side == 0 ? c.eq1 : c.in1;
    const double* kh = side == 0 ? c.eqh : c.inh;
    const double rho = sp[side]->rho;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      a0.J1[k] += rho * (k1[0] * R[side][0][k] + k1[1] * R[side][1][k] + k1[2] * R[side][2][k]);
      a0.Jh[k] += rho * (kh[0] * R[side][0][k] + kh[1] * R[side][1][k] + kh[2] * R[side][2][k]);
      a0.I1[k] += rho * (k1[0] * R[side][3][k] + k1[1] * R[side][4][k] + k1[2] * R[side][5][k]);
      a0.Ih[k] += rho * (kh[0] * R[side][3][k] + kh[1] * R[side][4][k] + kh[2] * R[side][5][k]);
    }
  }
#pragma unroll 1
  for (int i = 0; i < kXD0; ++i) {
    const int mv = i / 5;  // the side this input moves
    TT Xt[kXD0];
#pragma unroll
    for (int j = 0; j < kXD0; ++j) {
      Xt[j] = TT(X[j]);
      Xt[j].d[0] = j == i ? 1.0 : 0.0;
    }
    ZCoef<TT> ct;
    zflux_begin<VAR_MU>(g, Xt + kXQ0, Xt + kXQl, Xt + kXQr, TT(dt), ct);
    const ZPrim<TT>& st = mv == 0 ? ct.s0 : (mv == 1 ? ct.sl : ct.sr);
    const int base = mv == 0 ? kXD0 : (mv == 1 ? kXDl : kXDr);
    TT Dt[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int k = 0; k < 5; ++k) Dt[d][k] = TT(X[base + 5 * d + k]);
    ZAcc<TT> am;
    zside(st, Dt, mv == 0 ? 0 : (mv == 1 ? +1 : -1), TT(K), mv == 0 ? ct.eq1 : ct.in1, mv == 0 ? ct.eqh : ct.inh, am,
          true);
    // the accumulators on the tangent: their values the primal sums, their
    // derivatives the moved side's plus the others' rows times d(coefficients)
    ZAcc<TT> acc;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      acc.J1[k] = TT(a0.J1[k]);
      acc.Jh[k] = TT(a0.Jh[k]);
      acc.I1[k] = TT(a0.I1[k]);
      acc.Ih[k] = TT(a0.Ih[k]);
      acc.J1[k].d[0] = am.J1[k].d[0];
      acc.Jh[k].d[0] = am.Jh[k].d[0];
      acc.I1[k].d[0] = am.I1[k].d[0];
      acc.Ih[k].d[0] = am.Ih[k].d[0];
    }
#pragma unroll 1
    for (int side = 0; side < 3; ++side) {
      if (side == mv) continue;
      const TT* k1 = side == 0 ? ct.eq1 : ct.in1;
      const TT* kh = side == 0 ? ct.eqh : ct.inh;
      const double rho = sp[side]->rho;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        acc.J1[k].d[0] += rho * (k1[0].d[0] * R[side][0][k] + k1[1].d[0] * R[side][1][k] + k1[2].d[0] * R[side][2][k]);
        acc.Jh[k].d[0] += rho * (kh[0].d[0] * R[side][0][k] + kh[1].d[0] * R[side][1][k] + kh[2].d[0] * R[side][2][k]);
        acc.I1[k].d[0] += rho * (k1[0].d[0] * R[side][3][k] + k1[1].d[0] * R[side][4][k] + k1[2].d[0] * R[side][5][k]);
        acc.Ih[k].d[0] += rho * (kh[0].d[0] * R[side][3][k] + kh[1].d[0] * R[side][4][k] + kh[2].d[0] * R[side][5][k]);
      }
    }
    TT F[5], dF[5];
    zflux_end(g, ct, acc, TT(dt), F, dF);
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) sum += Fb[k] * F[k].d[0] + dFb[k] * dF[k].d[0];
    Xb[i] = sum;
  }
}

// All 60 entries of J^T (Fb, dFb): one moved side per value column, the linear
// side maps for the 45 slopes.
template <bool VAR_MU>
__host__ __device__ __forceinline__ void zflux_jt_all(const Geo& g, const double* X, double dt, const double* Fb,
                                                      const double* dFb, double* Xb) {
  zflux_jt_values<VAR_MU>(g, X, dt, Fb, dFb, Xb);
  zflux_jt_slopes<VAR_MU>(g, X, dt, Fb, dFb, Xb);
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
