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

// Transposes of the pieces of a side that are linear in its slopes (zside with
// the Maxwellian fixed): each maps the cotangents of a piece's outputs to those
// of its inputs.
// zslope: a = S b with S the closed-form solve of the 5 x 5 moment system.
template <typename T>
__host__ __device__ __forceinline__ void zslope_T(const T* ab, T U, T V, T W, const ZSlopeCoef<T>& c, T* bb) {
  // a0 = b0 - U a1 - V a2 - W a3 - Ep a4
  const T a1 = ab[1] - U * ab[0], a2 = ab[2] - V * ab[0], a3 = ab[3] - W * ab[0];
  // a1, a2, a3 = tl (B, C, D) - (U, V, W) a4
  const T a4 = ab[4] - c.Ep * ab[0] - U * a1 - V * a2 - W * a3;
  // a4 = c4 (b4 - Ep b0 - U B - V C - W D)
  const T t = c.c4 * a4;
  const T Bb = c.tl * a1 - U * t, Cb = c.tl * a2 - V * t, Db = c.tl * a3 - W * t;
  // B = b1 - U b0, C = b2 - V b0, D = b3 - W b0
  bb[0] = ab[0] - c.Ep * t - U * Bb - V * Cb - W * Db;
  bb[1] = Bb;
  bb[2] = Cb;
  bb[3] = Db;
  bb[4] = t;
}

// zrows<NC, BOTH>: adds to eb the cotangents of e from those of r0 (and r1).
template <int NC, bool BOTH, typename T>
__host__ __device__ __forceinline__ void zrows_T(const T* M, const T* r0b, const T* r1b, T (*eb)[4]) {
#pragma unroll
  for (int p = 0; p < (BOTH ? 2 : 1); ++p) {
    const T* rb = p ? r1b : r0b;
    const T h4 = T(0.5) * rb[4];
#pragma unroll
    for (int n = 0; n < NC; ++n) {
      eb[n][0] = eb[n][0] + M[n + p] * rb[0] + M[n + p + 1] * rb[1] + M[n + p + 2] * h4;
      eb[n][1] = eb[n][1] + M[n + p] * rb[2];
      eb[n][2] = eb[n][2] + M[n + p] * rb[3];
      eb[n][3] = eb[n][3] + M[n + p] * h4;
    }
  }
}

// zexpect<MASK>: cotangents of the coefficients c from those of e.
template <int MASK, typename T>
__host__ __device__ __forceinline__ void zexpect_T(const T* eb, const ZGauss<T>& G, T* cb) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    if (!((MASK >> i) & 1)) {
      cb[i] = T(0);
      continue;
    }
    const int b = zb_b(i), cc = zb_c(i), m = zb_m(i);
    cb[i] = eb[0] * G.E(b, cc, m) + eb[1] * G.E(b + 1, cc, m) + eb[2] * G.E(b, cc + 1, m) + eb[3] * G.E(b, cc, m + 1);
  }
}

// zexpect_slopes: cotangents of the slope polynomials a (along n, t1, t2).
template <typename T>
__host__ __device__ __forceinline__ void zexpect_slopes_T(const T (*eb)[4], const ZGauss<T>& G, T (*ab)[5]) {
  T c0[9], c1[9], c2[9], c3[9];
  zexpect_T<0x1BE>(eb[0], G, c0);
  zexpect_T<0x047>(eb[1], G, c1);
  zexpect_T<0x007>(eb[2], G, c2);
  zexpect_T<0x001>(eb[3], G, c3);
  T* n = ab[0];
  T* t = ab[1];
  T* r = ab[2];
  n[0] = c1[0];
  n[1] = c2[0];
  n[2] = c1[1];
  n[3] = c1[2];
  n[4] = T(0.5) * (c1[6] + c3[0]);
  t[0] = c0[1];
  t[1] = c1[1];
  t[2] = c0[3];
  t[3] = c0[4];
  t[4] = T(0.5) * (c0[7] + c2[1]);
  r[0] = c0[2];
  r[1] = c1[2];
  r[2] = c0[4];
  r[3] = c0[5];
  r[4] = T(0.5) * (c0[8] + c2[2]);
}

// zexpect_phi: cotangents of the time slope A.
template <typename T>
__host__ __device__ __forceinline__ void zexpect_phi_T(const T (*eb)[4], const ZGauss<T>& G, T* Ab) {
  T c0[9], c1[9], c2[9];
  zexpect_T<0x047>(eb[0], G, c0);
  zexpect_T<0x001>(eb[1], G, c1);
  zexpect_T<0x001>(eb[2], G, c2);
  Ab[0] = c0[0];
  Ab[1] = c1[0];
  Ab[2] = c0[1];
  Ab[3] = c0[2];
  Ab[4] = T(0.5) * (c0[6] + c2[0]);
}

// Cotangents of one side's slopes D[3][5] (local frame) from those of the Gauss
// point's F and dF/dt (Fb, dFb), with the Maxwellians and the collision time
// fixed: the transpose of the side's part that is linear in D (zside<true>)
// followed by the end formulas (zflux_end<true>), taken in reverse order.
template <typename T>
__host__ __device__ __forceinline__ void zside_slopes_T(const Geo& g, const ZCoef<T>& c, int side, T K, T dt,
                                                        const T* Fb, const T* dFb, T (*Db)[5]) {
  const ZPrim<T>& s = side == 0 ? c.s0 : (side == 1 ? c.sl : c.sr);
  const T* k1 = side == 0 ? c.eq1 : c.in1;
  const T* kh = side == 0 ? c.eqh : c.inh;
  const int half = side == 0 ? 0 : (side == 1 ? +1 : -1);
  // end formulas: F = (4 Ih - I1)/dt, dF = 4 (I1 - 2 Ih)/dt^2 after the Prandtl
  // correction I[4] += fix (h(I) - U0 h(J)), h(G) = G4 - U0.G(1:3) + |U0|^2/2 G0
  const T idt = T(1) / dt;
  T I1b[5], Ihb[5], J1b[5], Jhb[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    I1b[k] = -Fb[k] * idt + T(4) * dFb[k] * idt * idt;
    Ihb[k] = T(4) * Fb[k] * idt - T(8) * dFb[k] * idt * idt;
  }
  {
    const T U0 = c.s0.U, V0 = c.s0.V, W0 = c.s0.W;
    const T hg[5] = {T(0.5) * (U0 * U0 + V0 * V0 + W0 * W0), -U0, -V0, -W0, T(1)};
    const T fix = T(g.pr_fix);
    const T q1 = fix * I1b[4], qh = fix * Ihb[4];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      J1b[k] = -U0 * q1 * hg[k];
      Jhb[k] = -U0 * qh * hg[k];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      I1b[k] = I1b[k] + q1 * hg[k];
      Ihb[k] = Ihb[k] + qh * hg[k];
    }
  }
  // accumulation: J = rho (k . rows 0..2), I = rho (k . rows 3..5); the phi = 1
  // rows do not depend on D
  T ra0b[5], ra1b[5], rA0b[5], rA1b[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    ra0b[k] = s.rho * (k1[1] * J1b[k] + kh[1] * Jhb[k]);
    ra1b[k] = s.rho * (k1[1] * I1b[k] + kh[1] * Ihb[k]);
    rA0b[k] = s.rho * (k1[2] * J1b[k] + kh[2] * Jhb[k]);
    rA1b[k] = s.rho * (k1[2] * I1b[k] + kh[2] * Ihb[k]);
  }
  // the side's Gaussian moments, full-space (Mf) and of the rows' space (Mh)
  const T i2l = T(0.5) / s.lam;
  ZGauss<T> G;
  zmom_gauss(G.v, 6, s.V, i2l);
  zmom_gauss(G.w, 6, s.W, i2l);
  G.x1 = K * i2l;
  G.x2 = K * (K + T(2)) * i2l * i2l;
  T Mf[7], Mh[7];
  zmom_gauss(Mf, 7, s.U, i2l);
  if (half != 0) zmom_half(Mh, s.U, s.lam, i2l, T(half));
  else
#pragma unroll
    for (int n = 0; n < 7; ++n) Mh[n] = Mf[n];
  const ZSlopeCoef<T> sc = zslope_coef(s.U, s.V, s.W, s.lam, i2l, K);
  // A rows: (rA0, rA1) = zrows<3, true>(Mh, zexpect_phi(A)), A = zslope(-ra_full)
  T eAb[3][4] = {{T(0), T(0), T(0), T(0)}, {T(0), T(0), T(0), T(0)}, {T(0), T(0), T(0), T(0)}};
  zrows_T<3, true>(Mh, rA0b, rA1b, eAb);
  T Ab[5], btb[5];
  zexpect_phi_T(eAb, G, Ab);
  zslope_T(Ab, s.U, s.V, s.W, sc, btb);
  T rfb[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) rfb[k] = -btb[k];
  // a.u rows: (ra0, ra1) = zrows<4, true>(Mh, ea), ra_full = zrows<4, false>(Mf, ea)
  T eab[4][4];
#pragma unroll
  for (int n = 0; n < 4; ++n) eab[n][0] = eab[n][1] = eab[n][2] = eab[n][3] = T(0);
  zrows_T<4, true>(Mh, ra0b, ra1b, eab);
  zrows_T<4, false>(Mf, rfb, rfb, eab);
  T ab[3][5];
  zexpect_slopes_T(eab, G, ab);
  // a[d] = zslope(D[d] / rho)
  const T ir = T(1) / s.rho;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T bb[5];
    zslope_T(ab[d], s.U, s.V, s.W, sc, bb);
#pragma unroll
    for (int k = 0; k < 5; ++k) Db[d][k] = bb[k] * ir;
  }
}

// The 45 slope entries of J^T (Fb, dFb): with the three Maxwellians fixed by the
// values, each side's contribution is linear in its own slopes and the end
// formulas are linear in the accumulated moments, so the slopes' cotangents are
// that linear map's transpose applied once per side (zside_slopes_T).
template <bool VAR_MU>
__host__ __device__ __forceinline__ void zflux_jt_slopes(const Geo& g, const double* X, double dt, const double* Fb,
                                                         const double* dFb, double* Xb) {
  ZCoef<double> c;
  zflux_begin<VAR_MU>(g, X + kXQ0, X + kXQl, X + kXQr, dt, c);
  const double K = g.K;
#pragma unroll 1
  for (int side = 0; side < 3; ++side) {
    const int base = side == 0 ? kXD0 : (side == 1 ? kXDl : kXDr);
    double Db[3][5];
    zside_slopes_T(g, c, side, K, dt, Fb, dFb, Db);
#pragma unroll
    for (int i = 0; i < 15; ++i) Xb[base + i] = Db[i / 5][i % 5];
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
