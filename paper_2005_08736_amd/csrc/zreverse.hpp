// Reverse mode, written by hand, of the WENO-Z line reconstructions (edge pair
// and right-edge value and slope of five cell averages) and of the mode-Z full
// flux at one Gauss point (Eq. (flux) integrated over dt and dt/2,
// Eq. (expansion-1)).  For the flux: the cotangents of all 60 inputs (Q0, Q_l,
// Q_r and their slopes D0, D_l, D_r) from those of F^n and dF^n/dt in one
// backward sweep.  Each forward piece of zflux.hpp has its reverse here, taken in
// the opposite order: the end formulas and the Prandtl correction, the
// accumulation of the three sides, each side's moment rows (the u-power
// contractions, the Gaussian expectations in (v, w, xi), the closed-form slope
// solves, the full- and half-space moment recursions), the time-integral
// coefficients, the collision time and the primitive variables.  Host-and-device
// plain double arithmetic, so the CPU tests can check it against the
// forward-tangent Jacobians.
#pragma once

#include "zflux.hpp"

namespace hgks {

// ---------------------------------------------------------------------------
// WENO-Z on five cell averages (weno_z_edges, weno_z_right), reversed.
// ---------------------------------------------------------------------------
// The Z ratios r_k = (tau5 / (b_k + eps))^p, tau5 = |b0 - b2|: from their
// cotangents rb, adds those of the indicators to bb (d|x|/dx at 0 taken as +1).
__host__ __device__ __forceinline__ void zratios_rev(double b0, double b1, double b2, double eps, int p,
                                                     const double* rb, double* bb) {
  const double tau5 = fabs(b0 - b2);
  const double d[3] = {b0 + eps, b1 + eps, b2 + eps};
  double tb = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double x = tau5 / d[k];
    double xp = 1.0;  // x^(p-1)
    for (int i = 1; i < p; ++i) xp *= x;
    const double xb = double(p) * xp * rb[k];
    tb += xb / d[k];
    bb[k] -= xb * x / d[k];
  }
  const double sg = b0 - b2 >= 0.0 ? 1.0 : -1.0;
  bb[0] += sg * tb;
  bb[2] -= sg * tb;
}

// The Jiang-Shu indicators (zbeta): adds the cotangents of v from those of b.
__host__ __device__ __forceinline__ void zbeta_rev(const double* v, const double* bb, double* vb) {
  const double c13 = 13.0 / 12.0;
  const double s0 = v[0] - 2.0 * v[1] + v[2], t0 = v[0] - 4.0 * v[1] + 3.0 * v[2];
  const double s1 = v[1] - 2.0 * v[2] + v[3], t1 = v[1] - v[3];
  const double s2 = v[2] - 2.0 * v[3] + v[4], t2 = 3.0 * v[2] - 4.0 * v[3] + v[4];
  const double s0b = 2.0 * c13 * s0 * bb[0], t0b = 0.5 * t0 * bb[0];
  const double s1b = 2.0 * c13 * s1 * bb[1], t1b = 0.5 * t1 * bb[1];
  const double s2b = 2.0 * c13 * s2 * bb[2], t2b = 0.5 * t2 * bb[2];
  vb[0] += s0b + t0b;
  vb[1] += -2.0 * s0b - 4.0 * t0b + s1b + t1b;
  vb[2] += s0b + 3.0 * t0b - 2.0 * s1b + s2b + 3.0 * t2b;
  vb[3] += s1b - t1b - 2.0 * s2b - 4.0 * t2b;
  vb[4] += s2b + t2b;
}

// Indicators and Z ratios of a line (the forward of both edge functions).
__host__ __device__ __forceinline__ void zweights_fwd(const double* v, double eps, int p, double* b, double* r) {
  zbeta(v, b[0], b[1], b[2]);
  zratios(fabs(b[0] - b[2]), b[0], b[1], b[2], eps, p, r[0], r[1], r[2]);
}

// weno_z_edges: adds to vb the cotangents of the line from those of its left
// (eab) and right (ebb) edge values.
__host__ __device__ __forceinline__ void weno_z_edges_vjp(const double* v, double eps, int p, double eab,
                                                          double ebb, double* vb) {
  double b[3], r[3];
  zweights_fwd(v, eps, p, b, r);
  double rb[3] = {0.0, 0.0, 0.0};
  {
    // right edge: eb = sum a_k q_k / sum a_k, a = (0.1 (1 + r0), 0.6 (1 + r1), 0.3 (1 + r2))
    const double a[3] = {0.1 * (1.0 + r[0]), 0.6 * (1.0 + r[1]), 0.3 * (1.0 + r[2])};
    const double q[3] = {(1.0 / 3.0) * v[0] - (7.0 / 6.0) * v[1] + (11.0 / 6.0) * v[2],
                         (-1.0 / 6.0) * v[1] + (5.0 / 6.0) * v[2] + (1.0 / 3.0) * v[3],
                         (1.0 / 3.0) * v[2] + (5.0 / 6.0) * v[3] - (1.0 / 6.0) * v[4]};
    const double S = a[0] + a[1] + a[2];
    const double e = (a[0] * q[0] + a[1] * q[1] + a[2] * q[2]) / S;
    rb[0] += 0.1 * (q[0] - e) / S * ebb;
    rb[1] += 0.6 * (q[1] - e) / S * ebb;
    rb[2] += 0.3 * (q[2] - e) / S * ebb;
    const double q0b = a[0] / S * ebb, q1b = a[1] / S * ebb, q2b = a[2] / S * ebb;
    vb[0] += (1.0 / 3.0) * q0b;
    vb[1] += (-7.0 / 6.0) * q0b + (-1.0 / 6.0) * q1b;
    vb[2] += (11.0 / 6.0) * q0b + (5.0 / 6.0) * q1b + (1.0 / 3.0) * q2b;
    vb[3] += (1.0 / 3.0) * q1b + (5.0 / 6.0) * q2b;
    vb[4] += (-1.0 / 6.0) * q2b;
  }
  {
    // left edge on the reversed line: a = (0.1 (1 + r2), 0.6 (1 + r1), 0.3 (1 + r0))
    const double a[3] = {0.1 * (1.0 + r[2]), 0.6 * (1.0 + r[1]), 0.3 * (1.0 + r[0])};
    const double q[3] = {(1.0 / 3.0) * v[4] - (7.0 / 6.0) * v[3] + (11.0 / 6.0) * v[2],
                         (-1.0 / 6.0) * v[3] + (5.0 / 6.0) * v[2] + (1.0 / 3.0) * v[1],
                         (1.0 / 3.0) * v[2] + (5.0 / 6.0) * v[1] - (1.0 / 6.0) * v[0]};
    const double S = a[0] + a[1] + a[2];
    const double e = (a[0] * q[0] + a[1] * q[1] + a[2] * q[2]) / S;
    rb[2] += 0.1 * (q[0] - e) / S * eab;
    rb[1] += 0.6 * (q[1] - e) / S * eab;
    rb[0] += 0.3 * (q[2] - e) / S * eab;
    const double q0b = a[0] / S * eab, q1b = a[1] / S * eab, q2b = a[2] / S * eab;
    vb[4] += (1.0 / 3.0) * q0b;
    vb[3] += (-7.0 / 6.0) * q0b + (-1.0 / 6.0) * q1b;
    vb[2] += (11.0 / 6.0) * q0b + (5.0 / 6.0) * q1b + (1.0 / 3.0) * q2b;
    vb[1] += (1.0 / 3.0) * q1b + (5.0 / 6.0) * q2b;
    vb[0] += (-1.0 / 6.0) * q2b;
  }
  double bb[3] = {0.0, 0.0, 0.0};
  zratios_rev(b[0], b[1], b[2], eps, p, rb, bb);
  zbeta_rev(v, bb, vb);
}

// weno_z_right: adds to vb the cotangents of the line from those of the right
// edge value (valb) and slope (slopeb).
__host__ __device__ __forceinline__ void weno_z_right_vjp(const double* v, double eps, int p, double valb,
                                                          double slopeb, double* vb) {
  double b[3], r[3];
  zweights_fwd(v, eps, p, b, r);
  const double a[3] = {0.1 * (1.0 + r[0]), 0.6 * (1.0 + r[1]), 0.3 * (1.0 + r[2])};
  const double S = a[0] + a[1] + a[2];
  const double w[3] = {a[0] / S, a[1] / S, a[2] / S};
  const double q[3] = {(1.0 / 3.0) * v[0] - (7.0 / 6.0) * v[1] + (11.0 / 6.0) * v[2],
                       (-1.0 / 6.0) * v[1] + (5.0 / 6.0) * v[2] + (1.0 / 3.0) * v[3],
                       (1.0 / 3.0) * v[2] + (5.0 / 6.0) * v[3] - (1.0 / 6.0) * v[4]};
  const double d0 = v[0] - 3.0 * v[1] + 2.0 * v[2], d1 = v[3] - v[2];
  // val = sum w_k q_k, slope = w0 d0 + (w1 + w2) d1, w = a / sum a
  const double wb[3] = {q[0] * valb + d0 * slopeb, q[1] * valb + d1 * slopeb, q[2] * valb + d1 * slopeb};
  const double ww = w[0] * wb[0] + w[1] * wb[1] + w[2] * wb[2];
  const double rb[3] = {0.1 * (wb[0] - ww) / S, 0.6 * (wb[1] - ww) / S, 0.3 * (wb[2] - ww) / S};
  const double q0b = w[0] * valb, q1b = w[1] * valb, q2b = w[2] * valb;
  const double d0b = w[0] * slopeb, d1b = (w[1] + w[2]) * slopeb;
  vb[0] += (1.0 / 3.0) * q0b + d0b;
  vb[1] += (-7.0 / 6.0) * q0b + (-1.0 / 6.0) * q1b - 3.0 * d0b;
  vb[2] += (11.0 / 6.0) * q0b + (5.0 / 6.0) * q1b + (1.0 / 3.0) * q2b + 2.0 * d0b - d1b;
  vb[3] += (1.0 / 3.0) * q1b + (5.0 / 6.0) * q2b + d1b;
  vb[4] += (-1.0 / 6.0) * q2b;
  double bb[3] = {0.0, 0.0, 0.0};
  zratios_rev(b[0], b[1], b[2], eps, p, rb, bb);
  zbeta_rev(v, bb, vb);
}

// Cotangents of the Gaussian factors of a side (ZGauss).
struct ZGaussB {
  double v[6], w[6], x1, x2;
};

__host__ __device__ __forceinline__ void zgaussb_zero(ZGaussB& b) {
#pragma unroll
  for (int i = 0; i < 6; ++i) b.v[i] = b.w[i] = 0.0;
  b.x1 = b.x2 = 0.0;
}

// E(b, c, m) of ZGauss: adds Eb times its partial derivatives to Gb.
__host__ __device__ __forceinline__ void zgauss_E_rev(const ZGauss<double>& G, int b, int c, int m, double Eb,
                                                      ZGaussB& Gb) {
  if (m == 0) {
    Gb.v[b] += Eb * G.w[c];
    Gb.w[c] += Eb * G.v[b];
    return;
  }
  if (m == 1) {
    // v[b+2] w[c] + v[b] w[c+2] + v[b] w[c] x1
    Gb.v[b + 2] += Eb * G.w[c];
    Gb.w[c] += Eb * (G.v[b + 2] + G.v[b] * G.x1);
    Gb.v[b] += Eb * (G.w[c + 2] + G.w[c] * G.x1);
    Gb.w[c + 2] += Eb * G.v[b];
    Gb.x1 += Eb * G.v[b] * G.w[c];
    return;
  }
  // v[b+4] w[c] + v[b] w[c+4] + v[b] w[c] x2 + 2 (v[b+2] w[c+2] + v[b+2] w[c] x1 + v[b] w[c+2] x1)
  Gb.v[b + 4] += Eb * G.w[c];
  Gb.w[c] += Eb * (G.v[b + 4] + G.v[b] * G.x2 + 2.0 * G.v[b + 2] * G.x1);
  Gb.v[b] += Eb * (G.w[c + 4] + G.w[c] * G.x2 + 2.0 * G.w[c + 2] * G.x1);
  Gb.w[c + 4] += Eb * G.v[b];
  Gb.x2 += Eb * G.v[b] * G.w[c];
  Gb.v[b + 2] += Eb * 2.0 * (G.w[c + 2] + G.w[c] * G.x1);
  Gb.w[c + 2] += Eb * 2.0 * (G.v[b + 2] + G.v[b] * G.x1);
  Gb.x1 += Eb * 2.0 * (G.v[b + 2] * G.w[c] + G.v[b] * G.w[c + 2]);
}

// zexpect<MASK>: cotangents of the coefficients c (cb, overwritten) and of G
// (added) from those of e.
template <int MASK>
__host__ __device__ __forceinline__ void zexpect_rev(const double* c, const ZGauss<double>& G, const double* eb,
                                                     double* cb, ZGaussB& Gb) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    if (!((MASK >> i) & 1)) {
      cb[i] = 0.0;
      continue;
    }
    const int b = zb_b(i), cc = zb_c(i), m = zb_m(i);
    cb[i] = eb[0] * G.E(b, cc, m) + eb[1] * G.E(b + 1, cc, m) + eb[2] * G.E(b, cc + 1, m) + eb[3] * G.E(b, cc, m + 1);
    zgauss_E_rev(G, b, cc, m, c[i] * eb[0], Gb);
    zgauss_E_rev(G, b + 1, cc, m, c[i] * eb[1], Gb);
    zgauss_E_rev(G, b, cc + 1, m, c[i] * eb[2], Gb);
    zgauss_E_rev(G, b, cc, m + 1, c[i] * eb[3], Gb);
  }
}

// zexpect_slopes: cotangents of the slope polynomials a (ab, overwritten) and of G.
__host__ __device__ __forceinline__ void zexpect_slopes_rev(const double (*a)[5], const ZGauss<double>& G,
                                                            const double (*eb)[4], double (*ab)[5], ZGaussB& Gb) {
  const double* n = a[0];
  const double* t = a[1];
  const double* r = a[2];
  const double c0[9] = {0.0, t[0], r[0], t[2], t[3] + r[2], r[3], 0.0, 0.5 * t[4], 0.5 * r[4]};
  const double c1[9] = {n[0], n[2] + t[1], n[3] + r[1], 0.0, 0.0, 0.0, 0.5 * n[4], 0.0, 0.0};
  const double c2[9] = {n[1], 0.5 * t[4], 0.5 * r[4], 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double c3[9] = {0.5 * n[4], 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double b0[9], b1[9], b2[9], b3[9];
  zexpect_rev<0x1BE>(c0, G, eb[0], b0, Gb);
  zexpect_rev<0x047>(c1, G, eb[1], b1, Gb);
  zexpect_rev<0x007>(c2, G, eb[2], b2, Gb);
  zexpect_rev<0x001>(c3, G, eb[3], b3, Gb);
  double* nb = ab[0];
  double* tb = ab[1];
  double* rb = ab[2];
  nb[0] = b1[0];
  nb[1] = b2[0];
  nb[2] = b1[1];
  nb[3] = b1[2];
  nb[4] = 0.5 * (b1[6] + b3[0]);
  tb[0] = b0[1];
  tb[1] = b1[1];
  tb[2] = b0[3];
  tb[3] = b0[4];
  tb[4] = 0.5 * (b0[7] + b2[1]);
  rb[0] = b0[2];
  rb[1] = b1[2];
  rb[2] = b0[4];
  rb[3] = b0[5];
  rb[4] = 0.5 * (b0[8] + b2[2]);
}

// zexpect_phi: cotangents of the time slope A (Ab, overwritten) and of G.
__host__ __device__ __forceinline__ void zexpect_phi_rev(const double* A, const ZGauss<double>& G,
                                                         const double (*eb)[4], double* Ab, ZGaussB& Gb) {
  const double c0[9] = {A[0], A[2], A[3], 0.0, 0.0, 0.0, 0.5 * A[4], 0.0, 0.0};
  const double c1[9] = {A[1], 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double c2[9] = {0.5 * A[4], 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double b0[9], b1[9], b2[9];
  zexpect_rev<0x047>(c0, G, eb[0], b0, Gb);
  zexpect_rev<0x001>(c1, G, eb[1], b1, Gb);
  zexpect_rev<0x001>(c2, G, eb[2], b2, Gb);
  Ab[0] = b0[0];
  Ab[1] = b1[0];
  Ab[2] = b0[1];
  Ab[3] = b0[2];
  Ab[4] = 0.5 * (b0[6] + b2[0]);
}

// zrows<NC, BOTH>: adds the cotangents of e and of the u-moments M.
template <int NC, bool BOTH>
__host__ __device__ __forceinline__ void zrows_rev(const double* M, const double (*e)[4], const double* r0b,
                                                   const double* r1b, double (*eb)[4], double* Mb) {
#pragma unroll
  for (int p = 0; p < (BOTH ? 2 : 1); ++p) {
    const double* rb = p ? r1b : r0b;
    const double h4 = 0.5 * rb[4];
#pragma unroll
    for (int n = 0; n < NC; ++n) {
      eb[n][0] += M[n + p] * rb[0] + M[n + p + 1] * rb[1] + M[n + p + 2] * h4;
      eb[n][1] += M[n + p] * rb[2];
      eb[n][2] += M[n + p] * rb[3];
      eb[n][3] += M[n + p] * h4;
      Mb[n + p] += e[n][0] * rb[0] + e[n][1] * rb[2] + e[n][2] * rb[3] + e[n][3] * h4;
      Mb[n + p + 1] += e[n][0] * rb[1];
      Mb[n + p + 2] += e[n][0] * h4;
    }
  }
}

// Cotangents of the factors of the slope solves (ZSlopeCoef).
struct ZSlopeCoefB {
  double Ep, c4, tl;
};

// zslope: a = S(b; U, V, W, Ep, c4, tl), a given; adds the cotangents of b (bb,
// overwritten), U, V, W and the factors.
__host__ __device__ __forceinline__ void zslope_rev(const double* b, double U, double V, double W,
                                                    const ZSlopeCoef<double>& c, const double* a, const double* ab,
                                                    double* bb, double& Ub, double& Vb, double& Wb, ZSlopeCoefB& cb) {
  const double B = b[1] - U * b[0], C = b[2] - V * b[0], D = b[3] - W * b[0];
  const double t = b[4] - c.Ep * b[0] - U * B - V * C - W * D;
  // a0 = b0 - U a1 - V a2 - W a3 - Ep a4
  double b0b = ab[0];
  const double a1b = ab[1] - U * ab[0], a2b = ab[2] - V * ab[0], a3b = ab[3] - W * ab[0];
  double a4b = ab[4] - c.Ep * ab[0];
  Ub -= a[1] * ab[0];
  Vb -= a[2] * ab[0];
  Wb -= a[3] * ab[0];
  cb.Ep -= a[4] * ab[0];
  // a1, a2, a3 = tl (B, C, D) - (U, V, W) a4
  double Bb = c.tl * a1b, Cb = c.tl * a2b, Db = c.tl * a3b;
  cb.tl += B * a1b + C * a2b + D * a3b;
  a4b -= U * a1b + V * a2b + W * a3b;
  Ub -= a[4] * a1b;
  Vb -= a[4] * a2b;
  Wb -= a[4] * a3b;
  // a4 = c4 t, t = b4 - Ep b0 - U B - V C - W D
  const double tb = c.c4 * a4b;
  cb.c4 += t * a4b;
  bb[4] = tb;
  b0b -= c.Ep * tb;
  cb.Ep -= b[0] * tb;
  Bb -= U * tb;
  Cb -= V * tb;
  Db -= W * tb;
  Ub -= B * tb;
  Vb -= C * tb;
  Wb -= D * tb;
  // B = b1 - U b0, C = b2 - V b0, D = b3 - W b0
  bb[1] = Bb;
  bb[2] = Cb;
  bb[3] = Db;
  bb[0] = b0b - U * Bb - V * Cb - W * Db;
  Ub -= b[0] * Bb;
  Vb -= b[0] * Cb;
  Wb -= b[0] * Db;
}

// The recursion M[k] = U M[k-1] + (k-1) i2l M[k-2] for k = 2 .. n-1 from M[0],
// M[1]: moves the cotangents of M[k >= 2] onto M[0], M[1], U and i2l.
__host__ __device__ __forceinline__ void zmom_rec_rev(const double* M, int n, double U, double i2l, double* Mb,
                                                      double& Ub, double& i2lb) {
  for (int k = n - 1; k >= 2; --k) {
    Ub += Mb[k] * M[k - 1];
    Mb[k - 1] += U * Mb[k];
    i2lb += double(k - 1) * M[k - 2] * Mb[k];
    Mb[k - 2] += double(k - 1) * i2l * Mb[k];
  }
}

// zmom_half (u > 0 for sign = +1, u < 0 for -1): cotangents of U, lambda and i2l.
__host__ __device__ __forceinline__ void zmom_half_rev(const double* M, double U, double lam, double i2l, double sign,
                                                       double* Mb, double& Ub, double& lamb, double& i2lb) {
  const double kInvSqrtPi = 0.56418958354775628695;
  zmom_rec_rev(M, 7, U, i2l, Mb, Ub, i2lb);
  const double sl = sqrt(lam);
  const double x = sl * U;
  const double e = exp(-x * x);
  // M1 = U M0 + sign/2 e / (sqrt(pi) sl)
  Ub += M[0] * Mb[1];
  const double M0b = Mb[0] + U * Mb[1];
  const double eb = sign * 0.5 * kInvSqrtPi / sl * Mb[1];
  double slb = -sign * 0.5 * kInvSqrtPi * e / (sl * sl) * Mb[1];
  double xb = -2.0 * x * e * eb;
  // M0 = 1/2 + sign/2 erf(x)
  xb += sign * kInvSqrtPi * e * M0b;
  // x = sl U
  slb += U * xb;
  Ub += sl * xb;
  lamb += slb / (2.0 * sl);
}

// Cotangents of one side's primitive state.
struct ZPrimB {
  double rho, U, V, W, p, lam;
};

// zside_rows: from the cotangents of the six moment rows Rb, the cotangents of
// the side's primitive state (added to sb) and of its slopes (Db, overwritten).
__host__ __device__ __forceinline__ void zside_rows_rev(const ZPrim<double>& s, const double (*D)[5], int half,
                                                        double K, const double (*Rb)[5], ZPrimB& sb, double (*Db)[5]) {
  // forward, keeping what the reverse needs
  const double i2l = 0.5 / s.lam;
  ZGauss<double> G;
  zmom_gauss(G.v, 6, s.V, i2l);
  zmom_gauss(G.w, 6, s.W, i2l);
  G.x1 = K * i2l;
  G.x2 = K * (K + 2.0) * i2l * i2l;
  double Mf[7], Mh[7];
  zmom_gauss(Mf, 7, s.U, i2l);
  const ZSlopeCoef<double> sc = zslope_coef(s.U, s.V, s.W, s.lam, i2l, K);
  const double ir = 1.0 / s.rho;
  double b[3][5], a[3][5];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int k = 0; k < 5; ++k) b[d][k] = D[d][k] * ir;
    zslope(b[d], s.U, s.V, s.W, sc, a[d]);
  }
  double ea[4][4];
  zexpect_slopes(a, G, ea);
  double raf[5], unused[5], bt[5], A[5];
  zrows<4, false>(Mf, ea, raf, unused);
#pragma unroll
  for (int k = 0; k < 5; ++k) bt[k] = -raf[k];
  zslope(bt, s.U, s.V, s.W, sc, A);
  if (half != 0) zmom_half(Mh, s.U, s.lam, i2l, double(half));
  else
#pragma unroll
    for (int n = 0; n < 7; ++n) Mh[n] = Mf[n];
  double eA[3][4];
  zexpect_phi(A, G, eA);
  const double e1[1][4] = {{1.0, s.V, s.W, G.E(0, 0, 1)}};

  // reverse
  double Mhb[7], Mfb[7];
#pragma unroll
  for (int n = 0; n < 7; ++n) Mhb[n] = Mfb[n] = 0.0;
  double eab[4][4], eAb[3][4], e1b[1][4] = {{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
  for (int n = 0; n < 4; ++n) eab[n][0] = eab[n][1] = eab[n][2] = eab[n][3] = 0.0;
#pragma unroll
  for (int n = 0; n < 3; ++n) eAb[n][0] = eAb[n][1] = eAb[n][2] = eAb[n][3] = 0.0;
  ZGaussB Gb;
  zgaussb_zero(Gb);
  ZSlopeCoefB scb = {0.0, 0.0, 0.0};
  double Ub = 0.0, Vb = 0.0, Wb = 0.0, i2lb = 0.0, lamb = 0.0;
  // rows: (R0, R3) phi = 1, (R1, R4) a.u, (R2, R5) A, all over Mh
  zrows_rev<1, true>(Mh, e1, Rb[0], Rb[3], e1b, Mhb);
  zrows_rev<4, true>(Mh, ea, Rb[1], Rb[4], eab, Mhb);
  zrows_rev<3, true>(Mh, eA, Rb[2], Rb[5], eAb, Mhb);
  // e1 = (1, V, W, E(0, 0, 1))
  Vb += e1b[0][1];
  Wb += e1b[0][2];
  zgauss_E_rev(G, 0, 0, 1, e1b[0][3], Gb);
  // eA = zexpect_phi(A), A = zslope(-raf), raf = zrows<4, false>(Mf, ea)
  double Ab[5], btb[5], rafb[5];
  zexpect_phi_rev(A, G, eAb, Ab, Gb);
  zslope_rev(bt, s.U, s.V, s.W, sc, A, Ab, btb, Ub, Vb, Wb, scb);
#pragma unroll
  for (int k = 0; k < 5; ++k) rafb[k] = -btb[k];
  zrows_rev<4, false>(Mf, ea, rafb, rafb, eab, Mfb);
  // ea = zexpect_slopes(a), a[d] = zslope(b[d]), b = D / rho
  double ab[3][5];
  zexpect_slopes_rev(a, G, eab, ab, Gb);
  double irb = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double bb[5];
    zslope_rev(b[d], s.U, s.V, s.W, sc, a[d], ab[d], bb, Ub, Vb, Wb, scb);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      Db[d][k] = bb[k] * ir;
      irb += bb[k] * D[d][k];
    }
  }
  sb.rho -= irb * ir * ir;
  // Mh: half-space moments, or the full-space ones
  if (half != 0) zmom_half_rev(Mh, s.U, s.lam, i2l, double(half), Mhb, Ub, lamb, i2lb);
  else
#pragma unroll
    for (int n = 0; n < 7; ++n) Mfb[n] += Mhb[n];
  // Mf = gauss(U); G.v = gauss(V), G.w = gauss(W), x1 = K i2l, x2 = K (K + 2) i2l^2
  zmom_rec_rev(Mf, 7, s.U, i2l, Mfb, Ub, i2lb);
  Ub += Mfb[1];
  zmom_rec_rev(G.v, 6, s.V, i2l, Gb.v, Vb, i2lb);
  Vb += Gb.v[1];
  zmom_rec_rev(G.w, 6, s.W, i2l, Gb.w, Wb, i2lb);
  Wb += Gb.w[1];
  i2lb += K * Gb.x1 + 2.0 * K * (K + 2.0) * i2l * Gb.x2;
  // Ep = (U^2 + V^2 + W^2 + (K + 3) i2l) / 2, c4 = 8 lambda^2 / (K + 3), tl = 2 lambda
  Ub += s.U * scb.Ep;
  Vb += s.V * scb.Ep;
  Wb += s.W * scb.Ep;
  i2lb += 0.5 * (K + 3.0) * scb.Ep;
  lamb += 16.0 * s.lam / (K + 3.0) * scb.c4 + 2.0 * scb.tl;
  // i2l = 1 / (2 lambda)
  lamb -= 0.5 / (s.lam * s.lam) * i2lb;
  sb.U += Ub;
  sb.V += Vb;
  sb.W += Wb;
  sb.lam += lamb;
}

// ztime: cotangent of tau from those of the coefficients over [0, delta].
__host__ __device__ __forceinline__ double ztime_rev(double delta, double tau, const double* eqb, const double* inb) {
  const double e = exp(-delta / tau);
  const double om = 1.0 - e;
  // d e / d tau; where e has underflowed (tau = 0 in an inviscid run without the
  // artificial term, or delta >> tau) its limit 0 is taken instead of 0 / 0
  const double et = e > 0.0 ? e * delta / (tau * tau) : 0.0;
  double r = 0.0;
  r += eqb[0] * (-om + tau * et);
  r += eqb[1] * (4.0 * tau * om - 2.0 * tau * tau * et - delta * (1.0 + e) - tau * delta * et);
  r += eqb[2] * (-delta + 2.0 * tau * om - tau * tau * et);
  r += inb[0] * (om - tau * et);
  r += inb[1] * (-4.0 * tau * om + 2.0 * tau * tau * et + delta * e + tau * delta * et);
  r += inb[2] * (-2.0 * tau * om + tau * tau * et);
  return r;
}

// zprim: adds the cotangents of the deviation state dQ from those of the
// primitive state.
__host__ __device__ __forceinline__ void zprim_rev(const Geo& g, const double* dQ, const ZPrim<double>& s, ZPrimB sb,
                                                   double* dQb) {
  // lambda = rho / (2 p)
  sb.p -= sb.lam * 0.5 * s.rho / (s.p * s.p);
  sb.rho += sb.lam * 0.5 / s.p;
  // p = p_ref + (gamma - 1) (dQ4 - rho |U|^2 / 2)
  dQb[4] += g.gm1 * sb.p;
  sb.rho -= g.gm1 * 0.5 * (s.U * s.U + s.V * s.V + s.W * s.W) * sb.p;
  sb.U -= g.gm1 * s.rho * s.U * sb.p;
  sb.V -= g.gm1 * s.rho * s.V * sb.p;
  sb.W -= g.gm1 * s.rho * s.W * sb.p;
  // U = dQ1 / rho, V = dQ2 / rho, W = dQ3 / rho
  const double ir = 1.0 / s.rho;
  dQb[1] += sb.U * ir;
  dQb[2] += sb.V * ir;
  dQb[3] += sb.W * ir;
  sb.rho -= (sb.U * s.U + sb.V * s.V + sb.W * s.W) * ir;
  // rho = rho_ref + dQ0
  dQb[0] += sb.rho;
  (void)dQ;
}

// All 60 cotangents Xb (overwritten) of the Gauss-point flux with inputs X (the
// layout of zgp_flux) from those of F^n (Fb) and dF^n/dt (dFb).
template <bool VAR_MU>
__host__ __device__ __forceinline__ void zflux_vjp(const Geo& g, const double* X, double dt, const double* Fb,
                                                   const double* dFb, double* Xb, int iQ0, int iQl, int iQr, int iD0,
                                                   int iDl, int iDr) {
  const double K = g.K;
  // forward
  ZCoef<double> c;
  zflux_begin<VAR_MU>(g, X + iQ0, X + iQl, X + iQr, dt, c);
  const ZPrim<double>* sp[3] = {&c.s0, &c.sl, &c.sr};
  const int iQ[3] = {iQ0, iQl, iQr};
  const int iD[3] = {iD0, iDl, iDr};
  double R[3][6][5];
#pragma unroll 1
  for (int side = 0; side < 3; ++side)
    zside_rows(*sp[side], reinterpret_cast<const double(*)[5]>(X + iD[side]), side == 0 ? 0 : (side == 1 ? +1 : -1),
               K, R[side]);
  double J1[5], Jh[5], I1[5], Ih[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) J1[k] = Jh[k] = I1[k] = Ih[k] = 0.0;
#pragma unroll 1
  for (int side = 0; side < 3; ++side) {
    const double* k1 = side == 0 ? c.eq1 : c.in1;
    const double* kh = side == 0 ? c.eqh : c.inh;
    const double rho = sp[side]->rho;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      J1[k] += rho * (k1[0] * R[side][0][k] + k1[1] * R[side][1][k] + k1[2] * R[side][2][k]);
      Jh[k] += rho * (kh[0] * R[side][0][k] + kh[1] * R[side][1][k] + kh[2] * R[side][2][k]);
      I1[k] += rho * (k1[0] * R[side][3][k] + k1[1] * R[side][4][k] + k1[2] * R[side][5][k]);
      Ih[k] += rho * (kh[0] * R[side][3][k] + kh[1] * R[side][4][k] + kh[2] * R[side][5][k]);
    }
  }
  // reverse of the end formulas: F = (4 Ih - I1)/dt, dF = 4 (I1 - 2 Ih)/dt^2 after
  // I[4] += fix h(I, J; U0), h(G1, G0) = hv(G1) - U0 hv(G0), hv(G) = G4 - U0.G(1:3) + |U0|^2/2 G0
  const double idt = 1.0 / dt;
  double I1b[5], Ihb[5], J1b[5], Jhb[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    I1b[k] = -Fb[k] * idt + 4.0 * dFb[k] * idt * idt;
    Ihb[k] = 4.0 * Fb[k] * idt - 8.0 * dFb[k] * idt * idt;
  }
  ZPrimB sb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) sb[i] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  {
    const double U0 = c.s0.U, V0 = c.s0.V, W0 = c.s0.W;
    const double k0 = 0.5 * (U0 * U0 + V0 * V0 + W0 * W0);
    const double hg[5] = {k0, -U0, -V0, -W0, 1.0};
    const double fix = g.pr_fix;
    const double* Is[2] = {I1, Ih};
    const double* Js[2] = {J1, Jh};
    double* Ibs[2] = {I1b, Ihb};
    double* Jbs[2] = {J1b, Jhb};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double* I = Is[h];
      const double* J = Js[h];
      const double q = fix * Ibs[h][4];
      const double hvJ = J[4] - (U0 * J[1] + V0 * J[2] + W0 * J[3]) + k0 * J[0];
      // d h / d (U0, V0, W0)
      sb[0].U += q * ((-I[1] + U0 * I[0]) - hvJ - U0 * (-J[1] + U0 * J[0]));
      sb[0].V += q * ((-I[2] + V0 * I[0]) - U0 * (-J[2] + V0 * J[0]));
      sb[0].W += q * ((-I[3] + W0 * I[0]) - U0 * (-J[3] + W0 * J[0]));
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        Jbs[h][k] = -U0 * q * hg[k];
        Ibs[h][k] += q * hg[k];
      }
    }
  }
  // reverse of the accumulation and of each side's rows
  double eq1b[3] = {0.0, 0.0, 0.0}, eqhb[3] = {0.0, 0.0, 0.0}, in1b[3] = {0.0, 0.0, 0.0}, inhb[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
  for (int side = 0; side < 3; ++side) {
    const double* k1 = side == 0 ? c.eq1 : c.in1;
    const double* kh = side == 0 ? c.eqh : c.inh;
    double* k1b = side == 0 ? eq1b : in1b;
    double* khb = side == 0 ? eqhb : inhb;
    const double rho = sp[side]->rho;
    double Rb[6][5];
    double rhob = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s1 = 0.0, sh = 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        Rb[j][k] = rho * (k1[j] * J1b[k] + kh[j] * Jhb[k]);
        Rb[3 + j][k] = rho * (k1[j] * I1b[k] + kh[j] * Ihb[k]);
        s1 += J1b[k] * R[side][j][k] + I1b[k] * R[side][3 + j][k];
        sh += Jhb[k] * R[side][j][k] + Ihb[k] * R[side][3 + j][k];
      }
      k1b[j] += rho * s1;
      khb[j] += rho * sh;
      rhob += k1[j] * s1 + kh[j] * sh;
    }
    sb[side].rho += rhob;
    double Db[3][5];
    zside_rows_rev(*sp[side], reinterpret_cast<const double(*)[5]>(X + iD[side]),
                   side == 0 ? 0 : (side == 1 ? +1 : -1), K, Rb, sb[side], Db);
#pragma unroll
    for (int i = 0; i < 15; ++i) Xb[iD[side] + i] = Db[i / 5][i % 5];
  }
  // reverse of the time-integral coefficients and the collision time
  //   tau = mu(T0) / p0 + c_art |p_l - p_r| / (p_l + p_r) dt,  mu(T0) = mu_ref (T0 / T_ref)^omega
  {
    const double p0 = c.s0.p, rho0 = c.s0.rho;
    double mu = g.mu_ref;
    if (VAR_MU) mu = mu * pow(p0 / rho0 / g.T_ref, g.mu_exp);
    const double pl = c.sl.p, pr = c.sr.p, ps = pl + pr;
    const double r = (pl - pr) / ps;
    const double tau = mu / p0 + g.c_art * fabs(r) * dt;
    const double taub = ztime_rev(dt, tau, eq1b, in1b) + ztime_rev(0.5 * dt, tau, eqhb, inhb);
    const double om = VAR_MU ? g.mu_exp : 0.0;
    sb[0].p += taub * (om - 1.0) * mu / (p0 * p0);
    sb[0].rho -= taub * om * mu / (rho0 * p0);
    const double sg = r >= 0.0 ? 1.0 : -1.0;  // d|x|/dx at 0 taken as +1, as the tangents do
    const double ab = taub * g.c_art * dt * sg;
    sb[1].p += ab * 2.0 * pr / (ps * ps);
    sb[2].p -= ab * 2.0 * pl / (ps * ps);
  }
  // reverse of the primitive states
#pragma unroll
  for (int i = 0; i < 15; ++i) Xb[i < 5 ? iQ0 + i : (i < 10 ? iQl + i - 5 : iQr + i - 10)] = 0.0;
#pragma unroll 1
  for (int side = 0; side < 3; ++side) zprim_rev(g, X + iQ[side], *sp[side], sb[side], Xb + iQ[side]);
}

}  // namespace hgks
