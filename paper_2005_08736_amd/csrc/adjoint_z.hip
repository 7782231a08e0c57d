// Adjoint (vector-Jacobian product) of the mode-Z face fluxes of one direction:
// WENO-Z reconstruction with its smooth nonlinear weights (p = 2 in the Z
// ratios), the compatibility state and the full gas distribution of Eq. (flux)
// integrated over dt and dt/2, with the time step frozen.
//
// For cotangents mu_L, mu_dL on the cells, the cotangent of a face-averaged flux
// is (mu(i+1) - mu(i)) / h_d, a quarter of it per Gauss point.  One workgroup owns
// the forward kernel's 8 x 8 tile and
//   A. recomputes the face field and the t1 edge values of the tile and its halo
//      into LDS (the forward arithmetic, ztile.hpp);
//   B. per Gauss point: recomputes the 60 reconstructed values the flux takes,
//      takes the point's cotangent back through the Gauss-point flux with the
//      hand-written reverse sweep (zreverse.hpp), then transposes the
//      tangential reconstruction of each of the 30 fields (parabolas and WENO-Z
//      edge pairs, reversed by hand as well) into an LDS face-field cotangent
//      (LDS atomics);
//   C. per face-field entry: reverses the compatibility state (by hand,
//      adjoint_common.hpp) and the normal WENO-Z values and slopes (by hand,
//      zreverse.hpp), and adds the six cells' cotangents into lambda (device
//      atomics).
// Mixing the two cotangent sources mu = cA * A + cB * B inside the kernel lets one
// launch per direction serve both stages of the step adjoint.  This path is
// exact but not tuned: it is meant for the small boxes on which the mode-Z
// gradient is checked.
#include "adjoint_common.hpp"
#include "internal.hpp"
#include "zadjoint_common.hpp"
#include "ztile.hpp"

namespace hgks {

// The flux's vector-Jacobian product at one Gauss point (the hand-written
// reverse of zreverse.hpp), kept out of line: one copy serves the three face
// directions.
template <bool VAR_MU>
__device__ __noinline__ void zflux_vjp_pass(const Geo& g, const double* X, double dt, const double* Fb,
                                            const double* dFb, double* Xb) {
  zflux_vjp<VAR_MU>(g, X, dt, Fb, dFb, Xb, kXQ0, kXQl, kXQr, kXD0, kXDl, kXDr);
}

// Transpose of zgp_field for field f at Gauss point (sm, sl) of the face at tile
// position (a, t): cotangents vb of the value, d2b of the t2-derivative and d1b of
// the t1-derivative (T1DER) go to the 5 x 5 entries of the field in ffb.
template <int DIR, bool T1DER>
__device__ __forceinline__ void zgp_field_vjp(const Geo& g, const double* ff, const double* ed, double* ffb, int f,
                                              int a, int t, double sm, double sl, double vb, double d2b, double d1b) {
  using TG = ZTileGeom<DIR>;
  const double eps = g.weno_eps;
  const int p = g.weno_p;
  const double ih1 = g.inv_h[TG::A1], ih2 = g.inv_h[TG::A2];
  const double G = kGauss, S3 = kS3;
  double rv[5], rd[5];
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    const double m = ff[f * TG::NFF + (t + r) * TG::P + a + 2];
    const int li = f * TG::NROW + (t + r) * TG::B + a;
    const double ea = ed[2 * li], eb = ed[2 * li + 1];
    rv[r] = zpar_val(m, ea, eb, sm);
    rd[r] = zpar_der(m, ea, eb, sm);
  }
  double rvb[5] = {0, 0, 0, 0, 0}, rdb[5] = {0, 0, 0, 0, 0};
  {
    // val = rv2 + sl (B - A) G ;  d2 = ih2 ((B - A) + sl S3 (A + B - 2 rv2)),  (A, B) = edges(rv)
    const double Ab = -sl * G * vb + ih2 * d2b * (sl * S3 - 1.0);
    const double Bb = sl * G * vb + ih2 * d2b * (sl * S3 + 1.0);
    rvb[2] += vb - 2.0 * sl * S3 * ih2 * d2b;
    weno_z_edges_vjp(rv, eps, p, Ab, Bb, rvb);
  }
  if (T1DER) {
    // d1 = ih1 (rd2 + sl (B' - A') G),  (A', B') = edges(rd)
    const double Ab = -sl * G * ih1 * d1b, Bb = sl * G * ih1 * d1b;
    rdb[2] += ih1 * d1b;
    weno_z_edges_vjp(rd, eps, p, Ab, Bb, rdb);
  }
  // line r: rv = m + sm (eb - ea) G ;  rd = (eb - ea) + sm S3 (ea + eb - 2 m),  (ea, eb) = edges(line)
#pragma unroll 1
  for (int r = 0; r < 5; ++r) {
    const double eab = -sm * G * rvb[r] + rdb[r] * (sm * S3 - 1.0);
    const double ebb = sm * G * rvb[r] + rdb[r] * (sm * S3 + 1.0);
    const double mb = rvb[r] - 2.0 * sm * S3 * rdb[r];
    double* dst = ffb + f * TG::NFF + (t + r) * TG::P + a;
    const double* src = ff + f * TG::NFF + (t + r) * TG::P + a;
    double line[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) line[i] = src[i];
    double lb[5] = {0.0, 0.0, mb, 0.0, 0.0};
    weno_z_edges_vjp(line, eps, p, eab, ebb, lb);
#pragma unroll
    for (int i = 0; i < 5; ++i) lds_add(dst + i, lb[i]);
  }
}

template <int DIR, bool VAR_MU>
__global__ void __launch_bounds__(256) flux_z_vjp_kernel(Geo g, const double* __restrict__ q,
                                                         const double* __restrict__ A, const double* __restrict__ B,
                                                         double cLA, double cLB, double cDA, double cDB,
                                                         const double* __restrict__ dtp, double* __restrict__ lam,
                                                         int nt1, int nt2, int nper) {
  using TG = ZTileGeom<DIR>;
  __shared__ double ff[TG::NF * TG::NFF];
  __shared__ double ed[2 * TG::NF * TG::NROW];
  __shared__ double ffb[TG::NF * TG::NFF];
  const int tile = tile_of_block(nper);
  const int Nn = g.n[DIR];
  if (tile >= Nn * nt1 * nt2) return;  // whole workgroup leaves together
  const int on = tile % Nn;
  const int o1 = ((tile / Nn) % nt1) * TG::B;
  const int o2 = (tile / (Nn * nt1)) * TG::B;
  const int tid = threadIdx.x;

  // ---- A: forward recompute
  zface_field<double, DIR>(g, q, ff, on, o1, o2);
  for (int e = tid; e < TG::NF * TG::NFF; e += 256) ffb[e] = 0.0;
  __syncthreads();
  zrow_edges<double, DIR>(g, ff, ed);
  __syncthreads();

  // ---- B: per Gauss point
  {
    const int face = tid >> 2, gp = tid & 3;
    const int a = face % TG::B, t = face / TG::B;
    int cc[3];
    cc[DIR] = on;
    cc[TG::A1] = o1 + a;
    cc[TG::A2] = o2 + t;
    if (cc[TG::A1] < g.n[TG::A1] && cc[TG::A2] < g.n[TG::A2]) {
      const double sm = (gp & 2) ? 1.0 : -1.0;  // t1 Gauss point
      const double sl = (gp & 1) ? 1.0 : -1.0;  // t2 Gauss point
      const double dt = *dtp;
      // cotangent of this Gauss point's F and dF/dt (local frame)
      const long long idx = (long long)cc[0] + (long long)cc[1] * g.stride[1] + (long long)cc[2] * g.stride[2];
      const long long up = on == Nn - 1 ? idx - (long long)(Nn - 1) * g.stride[DIR] : idx + g.stride[DIR];
      double Fb[5], dFb[5];
      const double w = 0.25 * g.inv_h[DIR];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const long long o = (long long)gcomp_local<DIR>(k) * g.N;
        const double da = A[o + up] - A[o + idx];
        const double db = B ? B[o + up] - B[o + idx] : 0.0;
        Fb[k] = w * (cLA * da + cLB * db);
        dFb[k] = w * (cDA * da + cDB * db);
      }
      // the 60 flux inputs
      double X[kXN];
      double tok = 0.0, dum;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        zgp_field<double, DIR, true>(g, ff, ed, kZQ0 + k, a, t, sm, sl, X[kXQ0 + k], X[kXD0 + 5 + k],
                                     X[kXD0 + 10 + k], tok);
        zgp_field<double, DIR, true>(g, ff, ed, kZQl + k, a, t, sm, sl, X[kXQl + k], X[kXDl + 5 + k],
                                     X[kXDl + 10 + k], tok);
        zgp_field<double, DIR, true>(g, ff, ed, kZQr + k, a, t, sm, sl, X[kXQr + k], X[kXDr + 5 + k],
                                     X[kXDr + 10 + k], tok);
        zgp_field<double, DIR, false>(g, ff, ed, kZDn + k, a, t, sm, sl, X[kXD0 + k], dum, dum, tok);
        zgp_field<double, DIR, false>(g, ff, ed, kZDl + k, a, t, sm, sl, X[kXDl + k], dum, dum, tok);
        zgp_field<double, DIR, false>(g, ff, ed, kZDr + k, a, t, sm, sl, X[kXDr + k], dum, dum, tok);
      }
      // input cotangents Xb = J^T (Fb, dFb) by the reverse sweep
      double Xb[kXN];
      zflux_vjp_pass<VAR_MU>(g, X, dt, Fb, dFb, Xb);
      // transpose of the tangential reconstruction, field by field
#pragma unroll 1
      for (int k = 0; k < 5; ++k) {
        zgp_field_vjp<DIR, true>(g, ff, ed, ffb, kZQ0 + k, a, t, sm, sl, Xb[kXQ0 + k], Xb[kXD0 + 10 + k],
                                 Xb[kXD0 + 5 + k]);
        zgp_field_vjp<DIR, true>(g, ff, ed, ffb, kZQl + k, a, t, sm, sl, Xb[kXQl + k], Xb[kXDl + 10 + k],
                                 Xb[kXDl + 5 + k]);
        zgp_field_vjp<DIR, true>(g, ff, ed, ffb, kZQr + k, a, t, sm, sl, Xb[kXQr + k], Xb[kXDr + 10 + k],
                                 Xb[kXDr + 5 + k]);
        zgp_field_vjp<DIR, false>(g, ff, ed, ffb, kZDn + k, a, t, sm, sl, Xb[kXD0 + k], 0.0, 0.0);
        zgp_field_vjp<DIR, false>(g, ff, ed, ffb, kZDl + k, a, t, sm, sl, Xb[kXDl + k], 0.0, 0.0);
        zgp_field_vjp<DIR, false>(g, ff, ed, ffb, kZDr + k, a, t, sm, sl, Xb[kXDr + k], 0.0, 0.0);
      }
    }
  }
  __syncthreads();

  // ---- C: per face-field entry (tile and halo), reverse of zface_field
  const double ih = g.inv_h[DIR], ih12 = g.inv_h[DIR] * (1.0 / 12.0);
  const double eps = g.weno_eps;
  for (int e = tid; e < TG::NFF; e += 256) {
    const int i1 = e % TG::P, i2 = e / TG::P;
    int c[3];
    c[DIR] = on;
    c[TG::A1] = wrap_coord(o1 + i1 - 2, g.n[TG::A1]);
    c[TG::A2] = wrap_coord(o2 + i2 - 2, g.n[TG::A2]);
    const long long sn = g.stride[DIR];
    const long long base =
        (long long)c[0] + (long long)c[1] * g.stride[1] + (long long)c[2] * g.stride[2] - (long long)on * sn;
    long long off[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) off[m] = base + (long long)wrapi(on - 2 + m, Nn) * sn;
    double v[5][6], Ql[5], Qr[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double* fq = q + (long long)gcomp_local<DIR>(k) * g.N;
      const double ref = k == 0 ? g.rho_ref : (k == 4 ? g.E_ref : 0.0);
#pragma unroll
      for (int m = 0; m < 6; ++m) v[k][m] = fq[off[m]] - ref;
      double sl, sr;
      weno_z_right(v[k], eps, g.weno_p, Ql[k], sl);
      const double rv[5] = {v[k][5], v[k][4], v[k][3], v[k][2], v[k][1]};
      weno_z_right(rv, eps, g.weno_p, Qr[k], sr);
    }
    double Q0b[5], Qlb[5], Qrb[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      Q0b[k] = ffb[(kZQ0 + k) * TG::NFF + e];
      Qlb[k] = ffb[(kZQl + k) * TG::NFF + e];
      Qrb[k] = ffb[(kZQr + k) * TG::NFF + e];
    }
    compat_dev_vjp(g, Ql, Qr, Q0b, Qlb, Qrb);
#pragma unroll 1
    for (int k = 0; k < 5; ++k) {
      const double Dnb = ffb[(kZDn + k) * TG::NFF + e];
      const double slb = ffb[(kZDl + k) * TG::NFF + e] * ih;   // D_l = s_l / h
      const double srb = -ffb[(kZDr + k) * TG::NFF + e] * ih;  // D_r = -s_r / h
      double vb[6] = {0, 0, 0, 0, 0, 0};
      weno_z_right_vjp(v[k], eps, g.weno_p, Qlb[k], slb, vb);
      const double rv[5] = {v[k][5], v[k][4], v[k][3], v[k][2], v[k][1]};
      double rvb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      weno_z_right_vjp(rv, eps, g.weno_p, Qrb[k], srb, rvb);
#pragma unroll
      for (int i = 0; i < 5; ++i) vb[5 - i] += rvb[i];
      // D_n = (v1 - 15 v2 + 15 v3 - v4) / (12 h)
      vb[1] += ih12 * Dnb;
      vb[2] -= 15.0 * ih12 * Dnb;
      vb[3] += 15.0 * ih12 * Dnb;
      vb[4] -= ih12 * Dnb;
      double* lk = lam + (long long)gcomp_local<DIR>(k) * g.N;
#pragma unroll
      for (int m = 0; m < 6; ++m) global_add(lk + off[m], vb[m]);
    }
  }
}

template <int DIR, bool VAR_MU>
static void launch_z_vjp_dir(const Geo& g, const double* q, const double* A, const double* B, double cLA, double cLB,
                             double cDA, double cDB, const double* dtp, double* lam, hipStream_t st) {
  using TG = ZTileGeom<DIR>;
  const int nt1 = (g.n[TG::A1] + TG::B - 1) / TG::B;
  const int nt2 = (g.n[TG::A2] + TG::B - 1) / TG::B;
  const int tiles = g.n[DIR] * nt1 * nt2;
  const int nper = (tiles + 7) / 8;
  flux_z_vjp_kernel<DIR, VAR_MU><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, A, B, cLA, cLB, cDA, cDB, dtp,
                                                                                 lam, nt1, nt2, nper);
}

// lam += (dL/dQ)^T mu_L + (ddL/dQ)^T mu_dL of the mode-Z operator at state q for
// the faces of direction dir, with mu_L = cLA A + cLB B and mu_dL = cDA A + cDB B
// (B may be null); *dtp is the frozen time step the fluxes integrate over.
void launch_operator_vjp_z(const Geo& g, int dir, const double* q, const double* A, const double* B, double cLA,
                           double cLB, double cDA, double cDB, const double* dtp, double* lam, hipStream_t st) {
  if (g.mu_exp != 0.0) {
    if (dir == 0) launch_z_vjp_dir<0, true>(g, q, A, B, cLA, cLB, cDA, cDB, dtp, lam, st);
    else if (dir == 1) launch_z_vjp_dir<1, true>(g, q, A, B, cLA, cLB, cDA, cDB, dtp, lam, st);
    else launch_z_vjp_dir<2, true>(g, q, A, B, cLA, cLB, cDA, cDB, dtp, lam, st);
  } else {
    if (dir == 0) launch_z_vjp_dir<0, false>(g, q, A, B, cLA, cLB, cDA, cDB, dtp, lam, st);
    else if (dir == 1) launch_z_vjp_dir<1, false>(g, q, A, B, cLA, cLB, cDA, cDB, dtp, lam, st);
    else launch_z_vjp_dir<2, false>(g, q, A, B, cLA, cLB, cDA, cDB, dtp, lam, st);
  }
}

}  // namespace hgks
