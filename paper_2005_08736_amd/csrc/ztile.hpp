// Face-field tile of the WENO-Z / full-flux mode (mode Z): the tile geometry and
// the three reconstruction stages shared by the forward kernel and its adjoint.
//   zface_field: per face-field entry, the WENO-Z values and slopes Q_l, Q_r,
//     dQ_l/dn, dQ_r/dn from the six cells along the normal, Q0 by the
//     compatibility condition and dQ0/dn (Sec. 2.1): 30 fields;
//   zrow_edges: WENO-Z edge values along t1 of every five-entry t1 line centred
//     on a tile column;
//   zgp_field: one field's value and tangential derivatives at a Gauss point
//     (parabola through each line's average and edges, then WENO-Z across the
//     five lines in t2 and a second parabola).
#pragma once

#include "flux_tile.hpp"
#include "zflux.hpp"

namespace hgks {

template <int DIR>
struct ZTileGeom {
  static constexpr int A1 = (DIR + 1) % 3, A2 = (DIR + 2) % 3;  // t1, t2 axes
  static constexpr int B = 8;                                   // faces per tangential axis
  static constexpr int P = B + 4;                               // with the halo
  static constexpr int NFF = P * P;                             // face-field entries (t1 fastest)
  static constexpr int NROW = B * P;                            // t1 lines (t1 in the tile, t2 with halo)
  static constexpr int NF = 30;                                 // fields per entry
};

// Tile order.  x-faces: the normal axis fastest (neighbouring tiles along the
// normal share five of their six stencil planes).  y- and z-faces: the x tiles
// first, then the normal, then the remaining axis, so that the tiles resident on
// one XCD cover a few planes of a slab of rows whole in x.
template <int DIR>
__device__ __forceinline__ void zflux_tile_origin(int tile, int Nn, int nt1, int nt2, int& on, int& o1, int& o2) {
  using TG = ZTileGeom<DIR>;
  if (DIR == 0) {
    on = tile % Nn;
    o1 = ((tile / Nn) % nt1) * TG::B;
    o2 = (tile / (Nn * nt1)) * TG::B;
  } else if (DIR == 1) {  // t1 = z, t2 = x
    o2 = (tile % nt2) * TG::B;
    on = (tile / nt2) % Nn;
    o1 = (tile / (nt2 * Nn)) * TG::B;
  } else {  // t1 = x, t2 = y
    o1 = (tile % nt1) * TG::B;
    on = (tile / nt1) % Nn;
    o2 = (tile / (nt1 * Nn)) * TG::B;
  }
}

// field numbering in LDS
constexpr int kZQ0 = 0, kZDn = 5, kZQl = 10, kZQr = 15, kZDl = 20, kZDr = 25;

template <typename T, int DIR>
__device__ __forceinline__ void zface_field(const Geo& g, const double* __restrict__ q, T* ff, int on, int o1, int o2) {
  using TG = ZTileGeom<DIR>;
  const T ih = T(g.inv_h[DIR]);
  const T ih12 = T(g.inv_h[DIR] * (1.0 / 12.0));
  const T eps = T(g.weno_eps);
  for (int e = threadIdx.x; e < TG::NFF; e += 256) {
    const int i1 = e % TG::P, i2 = e / TG::P;
    int c[3];
    c[DIR] = on;
    c[TG::A1] = wrap_coord(o1 + i1 - 2, g.n[TG::A1]);
    c[TG::A2] = wrap_coord(o2 + i2 - 2, g.n[TG::A2]);
    const int Nn = g.n[DIR];
    const long long sn = g.stride[DIR];
    const long long base = (long long)c[0] + (long long)c[1] * g.stride[1] + (long long)c[2] * g.stride[2] -
                           (long long)on * sn;
    T Ql[5], Qr[5], Dl[5], Dr[5], Dn[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double* f = q + (long long)gcomp_local<DIR>(k) * g.N;
      const double ref = k == 0 ? g.rho_ref : (k == 4 ? g.E_ref : 0.0);
      T v[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) v[m] = T(f[base + (long long)wrapi(on - 2 + m, Nn) * sn] - ref);
      T sl, sr;
      weno_z_right(v, eps, g.weno_p, Ql[k], sl);
      T rv[5] = {v[5], v[4], v[3], v[2], v[1]};
      weno_z_right(rv, eps, g.weno_p, Qr[k], sr);
      Dl[k] = sl * ih;
      Dr[k] = -sr * ih;
      Dn[k] = (v[1] - T(15) * v[2] + T(15) * v[3] - v[4]) * ih12;
    }
    T Q0[5];
    compat_dev(g, Ql, Qr, Q0);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      ff[(kZQ0 + k) * TG::NFF + e] = Q0[k];
      ff[(kZDn + k) * TG::NFF + e] = Dn[k];
      ff[(kZQl + k) * TG::NFF + e] = Ql[k];
      ff[(kZQr + k) * TG::NFF + e] = Qr[k];
      ff[(kZDl + k) * TG::NFF + e] = Dl[k];
      ff[(kZDr + k) * TG::NFF + e] = Dr[k];
    }
  }
}

// Phase 2: WENO-Z edge values along t1 of line (a, i2): the five entries
// (a .. a+4, i2) of the patch, centred on entry (a+2, i2).
template <typename T, int DIR>
__device__ __forceinline__ void zrow_edges(const Geo& g, const T* ff, T* ed) {
  using TG = ZTileGeom<DIR>;
  const T eps = T(g.weno_eps);
  for (int it = threadIdx.x; it < TG::NF * TG::NROW; it += 256) {
    const int f = it / TG::NROW, r = it % TG::NROW;
    const int a = r % TG::B, i2 = r / TG::B;
    const T* src = ff + f * TG::NFF + i2 * TG::P + a;
    T line[5];
#pragma unroll
    for (int s = 0; s < 5; ++s) line[s] = src[s];
    T ea, eb;
    weno_z_edges(line, eps, g.weno_p, ea, eb);
    ed[2 * (f * TG::NROW + r)] = ea;
    ed[2 * (f * TG::NROW + r) + 1] = eb;
  }
}

// Phase 3 helper: the field's value (and t2-derivative, and optionally the
// t1-derivative) at Gauss point (sm, sl) of the face at tile position (a, t).
template <typename T, int DIR, bool T1DER>
__device__ __forceinline__ void zgp_field(const Geo& g, const T* ff, const T* ed, int f, int a, int t, T sm, T sl,
                                          T& val, T& d1, T& d2, T& token) {
  using TG = ZTileGeom<DIR>;
  const T eps = T(g.weno_eps);
  // one field at a time: the reads wait for the previous field's result, so the
  // scheduler cannot interleave the fields and hold all their temporaries at once
  zdep(a, token);
  T rv[5], rd[5];
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    const T m = ff[f * TG::NFF + (t + r) * TG::P + a + 2];
    const int li = f * TG::NROW + (t + r) * TG::B + a;
    const T ea = ed[2 * li], eb = ed[2 * li + 1];
    rv[r] = zpar_val(m, ea, eb, sm);
    if (T1DER) rd[r] = zpar_der(m, ea, eb, sm);
  }
  T ea, eb;
  weno_z_edges(rv, eps, g.weno_p, ea, eb);
  val = zpar_val(rv[2], ea, eb, sl);
  d2 = zpar_der(rv[2], ea, eb, sl) * T(g.inv_h[TG::A2]);
  if (T1DER) {
    weno_z_edges(rd, eps, g.weno_p, ea, eb);
    d1 = zpar_val(rd[2], ea, eb, sl) * T(g.inv_h[TG::A1]);
    token = d1;
  } else {
    token = val;
  }
}

// Phase 3 helper for two reconstructions at once, shared by the two Gauss points
// of a face with the same t1 point (adjacent lanes, sl = -1 and +1): the WENO-Z
// edge pair across the five lines does not depend on sl, so the lane with
// sl = -1 evaluates it for job A, the lane with sl = +1 for job B, and the two
// exchange their edges.  Job A is the value rows of field fA (value and
// t2-derivative out); job B the value rows of field fB (DB = false: value and
// t2-derivative out) or its t1-derivative rows (DB = true: t1-derivative out in
// outB).  Every lane of the workgroup must take part.
template <typename T, int DIR, bool DB>
__device__ __forceinline__ void zgp_pair(const Geo& g, const T* ff, const T* ed, int fA, int fB, int a, int t, T sm,
                                         T sl, T& valA, T& d2A, T& outB, T& outB2, T& token) {
  using TG = ZTileGeom<DIR>;
  const T eps = T(g.weno_eps);
  zdep(a, token);
  const bool mineB = sl > T(0);
  const int f = mineB ? fB : fA;
  // rows as c_m m + c_d (eb - ea) + c_s (ea + eb - 2 m): value rows (1, sm G, 0),
  // t1-derivative rows (0, 1, sm sqrt 3)
  const bool der = DB && mineB;
  const T c_m = der ? T(0) : T(1);
  const T c_d = der ? T(1) : sm * T(kGauss);
  const T c_s = der ? sm * T(kS3) : T(0);
  T row[5];
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    const T m = ff[f * TG::NFF + (t + r) * TG::P + a + 2];
    const int li = f * TG::NROW + (t + r) * TG::B + a;
    const T ea = ed[2 * li], eb = ed[2 * li + 1];
    row[r] = c_m * m + c_d * (eb - ea) + c_s * (ea + eb - T(2) * m);
  }
  T ea, eb;
  weno_z_edges(row, eps, g.weno_p, ea, eb);
  const T pa = __shfl_xor(ea, 1), pb = __shfl_xor(eb, 1);
  const T eaA = mineB ? pa : ea, ebA = mineB ? pb : eb;
  const T eaB = mineB ? ea : pa, ebB = mineB ? eb : pb;
  // middle rows of both jobs
  T midA, midB;
  {
    const T m = ff[fA * TG::NFF + (t + 2) * TG::P + a + 2];
    const int li = fA * TG::NROW + (t + 2) * TG::B + a;
    midA = zpar_val(m, ed[2 * li], ed[2 * li + 1], sm);
  }
  {
    const T m = ff[fB * TG::NFF + (t + 2) * TG::P + a + 2];
    const int li = fB * TG::NROW + (t + 2) * TG::B + a;
    midB = DB ? zpar_der(m, ed[2 * li], ed[2 * li + 1], sm) : zpar_val(m, ed[2 * li], ed[2 * li + 1], sm);
  }
  valA = zpar_val(midA, eaA, ebA, sl);
  d2A = zpar_der(midA, eaA, ebA, sl) * T(g.inv_h[TG::A2]);
  if (DB) {
    outB = zpar_val(midB, eaB, ebB, sl) * T(g.inv_h[TG::A1]);
    outB2 = T(0);
  } else {
    outB = zpar_val(midB, eaB, ebB, sl);
    outB2 = zpar_der(midB, eaB, ebB, sl) * T(g.inv_h[TG::A2]);
  }
  token = outB;
}

}  // namespace hgks
