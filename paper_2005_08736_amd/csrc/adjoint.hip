// Adjoint (vector-Jacobian product) of the HGKS operator and of the two-stage
// step, hand-written for gfx950.
//
// Operator: L_i = -sum_d (F_d(i+1/2) - F_d(i-1/2)) / h_d and the same for dL with
// dF (Eq. (finite)).  For cotangents mu_L, mu_dL on the cells, the cotangent of
// a face flux is (mu(i+1) - mu(i)) / h_d.  flux_vjp_kernel works on the same
// tiles as the forward kernel:
//   1. recompute the face field of the tile and halo into LDS (exactly the
//      forward arithmetic, flux_tile.hpp);
//   2. per face: recompute the Gauss-point data, run the reverse of the
//      gas-kinetic flux at each Gauss point (adjoint_common.hpp) and transpose the
//      tangential reconstruction, adding the face-field cotangents of the 5 x 5
//      neighbourhood into an LDS tile (LDS atomics);
//   3. y- and z-faces: add the tile's face-field cotangents (its own faces and the
//      halo's) into a global face array G (global atomics), where the
//      contributions of the tiles that share a face meet.  x-faces: per entry,
//      reverse the compatibility state and gather the normal-reconstruction
//      transpose per cell of the tile's footprint, adding into lambda with one
//      global atomic per cell and component.
// For y- and z-faces face_field_vjp_kernel then takes each face once: it reads and
// clears G, reverses the compatibility state and the normal reconstruction, and
// gathers the cell cotangents along the normal in LDS; the cells whose six faces
// all lie in the workgroup are written directly, only those at the ends of its
// run of faces by atomic adds.  That replaces 50 atomic adds per face by about
// 20, and the compatibility reverse of the tile halo (1.69 evaluations per face)
// by one.  Mixing the two cotangent sources mu = cA * A + cB * B inside the
// kernel lets one launch (pair) per direction serve both stages of the step
// adjoint.
#include "adjoint_common.hpp"
#include "flux_tile.hpp"
#include "internal.hpp"

namespace hgks {

// Tiles of the adjoint kernels: as the forward ones, except x-faces, whose
// forward 4 x 8 x 8 tile would need 92 KB of LDS here (face field and its
// cotangent) and leave one block per CU; 2 x 16 x 8 needs 77 KB (two blocks).
template <int DIR> struct AdjTile { static constexpr int B[3] = {FluxTile<DIR>::B[0], FluxTile<DIR>::B[1], FluxTile<DIR>::B[2]}; };
template <> struct AdjTile<0> { static constexpr int B[3] = {2, 16, 8}; };
template <int DIR>
using AdjGeom = TileGeomB<DIR, AdjTile<DIR>::B[0], AdjTile<DIR>::B[1], AdjTile<DIR>::B[2]>;

// Tile order of the adjoint.  y- and z-face tiles are numbered with the normal
// axis slowest, so that the tiles whose footprints share cells along the normal
// run far apart in time and their atomic adds into lambda do not contend (z-faces
// 11% faster, y-faces 4%).  x-face tiles keep the forward order, normal axis
// fastest: there the L2 reuse of the shared x-stencil matters more (the other
// order made them 20-45% slower).
template <int DIR, class TG>
__device__ __forceinline__ void adj_tile_origin(int tile, int ntx, int nty, int ntz, int& x0, int& y0, int& z0) {
  if (DIR == 0) {
    tile_origin<DIR, TG>(tile, ntx, nty, ntz, x0, y0, z0);
    return;
  }
  const int nt1 = ntx, nt2 = DIR == 1 ? ntz : nty;  // tangential tile counts (x first)
  const int a = tile % nt1, r = tile / nt1, b = r % nt2, n = r / nt2;
  x0 = a * TG::BX;
  if (DIR == 1) {
    y0 = n * TG::BY;
    z0 = b * TG::BZ;
  } else {
    y0 = b * TG::BY;
    z0 = n * TG::BZ;
  }
}

// T is the arithmetic of the recomputed forward and of its reverse (double, or
// float for the FP32-flux form); the cotangents A, B and lambda stay in double.
template <typename T, int DIR, bool NEED_F>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) flux_vjp_kernel(Geo g, const double* __restrict__ q,
                                                       const double* __restrict__ A, const double* __restrict__ B,
                                                       double cLA, double cLB, double cDA, double cDB,
                                                       double* __restrict__ G, double* __restrict__ lam, int ntx,
                                                       int nty, int ntz, int nper) {
  using TG = AdjGeom<DIR>;
  __shared__ T ff[10 * TG::NFF];
  // the cotangent tile accumulates in double in both forms: LDS atomic adds of
  // FP32 stalled the FP32 kernel on LDS waits five times over the FP64 one
  __shared__ double ffb[10 * TG::NFF];
  const int tile = tile_of_block(nper);
  if (tile >= ntx * nty * ntz) return;
  int x0, y0, z0;
  adj_tile_origin<DIR, TG>(tile, ntx, nty, ntz, x0, y0, z0);
  const int tid = threadIdx.x;

  face_field_tile<T, DIR, false, TG>(g, q, ff, x0, y0, z0, g.inv_h[DIR]);
  for (int e = tid; e < 10 * TG::NFF; e += 256) ffb[e] = 0.0;
  __syncthreads();

  // ---- phase 2: per face
  {
    const int fx = tid % TG::BX, fy = (tid / TG::BX) % TG::BY, fz = tid / (TG::BX * TG::BY);
    const int gx = x0 + fx, gy = y0 + fy, gz = z0 + fz;
    if (gx < g.n[0] && gy < g.n[1] && gz < g.n[2]) {
      constexpr int A1 = (DIR + 1) % 3, A2 = (DIR + 2) % 3;
      constexpr int s1 = TG::S[A1], s2 = TG::S[A2];
      const int centre = (fx + TG::HX) + (fy + TG::HY) * TG::FX + (fz + TG::HZ) * TG::FX * TG::FY;
      const int corner = centre - 2 * s1 - 2 * s2;
      const T i1 = T(g.inv_h[A1]), i2 = T(g.inv_h[A2]);
      // cotangents of the face average (local frame): (mu(i+1) - mu(i)) / h, then 1/4 per Gauss point
      const long long idx = (long long)gx + (long long)gy * g.stride[1] + (long long)gz * g.stride[2];
      int c[3] = {gx, gy, gz};
      const long long up = c[DIR] == g.n[DIR] - 1 ? idx - (long long)(g.n[DIR] - 1) * g.stride[DIR]
                                                  : idx + g.stride[DIR];
      // (formed in double, then rounded once to T)
      T Fb[5], dFb[5];
      const double w = 0.25 * g.inv_h[DIR];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const long long o = (long long)gcomp_local<DIR>(k) * g.N;
        const double a = A[o + up] - A[o + idx];
        const double b = B ? B[o + up] - B[o + idx] : 0.0;
        Fb[k] = NEED_F ? T(w * (cLA * a + cLB * b)) : T(0);
        dFb[k] = T(w * (cDA * a + cDB * b));
      }
#pragma unroll 1
      for (int m = 0; m < 2; ++m) {
        T Qg[2][5], Dg[2][3][5];
        gp_data<T, DIR, TG>(ff, corner, m, i1, i2, i2, Qg, Dg);
        T Qgb[2][5], Dgb[2][3][5];
#pragma unroll
        for (int l = 0; l < 2; ++l) {
#pragma unroll
          for (int k = 0; k < 5; ++k) {
            Qgb[l][k] = T(0);
            Dgb[l][0][k] = Dgb[l][1][k] = Dgb[l][2][k] = T(0);
          }
          // one Gauss point at a time: the second reverse sweep waits for the first
          if (l == 1) zdep(Qg[1][0], Qgb[0][0]);
          smooth_flux_vjp<NEED_F, false>(g, Qg[l], Dg[l], Fb, dFb, Qgb[l], Dgb[l]);
        }
        // transpose of the tangential reconstruction for this m
        T wvm[5], wdm[5], wv0[5], wd0[5], wv1[5], wd1[5];
        tang_weights(m, wvm, wdm);
        tang_weights(0, wv0, wd0);
        tang_weights(1, wv1, wd1);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          double* f0b = ffb + k * TG::NFF + corner;
          double* fnb = ffb + (5 + k) * TG::NFF + corner;
#pragma unroll
          for (int r = 0; r < 5; ++r) {
            // cotangents of the row values at (m, row r): value, t1-derivative, normal slope
            T rv = wv0[r] * Qgb[0][k] + wv1[r] * Qgb[1][k] + (wd0[r] * Dgb[0][2][k] + wd1[r] * Dgb[1][2][k]) * i2;
            T rd = (wv0[r] * Dgb[0][1][k] + wv1[r] * Dgb[1][1][k]) * i1;
            T rn = wv0[r] * Dgb[0][0][k] + wv1[r] * Dgb[1][0][k];
#pragma unroll
            for (int a = 0; a < 5; ++a) {
              lds_add(f0b + a * s1 + r * s2, double(wvm[a] * rv + wdm[a] * rd));
              lds_add(fnb + a * s1 + r * s2, double(wvm[a] * rn));
            }
          }
        }
      }
    }
  }
  __syncthreads();

  if constexpr (DIR == 0) {
  // x-faces finish in this launch: their face-field cotangents, scattered into G
  // from a 2-face-wide tile, touched a cache line per lane and made the two-launch
  // form slower than this one
  // ---- phase 3a: per face-field entry, reverse of the compatibility state.  The
  // entry's cotangents of the normal reconstruction, l = Q_l-bar/60,
  // r = Q_r-bar/60 and d = D_n-bar/(12 h), go to LDS: l over Q0-bar (ffb fields
  // 0..4), d over D_n-bar (ffb fields 5..9), r into the face field's space, which
  // is not read any more.
  const T ih12 = T(g.inv_h[DIR] * (1.0 / 12.0));
  double* cl = ffb;
  double* cd = ffb + 5 * TG::NFF;
  T* cr = ff;
  for (int e = tid; e < TG::NFF; e += 256) {
    T Q0b[5], Dnb[5];
    bool any = false;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      Q0b[k] = T(ffb[k * TG::NFF + e]);
      Dnb[k] = T(ffb[(5 + k) * TG::NFF + e]);
      any = any || Q0b[k] != T(0) || Dnb[k] != T(0);
    }
    T Qlb[5] = {0, 0, 0, 0, 0}, Qrb[5] = {0, 0, 0, 0, 0};
    if (any) {
      T v[5][6];
      long long off[6];
      normal_stencil<T, DIR, false, TG>(g, q, e, x0, y0, z0, v, off);
      T Ql[5], Qr[5], Dn[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) normal_recon(v[k], ih12, Ql[k], Qr[k], Dn[k]);
      compat_dev_vjp(g, Ql, Qr, Q0b, Qlb, Qrb);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      cl[k * TG::NFF + e] = Qlb[k] * T(1.0 / 60.0);
      cr[k * TG::NFF + e] = Qrb[k] * T(1.0 / 60.0);
      cd[k * TG::NFF + e] = Dnb[k] * ih12;
    }
  }
  __syncthreads();

  // ---- phase 3b: per cell of the tile's footprint (the faces' normal extent plus
  // the five further cells of the six-cell stencil, times the tangential patch),
  // the transpose of the normal reconstruction gathered over the entries whose
  // stencil holds the cell, then one atomic add per component.  The weights of
  // stencil position m = 0..5 (cells n-2 .. n+3 of face n+1/2) are
  //   l (2, -13, 47, 27, -3, 0) + r (0, -3, 27, 47, -13, 2) + d (0, 1, -15, 15, -1, 0).
  constexpr int BN = DIR == 0 ? TG::BX : (DIR == 1 ? TG::BY : TG::BZ);
  constexpr int PX = DIR == 0 ? BN + 5 : TG::FX;
  constexpr int PY = DIR == 1 ? BN + 5 : TG::FY;
  constexpr int PZ = DIR == 2 ? BN + 5 : TG::FZ;
  for (int c = tid; c < PX * PY * PZ; c += 256) {
    const int px = c % PX, py = (c / PX) % PY, pz = c / (PX * PY);
    const int pc[3] = {px, py, pz};
    const int pn = pc[DIR];
    // global cell: the normal axis starts two cells before the tile's first face
    // row, the tangential axes at the patch origin (halo of two)
    const int gc[3] = {wrap_coord(x0 - 2 + px, g.n[0]), wrap_coord(y0 - 2 + py, g.n[1]), wrap_coord(z0 - 2 + pz, g.n[2])};
    const long long cell = (long long)gc[0] + (long long)gc[1] * g.stride[1] + (long long)gc[2] * g.stride[2];
    double acc[5] = {0, 0, 0, 0, 0};
    const int ilo = pn - 5 > 0 ? pn - 5 : 0, ihi = pn < BN - 1 ? pn : BN - 1;
    for (int i = ilo; i <= ihi; ++i) {
      int ec[3] = {px, py, pz};
      ec[DIR] = i;
      const int e = ec[0] + TG::FX * (ec[1] + TG::FY * ec[2]);
      const int m = pn - i;
      const T wl = m == 0 ? T(2) : m == 1 ? T(-13) : m == 2 ? T(47) : m == 3 ? T(27) : m == 4 ? T(-3) : T(0);
      const T wr = m == 1 ? T(-3) : m == 2 ? T(27) : m == 3 ? T(47) : m == 4 ? T(-13) : m == 5 ? T(2) : T(0);
      const T wd = m == 1 ? T(1) : m == 2 ? T(-15) : m == 3 ? T(15) : m == 4 ? T(-1) : T(0);
#pragma unroll
      for (int k = 0; k < 5; ++k)
        acc[k] += wl * cl[k * TG::NFF + e] + wr * cr[k * TG::NFF + e] + wd * cd[k * TG::NFF + e];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) global_add(lam + (long long)gcomp_local<DIR>(k) * g.N + cell, double(acc[k]));
  }
  } else {
  // ---- phase 3: the face-field cotangents of the tile and its halo into G
  // (10 fields of N faces, face n+1/2 at cell n, local-frame components); face
  // rows past the end of a partial tile carry nothing
  {
    constexpr int A1 = (DIR + 1) % 3, A2 = (DIR + 2) % 3;
    for (int e = tid; e < TG::NFF; e += 256) {
      const int ex = e % TG::FX, ey = (e / TG::FX) % TG::FY, ez = e / (TG::FX * TG::FY);
      int c[3] = {x0 + ex - TG::HX, y0 + ey - TG::HY, z0 + ez - TG::HZ};
      if (c[DIR] >= g.n[DIR]) continue;
      c[A1] = wrap_coord(c[A1], g.n[A1]);
      c[A2] = wrap_coord(c[A2], g.n[A2]);
      const long long f = (long long)c[0] + (long long)c[1] * g.stride[1] + (long long)c[2] * g.stride[2];
#pragma unroll
      for (int k = 0; k < 10; ++k) {
        const double v = ffb[k * TG::NFF + e];
        if (v != 0.0) global_add(G + (long long)k * g.N + f, v);
      }
    }
  }
  }
}

// Faces per workgroup of face_field_vjp_kernel (y- and z-faces): a run of L faces
// along the normal times W along x, so that loads are contiguous across lanes.
template <int DIR> struct FfvTile { static constexpr int L = 16, W = 16; };

// Per face: read and clear G (Q0-bar, D_n-bar), reverse the compatibility state
// and the normal reconstruction into the cotangents l = Q_l-bar/60, r =
// Q_r-bar/60, d = D_n-bar/(12 h) (LDS).  Per cell of the workgroup's footprint
// (its W columns, L + 5 cells along the normal): the transpose of the normal
// reconstruction gathered over the run's faces whose stencil holds the cell, with
// stencil weights (position m = 0..5, cells n-2 .. n+3 of face n+1/2)
//   l (2, -13, 47, 27, -3, 0) + r (0, -3, 27, 47, -13, 2) + d (0, 1, -15, 15, -1, 0),
// added into lambda.  A cell whose six faces are all in the run (positions 5 ..
// L-1 of the footprint, on an axis of at least L + 5 cells, where the footprint
// does not wrap onto itself) belongs to this workgroup alone and is updated by a
// plain read-modify-write; the five cells at either end by atomic adds.
template <typename T, int DIR>
__global__ void __launch_bounds__(256) face_field_vjp_kernel(Geo g, const double* __restrict__ q,
                                                             double* __restrict__ G, double* __restrict__ lam) {
  static_assert(DIR != 0, "x-faces finish in flux_vjp_kernel");
  constexpr int L = FfvTile<DIR>::L, W = FfvTile<DIR>::W;
  static_assert(L * W == 256, "one face per thread");
  constexpr int AW = 0;            // tangential axis of the W columns
  constexpr int AO = 3 - DIR;      // the other tangential axis (one index per workgroup)
  __shared__ double sc[15][256];
  const int tid = threadIdx.x;
  // lanes run along x, the W axis
  const int ln = tid / W, lw = tid % W;
  const int n0 = int(blockIdx.x) * L, w0 = int(blockIdx.y) * W, o = int(blockIdx.z);
  const int Nn = g.n[DIR], Nw = g.n[AW];
  const int nf = n0 + ln, wf = w0 + lw;
  double cot[15];
#pragma unroll
  for (int j = 0; j < 15; ++j) cot[j] = 0.0;
  if (nf < Nn && wf < Nw) {
    int c[3];
    c[DIR] = nf;
    c[AW] = wf;
    c[AO] = o;
    const long long f = (long long)c[0] + (long long)c[1] * g.stride[1] + (long long)c[2] * g.stride[2];
    T Q0b[5], Dnb[5];
    bool any = false;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double a = G[(long long)k * g.N + f], d = G[(long long)(5 + k) * g.N + f];
      G[(long long)k * g.N + f] = 0.0;
      G[(long long)(5 + k) * g.N + f] = 0.0;
      Q0b[k] = T(a);
      Dnb[k] = T(d);
      any = any || a != 0.0 || d != 0.0;
    }
    if (any) {
      // the six cells of the normal stencil, deviations from the reference
      // state in the local frame, rounded to T as in the forward
      const long long sn = g.stride[DIR];
      const long long base = f - (long long)nf * sn;
      T v[5][6];
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        const long long cell = base + (long long)wrapi(nf - 2 + m, Nn) * sn;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const double ref = k == 0 ? g.rho_ref : (k == 4 ? g.E_ref : 0.0);
          v[k][m] = T(q[(long long)gcomp_local<DIR>(k) * g.N + cell] - ref);
        }
      }
      const T ih12 = T(g.inv_h[DIR] * (1.0 / 12.0));
      T Ql[5], Qr[5], Dn[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) normal_recon(v[k], ih12, Ql[k], Qr[k], Dn[k]);
      T Qlb[5] = {0, 0, 0, 0, 0}, Qrb[5] = {0, 0, 0, 0, 0};
      compat_dev_vjp(g, Ql, Qr, Q0b, Qlb, Qrb);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        cot[k] = double(Qlb[k] * T(1.0 / 60.0));
        cot[5 + k] = double(Qrb[k] * T(1.0 / 60.0));
        cot[10 + k] = double(Dnb[k] * ih12);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 15; ++j) sc[j][tid] = cot[j];
  __syncthreads();

  const int Lb = Nn - n0 < L ? Nn - n0 : L;  // faces of the run
  const bool own_ok = Nn >= L + 5;
  for (int cid = tid; cid < W * (L + 5); cid += 256) {
    const int cj = cid / W;  // footprint position along the normal
    const int cw = cid % W;
    if (w0 + cw >= Nw) continue;
    double acc[5] = {0, 0, 0, 0, 0};
    const int ilo = cj - 5 > 0 ? cj - 5 : 0, ihi = cj < Lb - 1 ? cj : Lb - 1;
    for (int i = ilo; i <= ihi; ++i) {
      const int m = cj - i;
      const double wl = m == 0 ? 2.0 : m == 1 ? -13.0 : m == 2 ? 47.0 : m == 3 ? 27.0 : m == 4 ? -3.0 : 0.0;
      const double wr = m == 1 ? -3.0 : m == 2 ? 27.0 : m == 3 ? 47.0 : m == 4 ? -13.0 : m == 5 ? 2.0 : 0.0;
      const double wd = m == 1 ? 1.0 : m == 2 ? -15.0 : m == 3 ? 15.0 : m == 4 ? -1.0 : 0.0;
      const int t = cw + W * i;  // thread of face i in column cw
#pragma unroll
      for (int k = 0; k < 5; ++k) acc[k] += wl * sc[k][t] + wr * sc[5 + k][t] + wd * sc[10 + k][t];
    }
    int c[3];
    c[DIR] = wrap_coord(n0 - 2 + cj, Nn);
    c[AW] = w0 + cw;
    c[AO] = o;
    const long long cell = (long long)c[0] + (long long)c[1] * g.stride[1] + (long long)c[2] * g.stride[2];
    const bool own = own_ok && cj >= 5 && cj < Lb;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      if (acc[k] == 0.0) continue;
      double* p = lam + (long long)gcomp_local<DIR>(k) * g.N + cell;
      if (own)
        *p += acc[k];
      else
        global_add(p, acc[k]);
    }
  }
}

template <typename T, int DIR, bool NEED_F>
static void launch_vjp_dir(const Geo& g, const double* q, const double* A, const double* B, double cLA, double cLB,
                           double cDA, double cDB, double* G, double* lam, hipStream_t st) {
  using TG = AdjGeom<DIR>;
  const int ntx = (g.n[0] + TG::BX - 1) / TG::BX;
  const int nty = (g.n[1] + TG::BY - 1) / TG::BY;
  const int ntz = (g.n[2] + TG::BZ - 1) / TG::BZ;
  const int nper = (ntx * nty * ntz + 7) / 8;
  flux_vjp_kernel<T, DIR, NEED_F><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, A, B, cLA, cLB, cDA, cDB, G,
                                                                                lam, ntx, nty, ntz, nper);
  if constexpr (DIR != 0) {
    constexpr int L = FfvTile<DIR>::L, W = FfvTile<DIR>::W;
    constexpr int AW = 0, AO = 3 - DIR;
    const dim3 grid(unsigned((g.n[DIR] + L - 1) / L), unsigned((g.n[AW] + W - 1) / W), unsigned(g.n[AO]));
    face_field_vjp_kernel<T, DIR><<<grid, dim3(256), 0, st>>>(g, q, G, lam);
  }
}

template <typename T>
static void operator_vjp_t(const Geo& g, int dir, const double* q, const double* A, const double* B, double cLA,
                           double cLB, double cDA, double cDB, double* G, double* lam, hipStream_t st) {
  const bool need_f = cLA != 0.0 || cLB != 0.0;
  if (need_f) {
    if (dir == 0) launch_vjp_dir<T, 0, true>(g, q, A, B, cLA, cLB, cDA, cDB, G, lam, st);
    else if (dir == 1) launch_vjp_dir<T, 1, true>(g, q, A, B, cLA, cLB, cDA, cDB, G, lam, st);
    else launch_vjp_dir<T, 2, true>(g, q, A, B, cLA, cLB, cDA, cDB, G, lam, st);
  } else {
    if (dir == 0) launch_vjp_dir<T, 0, false>(g, q, A, B, cLA, cLB, cDA, cDB, G, lam, st);
    else if (dir == 1) launch_vjp_dir<T, 1, false>(g, q, A, B, cLA, cLB, cDA, cDB, G, lam, st);
    else launch_vjp_dir<T, 2, false>(g, q, A, B, cLA, cLB, cDA, cDB, G, lam, st);
  }
}

// lam += (dL/dQ)^T mu_L + (ddL/dQ)^T mu_dL at state q for the faces of direction
// dir, with mu_L = cLA A + cLB B and mu_dL = cDA A + cDB B (B may be null).  With
// f32 the forward recompute and its reverse run in FP32 (the FP32-flux form).  G
// is a scratch array of 10 N doubles that must hold zeros on entry; it holds
// zeros again on return.
void launch_operator_vjp(const Geo& g, int dir, bool f32, const double* q, const double* A, const double* B,
                         double cLA, double cLB, double cDA, double cDB, double* G, double* lam, hipStream_t st) {
  if (f32) operator_vjp_t<float>(g, dir, q, A, B, cLA, cLB, cDA, cDB, G, lam, st);
  else operator_vjp_t<double>(g, dir, q, A, B, cLA, cLB, cDA, cDB, G, lam, st);
}

// out = a * X + b * Y (elementwise over n doubles)
__global__ void __launch_bounds__(256) axpby_kernel(double a, const double* __restrict__ X, double b,
                                                    const double* __restrict__ Y, double* __restrict__ out, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = a * X[i] + b * Y[i];
}

__global__ void __launch_bounds__(256) fill_kernel(double* __restrict__ out, double v, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = v;
}

__global__ void set_dt_kernel(Ctrl* ctrl, double dt) {
  ctrl->dt = dt;
  ctrl->flag = 0;
  ctrl->zero = 0;
}

static unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  return unsigned(b > 65536 ? 65536 : b);
}

void launch_axpby(double a, const double* X, double b, const double* Y, double* out, long long n, hipStream_t st) {
  axpby_kernel<<<grid_for(n), 256, 0, st>>>(a, X, b, Y, out, n);
}

void launch_fill(double* out, double v, long long n, hipStream_t st) { fill_kernel<<<grid_for(n), 256, 0, st>>>(out, v, n); }

void launch_set_dt(Ctrl* ctrl, double dt, hipStream_t st) { set_dt_kernel<<<1, 1, 0, st>>>(ctrl, dt); }

}  // namespace hgks
