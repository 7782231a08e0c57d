// Tile geometry and the two reconstruction phases shared by the fused face-flux
// kernel (flux_fused.hip) and its adjoint (adjoint.hip), so that the adjoint
// recomputes exactly the forward arithmetic.
//
// A workgroup of 256 threads owns a tile of 256 faces of direction DIR plus a
// halo of two faces along both tangential axes.  y- and z-faces use 32 x 8 tiles
// along x and the other tangential axis, so that x, the contiguous axis, is wide
// in every load; square 16 x 16 tangential tiles, which evaluate fewer halo faces
// (1.56 instead of 1.69 per face), measured no faster.  x-face tiles are
// necessarily short in x.  TileGeom's 4 x 8 x 8 x-tile loads each entry's
// six-cell x-stencil directly (a one-face-wide tile doing so runs 40% slower);
// the periodic flux kernel instead uses a 2 x 16 x 8 x-tile whose cell block is
// staged through LDS (face_field_tile_x_staged).
#pragma once

#include <type_traits>

#include "device_common.hpp"

namespace hgks {

template <int DIR> struct FluxTile;
template <> struct FluxTile<0> { static constexpr int B[3] = {4, 8, 8}; };
template <> struct FluxTile<1> { static constexpr int B[3] = {32, 1, 8}; };
template <> struct FluxTile<2> { static constexpr int B[3] = {32, 8, 1}; };

// Geometry of a tile of BX_ x BY_ x BZ_ faces of direction DIR with its halo.
template <int DIR, int BX_, int BY_, int BZ_>
struct TileGeomB {
  static constexpr int BX = BX_, BY = BY_, BZ = BZ_;
  static constexpr int HX = DIR == 0 ? 0 : 2, HY = DIR == 1 ? 0 : 2, HZ = DIR == 2 ? 0 : 2;
  static constexpr int FX = BX + 2 * HX, FY = BY + 2 * HY, FZ = BZ + 2 * HZ;
  static constexpr int NFF = FX * FY * FZ;
  static constexpr int S[3] = {1, FX, FX * FY};  // LDS strides of the face-field tile
  static constexpr int BA[3] = {BX, BY, BZ};      // faces along each axis
  static_assert(BX * BY * BZ == 256, "one face per thread");
};
template <int DIR>
using TileGeom = TileGeomB<DIR, FluxTile<DIR>::B[0], FluxTile<DIR>::B[1], FluxTile<DIR>::B[2]>;

__device__ __forceinline__ int wrapmod(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// global component of local-frame component `local` for face direction DIR:
// (rho, m_n, m_t1, m_t2, E) with (n, t1, t2) = (x, y, z), (y, z, x), (z, x, y)
template <int DIR>
__host__ __device__ __forceinline__ int gcomp_local(int local) {
  return (local == 0 || local == 4) ? local : 1 + (DIR + local - 1) % 3;
}

// XCD-aware tile order: block b runs on XCD b % 8 and takes tile (b % 8) * nper + b / 8
__device__ __forceinline__ int tile_of_block(int nper) { return int(blockIdx.x % 8u) * nper + int(blockIdx.x / 8u); }

// Origin (first face) of a tile.  x-face tiles are numbered with the normal
// axis fastest: the next tile along the normal shares five of the six stencil
// planes, and the blocks resident on one XCD at a time (a contiguous range of
// tiles) cover a short column of planes that stays in its L2.  y- and z-face
// tiles are numbered x first (see each branch).
template <int DIR, class TG = TileGeom<DIR>>
__device__ __forceinline__ void tile_origin(int tile, int ntx, int nty, int ntz, int& x0, int& y0, int& z0) {
  if (DIR == 0) {
    x0 = (tile % ntx) * TG::BX;
    const int r = tile / ntx;
    y0 = (r % nty) * TG::BY;
    z0 = (r / nty) * TG::BZ;
  } else if (DIR == 1) {
    // y-faces: x first, then y (a y-face tile is one row thick, so the next row
    // follows after ntx tiles); walking y first doubled the HBM fetch
    x0 = (tile % ntx) * TG::BX;
    const int r = tile / ntx;
    y0 = (r % nty) * TG::BY;
    z0 = (r / nty) * TG::BZ;
  } else {
    // z-faces: x first, then z, then y: the tiles resident on one XCD cover a
    // few z-planes of a slab of y-rows whole in x, so that both the x-halo and
    // the shared stencil planes along z stay in its L2
    x0 = (tile % ntx) * TG::BX;
    const int r = tile / ntx;
    z0 = (r % ntz) * TG::BZ;
    y0 = (r / ntz) * TG::BY;
  }
}

// Periodic coordinate c >= -n wrapped into [0, n): one conditional add or
// subtract when c < 2 n (every tile on an axis at least as long as the tile and
// its halo), the remainder otherwise.
__device__ __forceinline__ int wrap_coord(int c, int n) {
  c = c < 0 ? c + n : c;
  if (c >= n) {
    c -= n;
    if (c >= n) c = c % n;
  }
  return c;
}

// Cell averages along the normal of face-field entry e (six cells n-2 .. n+3),
// as deviations from the reference state, in the local frame; the global cell
// offsets of the six cells are returned in off.  Periodic axes wrap; with WALL,
// y is not periodic and rows outside [0, ny) are wall ghosts (their offsets are
// those of the mirror cells).  OFF32 (for N <= 2^29 cells, where every byte
// offset into a field fits 32 bits) forms one 32-bit byte offset per cell and
// adds it to each field's base in the load itself, instead of one 64-bit
// address per load.
template <typename T, int DIR, bool WALL = false, class TG = TileGeom<DIR>, bool OFF32 = false>
__device__ __forceinline__ void normal_stencil(const Geo& g, const double* __restrict__ q, int e, int x0, int y0,
                                               int z0, T (*v)[6], long long* off) {
  const int ex = e % TG::FX, ey = (e / TG::FX) % TG::FY, ez = e / (TG::FX * TG::FY);
  if (!WALL) {
    int c[3] = {wrap_coord(x0 + ex - TG::HX, g.n[0]), wrap_coord(y0 + ey - TG::HY, g.n[1]),
                wrap_coord(z0 + ez - TG::HZ, g.n[2])};
    const int nn = c[DIR], Nn = g.n[DIR];
    if (OFF32) {
      const unsigned sn = unsigned(g.stride[DIR]);
      const unsigned base = unsigned(c[0]) + unsigned(c[1]) * unsigned(g.stride[1]) +
                            unsigned(c[2]) * unsigned(g.stride[2]) - unsigned(nn) * sn;
      unsigned boff[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        const unsigned o = base + unsigned(wrapi(nn - 2 + m, Nn)) * sn;
        off[m] = (long long)o;
        boff[m] = o * 8u;
      }
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const char* f = (const char*)(q + (long long)gcomp_local<DIR>(k) * g.N);
        const double ref = k == 0 ? g.rho_ref : (k == 4 ? g.E_ref : 0.0);
#pragma unroll
        for (int m = 0; m < 6; ++m) v[k][m] = T(*(const double*)(f + boff[m]) - ref);
      }
      return;
    }
    const long long sn = g.stride[DIR];
    const long long base = (long long)c[0] + (long long)c[1] * g.stride[1] + (long long)c[2] * g.stride[2] -
                           (long long)nn * sn;
#pragma unroll
    for (int m = 0; m < 6; ++m) off[m] = base + (long long)wrapi(nn - 2 + m, Nn) * sn;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double* f = q + (long long)gcomp_local<DIR>(k) * g.N;
      const double ref = k == 0 ? g.rho_ref : (k == 4 ? g.E_ref : 0.0);
#pragma unroll
      for (int m = 0; m < 6; ++m) v[k][m] = T(f[off[m]] - ref);
    }
  } else {
    // x and z periodic, y unwrapped (ghost rows allowed)
    int c[3] = {wrap_coord(x0 + ex - TG::HX, g.n[0]), y0 + ey - TG::HY, wrap_coord(z0 + ez - TG::HZ, g.n[2])};
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      int cc[3] = {c[0], c[1], c[2]};
      cc[DIR] = DIR == 1 ? c[1] - 2 + m : wrapi(c[DIR] - 2 + m, g.n[DIR]);
      double Q[5];
      load_cell_wall(g, q, cc[0], cc[1], cc[2], Q);
      bool ghost;
      const int ym = wall_row(g, cc[1], ghost);
      off[m] = (long long)cc[0] + (long long)ym * g.stride[1] + (long long)cc[2] * g.stride[2];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const double ref = k == 0 ? g.rho_ref : (k == 4 ? g.E_ref : 0.0);
        v[k][m] = T(Q[gcomp_local<DIR>(k)] - ref);
      }
    }
  }
}

// Normal reconstruction at the face between cells 2 and 3 of the six:
// fifth-order left/right values (WENO5 with its optimal linear weights) and the
// derivative of the cubic through the four middle cells.
template <typename T>
__host__ __device__ __forceinline__ void normal_recon(const T* v, T ih12, T& ql, T& qr, T& dn) {
  ql = (T(2) * v[0] - T(13) * v[1] + T(47) * v[2] + T(27) * v[3] - T(3) * v[4]) * T(1.0 / 60.0);
  qr = (T(-3) * v[1] + T(27) * v[2] + T(47) * v[3] - T(13) * v[4] + T(2) * v[5]) * T(1.0 / 60.0);
  dn = (v[1] - T(15) * v[2] + T(15) * v[3] - v[4]) * ih12;
}

// Phase 1: face field (Q0 deviation and dQ0/dn, local frame) of the tile and its
// tangential halo into ff[10][NFF].  dn_scale is 1/h of the normal axis (for
// y-faces of a stretched mesh, 1/(y' h) at the tile's face row).  The caller
// synchronizes.
template <typename T, int DIR, bool WALL = false, class TG = TileGeom<DIR>, bool OFF32 = false>
__device__ __forceinline__ void face_field_tile(const Geo& g, const double* __restrict__ q, T* ff, int x0, int y0,
                                                int z0, double dn_scale) {
  const T ih12 = T(dn_scale * (1.0 / 12.0));
  for (int e = threadIdx.x; e < TG::NFF; e += 256) {
    T v[5][6];
    long long off[6];
    normal_stencil<T, DIR, WALL, TG, OFF32>(g, q, e, x0, y0, z0, v, off);
    T Ql[5], Qr[5], Dn[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) normal_recon(v[k], ih12, Ql[k], Qr[k], Dn[k]);
    T Q0[5];
    compat_dev(g, Ql, Qr, Q0);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      ff[k * TG::NFF + e] = Q0[k];
      ff[(5 + k) * TG::NFF + e] = Dn[k];
    }
  }
}

// Phase 1 for x-faces staged through LDS.  An x-face tile is only a few faces
// long in x, the contiguous axis, so per-entry stencil loads touch many cache
// lines per instruction.  Here the workgroup loads the tile's cell block (x from
// x0-2 to x0+BX+2, the tangential extent with its halo) one component at a time
// into blk, x fastest, so each load instruction covers consecutive runs of cells;
// every entry then takes its six-cell stencil from LDS and keeps Q_l, Q_r and D_n
// in registers until all five components are in, when the compatibility state is
// formed.  blk holds BX+5 by FY by FZ values (deviations from the reference
// state, rounded to T as in normal_stencil), or twice that with PAIRS, which
// stages two components per round (three rounds instead of five).  The caller
// synchronizes after.
template <typename T, class TG, bool OFF32, bool PAIRS>
__device__ __forceinline__ void face_field_tile_x_staged(const Geo& g, const double* __restrict__ q, T* ff, T* blk,
                                                         int x0, int y0, int z0, double dn_scale) {
  static_assert(TG::HX == 0 && TG::HY == 2 && TG::HZ == 2, "x-face tile");
  constexpr int CX = TG::BX + 5;                 // cells along x
  constexpr int NB = CX * TG::FY * TG::FZ;       // cells of the block
  constexpr int NL = (NB + 255) / 256;           // block cells per thread
  const T ih12 = T(dn_scale * (1.0 / 12.0));
  const int tid = threadIdx.x;
  // element offsets of this thread's block cells (the last slot may be empty);
  // a block that crosses no periodic boundary (most tiles) needs no wrapping
  long long off[NL];
  const bool inner = x0 >= 2 && x0 + CX - 2 <= g.n[0] && y0 >= 2 && y0 + TG::FY - 2 <= g.n[1] && z0 >= 2 &&
                     z0 + TG::FZ - 2 <= g.n[2];
  if (inner) {
    const long long c0 = (long long)(x0 - 2) + (long long)(y0 - 2) * g.stride[1] + (long long)(z0 - 2) * g.stride[2];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int b = tid + 256 * i < NB ? tid + 256 * i : NB - 1;
      const int bx = b % CX, r = b / CX, by = r % TG::FY, bz = r / TG::FY;
      off[i] = c0 + (long long)bx + (long long)by * g.stride[1] + (long long)bz * g.stride[2];
    }
  } else {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int b = tid + 256 * i < NB ? tid + 256 * i : NB - 1;
      const int bx = b % CX, r = b / CX, by = r % TG::FY, bz = r / TG::FY;
      const int cx = wrap_coord(x0 - 2 + bx, g.n[0]);
      const int cy = wrap_coord(y0 - 2 + by, g.n[1]);
      const int cz = wrap_coord(z0 - 2 + bz, g.n[2]);
      off[i] = (long long)cx + (long long)cy * g.stride[1] + (long long)cz * g.stride[2];
    }
  }
  auto load = [&](int k, double* val) {
    const double* f = q + (long long)k * g.N;
#pragma unroll
    for (int i = 0; i < NL; ++i)
      val[i] = OFF32 ? *(const double*)((const char*)f + unsigned(off[i]) * 8u) : f[off[i]];
  };
  // one thread per block row (fixed y, z): it reads the row's CX cells once and
  // reconstructs the BX entries of that row (a row stride of CX doubles keeps the
  // reads of sixteen consecutive lanes on distinct LDS banks)
  constexpr int NR = TG::FY * TG::FZ;
  static_assert(NR <= 256 && TG::FX == TG::BX, "one block row per thread");
  T Ql[TG::BX][5], Qr[TG::BX][5], Dn[TG::BX][5];
  if constexpr (PAIRS) {
  // two components per round (blk holds two blocks): three rounds, six barriers
  double val2[2][NL];
  load(0, val2[0]);
  load(1, val2[1]);
#pragma unroll
  for (int k0 = 0; k0 < 5; k0 += 2) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = k0 + j;
      if (k < 5) {
        const double ref = k == 0 ? g.rho_ref : (k == 4 ? g.E_ref : 0.0);
#pragma unroll
        for (int i = 0; i < NL; ++i)
          if (tid + 256 * i < NB) blk[j * NB + tid + 256 * i] = T(val2[j][i] - ref);
      }
    }
    __syncthreads();
    if (k0 + 2 < 5) load(k0 + 2, val2[0]);
    if (k0 + 3 < 5) load(k0 + 3, val2[1]);
    if (tid < NR) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int k = k0 + j;
        if (k < 5) {
          const T* c = blk + j * NB + CX * tid;
          T v[CX];
#pragma unroll
          for (int m = 0; m < CX; ++m) v[m] = c[m];
#pragma unroll
          for (int ex = 0; ex < TG::BX; ++ex) normal_recon(v + ex, ih12, Ql[ex][k], Qr[ex][k], Dn[ex][k]);
        }
      }
    }
    __syncthreads();
  }
  } else {
  double val[NL];
  load(0, val);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double ref = k == 0 ? g.rho_ref : (k == 4 ? g.E_ref : 0.0);
#pragma unroll
    for (int i = 0; i < NL; ++i)
      if (tid + 256 * i < NB) blk[tid + 256 * i] = T(val[i] - ref);
    __syncthreads();
    // the next component's loads are in flight while this one is reconstructed
    if (k < 4) load(k + 1, val);
    if (tid < NR) {
      const T* c = blk + CX * tid;
      T v[CX];
#pragma unroll
      for (int m = 0; m < CX; ++m) v[m] = c[m];
#pragma unroll
      for (int ex = 0; ex < TG::BX; ++ex) normal_recon(v + ex, ih12, Ql[ex][k], Qr[ex][k], Dn[ex][k]);
    }
    __syncthreads();
  }
  }
  if (tid < NR) {
    T Q0[TG::BX][5];
#pragma unroll
    for (int ex = 0; ex < TG::BX; ++ex) compat_dev(g, Ql[ex], Qr[ex], Q0[ex]);
    if constexpr (TG::BX == 2) {
      // the row's two entries are adjacent in ff: one vector store per field
      static_assert(TG::NFF % 2 == 0, "pairs of entries");
      using T2 = typename std::conditional<sizeof(T) == sizeof(double), double2, float2>::type;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        T2 a, d;
        a.x = Q0[0][k];
        a.y = Q0[1][k];
        d.x = Dn[0][k];
        d.y = Dn[1][k];
        *(T2*)(ff + k * TG::NFF + 2 * tid) = a;
        *(T2*)(ff + (5 + k) * TG::NFF + 2 * tid) = d;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
#pragma unroll
        for (int ex = 0; ex < TG::BX; ++ex) {
          ff[k * TG::NFF + TG::BX * tid + ex] = Q0[ex][k];
          ff[(5 + k) * TG::NFF + TG::BX * tid + ex] = Dn[ex][k];
        }
      }
    }
  }
}

// Explicit tangential weights at Gauss point m (0: -, 1: +) for value and
// derivative, cell order j-2 .. j+2 (the even/odd forms of tang_val/tang_der).
template <typename T>
__host__ __device__ __forceinline__ void tang_weights(int m, T* wv, T* wd) {
  const T s = m ? T(1) : T(-1);
  wv[0] = T(kVe2) - s * T(kVo2);
  wv[1] = T(kVe1) - s * T(kVo1);
  wv[2] = T(kVe0);
  wv[3] = T(kVe1) + s * T(kVo1);
  wv[4] = T(kVe2) + s * T(kVo2);
  wd[0] = s * T(kDs2) - T(kDa2);
  wd[1] = s * T(kDs1) - T(kDa1);
  wd[2] = s * T(kDs0);
  wd[3] = s * T(kDs1) + T(kDa1);
  wd[4] = s * T(kDs2) + T(kDa2);
}

// The same weights as tables, [m][value 0..4, derivative 0..4].
#define HGKS_TANG_ROW(sg)                                                                                        \
  {kVe2 - (sg) * kVo2, kVe1 - (sg) * kVo1, kVe0, kVe1 + (sg) * kVo1, kVe2 + (sg) * kVo2, (sg) * kDs2 - kDa2,      \
   (sg) * kDs1 - kDa1, (sg) * kDs0, (sg) * kDs1 + kDa1, (sg) * kDs2 + kDa2}
static __constant__ double kTangW64[2][10] = {HGKS_TANG_ROW(-1.0), HGKS_TANG_ROW(1.0)};
static __constant__ float kTangW32[2][10] = {HGKS_TANG_ROW(-1.0), HGKS_TANG_ROW(1.0)};
#undef HGKS_TANG_ROW
template <typename T>
__device__ __forceinline__ const T* tang_table(int m);
template <>
__device__ __forceinline__ const double* tang_table<double>(int m) {
  return kTangW64[m];
}
template <>
__device__ __forceinline__ const float* tang_table<float>(int m) {
  return kTangW32[m];
}

// Phase 2 data: tangential fourth-order reconstruction, for the t1 Gauss point m
// and both t2 Gauss points l, of Q0 (value, d/dt1, d/dt2) and of dQ0/dn (value)
// from the 5 x 5 face neighbourhood whose corner sits at LDS index `corner`.
// Qg[l][k] = Q0 deviation, Dg[l][a][k] = dQ0_k/dx_a along (n, t1, t2).  i1 is the
// t1 metric factor at this Gauss point, i2m / i2p the t2 factors at l = 0 / 1.
template <typename T, int DIR, class TG = TileGeom<DIR>>
__device__ __forceinline__ void gp_data(const T* ff, int corner, int m, T i1, T i2m, T i2p, T (*Qg)[5],
                                        T (*Dg)[3][5]) {
  constexpr int A1 = (DIR + 1) % 3, A2 = (DIR + 2) % 3;
  constexpr int s1 = TG::S[A1], s2 = TG::S[A2];
  // the rows (t1 lines) are needed at one t1 Gauss point only: weighted sums
  // with that point's weights (15 FMAs per row) instead of both points' values;
  // the weights come from a constant table indexed by the uniform m (scalar loads)
  const T* wv = tang_table<T>(m);
  const T* wd = wv + 5;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    // keep the scheduler from hoisting the next component's LDS reads: it would
    // otherwise hold all 250 values at once and drop the occupancy to one wave
    asm volatile("" ::: "memory");
    const T* f0 = ff + k * TG::NFF + corner;
    const T* fn = ff + (5 + k) * TG::NFF + corner;
    T rv[5], rd[5], rn[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      T v = wv[0] * f0[r * s2], d = wd[0] * f0[r * s2], n = wv[0] * fn[r * s2];
#pragma unroll
      for (int a = 1; a < 5; ++a) {
        const T x = f0[a * s1 + r * s2], y = fn[a * s1 + r * s2];
        v = v + wv[a] * x;
        d = d + wd[a] * x;
        n = n + wv[a] * y;
      }
      rv[r] = v;
      rd[r] = d;
      rn[r] = n;
    }
    T vm, vp, d2m, d2p, d1m, d1p, nm, np;
    tang_val(rv, vm, vp);
    tang_der(rv, d2m, d2p);
    tang_val(rd, d1m, d1p);
    tang_val(rn, nm, np);
    Qg[0][k] = vm;
    Qg[1][k] = vp;
    Dg[0][0][k] = nm;
    Dg[1][0][k] = np;
    Dg[0][1][k] = d1m * i1;
    Dg[1][1][k] = d1p * i1;
    Dg[0][2][k] = d2m * i2m;
    Dg[1][2][k] = d2p * i2p;
  }
}

// ---------------------------------------------------------------------------
// Phase 2 with shared rows.  The tangential reconstruction at a Gauss point is a
// tensor product: five-point sums along one tangential axis (S, "rows"), then a
// five-point combination of five rows along the other (R).  A row sum depends on
// the face's S position and on the row's R position only, so the faces of the
// tile that share an S position share their rows: each row is summed once per
// tile (pass A, into LDS) instead of once per face that uses it (five times).
// S is the tile's shorter tangential extent, which keeps the R halo (two rows on
// each side) a small fraction: (B_R + 4) / B_R rows per face.
// ---------------------------------------------------------------------------
template <int DIR, class TG = TileGeom<DIR>>
struct RowGeom {
  static constexpr int A1 = (DIR + 1) % 3, A2 = (DIR + 2) % 3;
  static constexpr bool SWAP = TG::BA[A2] < TG::BA[A1];  // S = t2 when t2 is the shorter axis
  static constexpr int AS = SWAP ? A2 : A1, AR = SWAP ? A1 : A2;
  static constexpr int BN = TG::BA[DIR], BS = TG::BA[AS], BR = TG::BA[AR];
  // row entries: normal position, S position and R row (with its halo of two);
  // laid out x fastest, as the threads are, so that neighbouring lanes touch
  // neighbouring words (no LDS bank conflicts)
  static constexpr int E[3] = {DIR == 0 ? BN : (AS == 0 ? BS : BR + 4), DIR == 1 ? BN : (AS == 1 ? BS : BR + 4),
                               DIR == 2 ? BN : (AS == 2 ? BS : BR + 4)};
  static constexpr int ES[3] = {1, E[0], E[0] * E[1]};
  static constexpr int NE = E[0] * E[1] * E[2];
  static constexpr int NBUF = 3 * NE;  // value, S-derivative and normal-derivative rows
};

// Pass A for S Gauss point pt (0: -, 1: +) and component k: the rows of Q0 (value
// and S-derivative weights) and of dQ0/dn (value weights) into buf[3][NE].
template <typename T, int DIR, class TG = TileGeom<DIR>>
__device__ __forceinline__ void rows_pass(const T* ff, T* buf, int pt, int k) {
  using RG = RowGeom<DIR, TG>;
  const T* wv = tang_table<T>(pt);
  const T* wd = wv + 5;
  constexpr int sS = TG::S[RG::AS];
  for (int e = threadIdx.x; e < RG::NE; e += 256) {
    // (normal, S position, R row) in face-field coordinates: the S taps start at
    // the face's own position (halo of two), the R row is already in halo coordinates
    const int c0 = e % RG::E[0], c1 = (e / RG::E[0]) % RG::E[1], c2 = e / (RG::E[0] * RG::E[1]);
    const int base = c0 * TG::S[0] + c1 * TG::S[1] + c2 * TG::S[2];
    const T* f0 = ff + k * TG::NFF + base;
    const T* fn = ff + (5 + k) * TG::NFF + base;
    T v = wv[0] * f0[0], d = wd[0] * f0[0], w = wv[0] * fn[0];
#pragma unroll
    for (int a = 1; a < 5; ++a) {
      const T x = f0[a * sS], y = fn[a * sS];
      v = v + wv[a] * x;
      d = d + wd[a] * x;
      w = w + wv[a] * y;
    }
    buf[e] = v;
    buf[RG::NE + e] = d;
    buf[2 * RG::NE + e] = w;
  }
}

// Pass B for the face at tile position (n, s, rr) (normal, S, R): values and
// derivatives of component k at the two R Gauss points l = 0 (-), 1 (+) from its
// five rows.  vR[l] = Q0, dR[l] = dQ0/dR, dS[l] = dQ0/dS (per unit width), dn[l] = dQ0/dn.
template <typename T, int DIR, class TG = TileGeom<DIR>>
__device__ __forceinline__ void rows_combine(const T* buf, int n, int s, int rr, T* vR, T* dR, T* dS, T* dn) {
  using RG = RowGeom<DIR, TG>;
  const int e0 = n * RG::ES[DIR] + s * RG::ES[RG::AS] + rr * RG::ES[RG::AR];
  constexpr int st = RG::ES[RG::AR];
  T rv[5], rd[5], rn[5];
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    rv[b] = buf[e0 + b * st];
    rd[b] = buf[RG::NE + e0 + b * st];
    rn[b] = buf[2 * RG::NE + e0 + b * st];
  }
  tang_val(rv, vR[0], vR[1]);
  tang_der(rv, dR[0], dR[1]);
  tang_val(rd, dS[0], dS[1]);
  tang_val(rn, dn[0], dn[1]);
}

}  // namespace hgks
