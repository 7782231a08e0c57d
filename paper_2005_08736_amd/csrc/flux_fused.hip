// Fused face-flux kernel of one face direction, LDS-tiled for gfx950.
//
// One workgroup (256 threads) owns a tile of 256 faces of direction DIR.  It
//   1. reconstructs, for the tile and a halo of two faces along both tangential
//      axes, the face field: fifth-order normal values Q_l, Q_r from the cell
//      averages, the equilibrium state Q0 by the compatibility condition and the
//      normal derivative of Q0 (Sec. 2.1), into LDS;
//   2. reconstructs Q0, its three derivatives and the normal derivative to the
//      2x2 Gauss points of each face with the tangential fourth-order polynomials
//      (Remark 1 of Sec. 2.1) and evaluates the gas-kinetic flux there;
//   3. writes the face average of F^n and dF^n/dt (Eq. (expansion-1)).
// The arithmetic type T is double for the FP64 path and float for the FP32-flux
// form; cell averages are read in FP64 and turned into deviations from the
// reference state before they are rounded to T, and face fluxes are stored in T.
// Tiles are dealt to the eight XCDs in contiguous ranges so that neighbouring
// tiles, which share halo cells, meet in the same L2.
#include "flux_tile.hpp"
#include "internal.hpp"

namespace hgks {

// Tile shapes.  y- and z-faces use TileGeom (32 x 8 along x and the other
// tangential axis).  FP64 x-faces of the periodic kernels use a 2 x 16 x 8 tile whose
// phase 1 is staged through LDS (face_field_tile_x_staged, the cell blocks in
// the face field's own space) and whose phase 2 shares rows: its face field
// (38 KB) and two row buffers (15 KB) fit three workgroups per CU.  The channel
// kernel keeps the 4 x 8 x 8 x-tile with direct stencil loads (its wall ghosts
// need all five components of a mirror cell at once); in FP64 that tile's face
// field already fills 46 KB, so its phase 2 goes per face (gp_data) rather than
// drop to two workgroups per CU.
template <typename T, int DIR, bool CHAN>
struct FusedTile {
  using TG = TileGeom<DIR>;
  static constexpr bool kStaged = false;
};
template <typename T>
struct FusedTile<T, 0, false> {
  using TG = TileGeomB<0, 2, 16, 8>;
  static constexpr bool kStaged = true;
};
// FP32 x-faces: a 4 x 8 x 8 tile (2.25 face-field entries per face instead of
// 1.88) writes 16-byte runs of each output field instead of 8-byte ones, and
// its staged block (9 x 12 x 12 cells) and rows fit in 32 KB: 3% faster in FP32
template <>
struct FusedTile<float, 0, false> {
  using TG = TileGeomB<0, 4, 8, 8>;
  static constexpr bool kStaged = true;
};
template <typename T, int DIR, bool CHAN>
constexpr bool kSharedRows = !(DIR == 0 && CHAN && sizeof(T) == sizeof(double));
template <typename T, int DIR, bool CHAN>
constexpr int kRowBuf =
    kSharedRows<T, DIR, CHAN> ? 2 * RowGeom<DIR, typename FusedTile<T, DIR, CHAN>::TG>::NBUF : 1;

// Per-face phase 2: each face sums its own 5 x 5 neighbourhood (gp_data), one t1
// Gauss point at a time; with a stretched y (channel), y is t1 of x-faces.
template <typename T, int DIR, bool STAGE2, bool VAR_MU, class TG>
__device__ __forceinline__ void per_face_phase2(const Geo& g, const T* ff, const int* tp, int gy, bool ys, T* Fs,
                                                T* dFs) {
  static_assert(DIR == 0, "per-face phase 2 serves x-faces, whose t1 is the stretched y");
  constexpr int A1 = (DIR + 1) % 3, A2 = (DIR + 2) % 3;
  const int centre = (tp[0] + TG::HX) + (tp[1] + TG::HY) * TG::FX + (tp[2] + TG::HZ) * TG::FX * TG::FY;
  const int corner = centre - 2 * TG::S[A1] - 2 * TG::S[A2];
  const T i2 = T(g.inv_h[A2]);
#pragma unroll 1
  for (int m = 0; m < 2; ++m) {  // t1 Gauss point (-, +)
    T i1 = T(g.inv_h[A1]), w1 = T(1);
    if (ys && A1 == 1) {
      i1 = T(ym_gp_inv(g, gy, m));
      w1 = T(ym_gp_w(g, gy, m));
    }
    T Qg[2][5], Dg[2][3][5];
    gp_data<T, DIR, TG>(ff, corner, m, i1, i2, i2, Qg, Dg);
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      T F[5], dF[5];
      smooth_flux<!STAGE2, VAR_MU>(g, Qg[l], Dg[l], F, dF);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        if (!STAGE2) Fs[k] += ys ? w1 * F[k] : F[k];
        dFs[k] += ys ? w1 * dF[k] : dF[k];
      }
    }
  }
}

template <typename T, int DIR, bool STAGE2, bool VAR_MU, bool CHAN, bool OFF32>
__device__ __forceinline__ void flux_fused_body(const Geo& g, const double* __restrict__ q, T* __restrict__ fl,
                                                T* ff, T* rowbuf, int ntx, int nty, int ntz, int nper) {
  using FT = FusedTile<T, DIR, CHAN>;
  using TG = typename FT::TG;
  using RG = RowGeom<DIR, TG>;
  const int tile = tile_of_block(nper);
  if (tile >= ntx * nty * ntz) return;
  int x0, y0, z0;
  tile_origin<DIR, TG>(tile, ntx, nty, ntz, x0, y0, z0);
  // channel: y-face rows run from the bottom wall face (row -1) to the top one
  if (CHAN && DIR == 1) y0 -= 1;
  double dn_scale = g.inv_h[DIR];
  if (CHAN && DIR == 1 && g.stretch_y) dn_scale = ym_face_inv(g, y0 + 1);

  if constexpr (FT::kStaged) {
    // FP64 stages two components per round, in the face field's space (5% faster
    // than one per round); FP32 one per round in the row buffers (2% faster)
    constexpr int NB = (TG::BX + 5) * TG::FY * TG::FZ;
    constexpr bool pairs = sizeof(T) == sizeof(double);
    static_assert(pairs ? 10 * TG::NFF >= 2 * NB : 2 * RowGeom<DIR, TG>::NBUF >= NB, "cell blocks fit");
    face_field_tile_x_staged<T, TG, OFF32, pairs>(g, q, ff, pairs ? ff : rowbuf, x0, y0, z0, dn_scale);
  } else {
    face_field_tile<T, DIR, CHAN, TG, OFF32>(g, q, ff, x0, y0, z0, dn_scale);
  }
  __syncthreads();

  const int tid = threadIdx.x;
  const int fx = tid % TG::BX, fy = (tid / TG::BX) % TG::BY, fz = tid / (TG::BX * TG::BY);
  const int gx = x0 + fx, gy = y0 + fy, gz = z0 + fz;
  // faces past the end of a partial tile take part in the row passes (and their
  // barriers) but store nothing
  const bool active = gx < g.n[0] && gy < g.n[1] && gz < g.n[2];
  const int tp[3] = {fx, fy, fz};
  // the stretched y of the channel, when tangential, is the row axis S (it is the
  // tile's shorter tangential extent); R is never stretched
  const bool ys = CHAN && DIR != 1 && g.stretch_y;
  const T iR = T(g.inv_h[RG::AR]);
  T Fs[5] = {0, 0, 0, 0, 0}, dFs[5] = {0, 0, 0, 0, 0};
  if constexpr (!kSharedRows<T, DIR, CHAN>) {
    if (!active) return;
    per_face_phase2<T, DIR, STAGE2, VAR_MU, TG>(g, ff, tp, gy, ys, Fs, dFs);
  } else {
#pragma unroll 1
  for (int pt = 0; pt < 2; ++pt) {  // S Gauss point (-, +)
    T iS = T(g.inv_h[RG::AS]), wS = T(1);
    if (ys) {
      iS = T(ym_gp_inv(g, gy, pt));
      wS = T(ym_gp_w(g, gy, pt));
    }
    T Qg[2][5], Dg[2][3][5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      // two row buffers in turn: the rows of the next component are written while
      // no thread can still be reading the buffer from two components back
      T* buf = rowbuf + ((pt + k) & 1) * RG::NBUF;
      rows_pass<T, DIR, TG>(ff, buf, pt, k);
      __syncthreads();
      T vR[2], dR[2], dS[2], dn[2];
      rows_combine<T, DIR, TG>(buf, tp[DIR], tp[RG::AS], tp[RG::AR], vR, dR, dS, dn);
      // finish this component's combination before the next pass starts: left to
      // itself the scheduler keeps the rows of all five components in registers
      // and combines them at the end, which spills (10% slower)
      asm volatile("" ::"v"(vR[0]), "v"(vR[1]), "v"(dR[0]), "v"(dR[1]), "v"(dS[0]), "v"(dS[1]), "v"(dn[0]), "v"(dn[1])
                   : "memory");
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        Qg[l][k] = vR[l];
        Dg[l][0][k] = dn[l];
        Dg[l][RG::SWAP ? 2 : 1][k] = dS[l] * iS;
        Dg[l][RG::SWAP ? 1 : 2][k] = dR[l] * iR;
      }
    }
    if (active) {
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        T F[5], dF[5];
        smooth_flux<!STAGE2, VAR_MU>(g, Qg[l], Dg[l], F, dF);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          if (!STAGE2) Fs[k] += ys ? wS * F[k] : F[k];
          dFs[k] += ys ? wS * dF[k] : dF[k];
        }
      }
    }
  }
  }
  if (!active) return;
  // face n+1/2 is stored at cell n; the bottom wall face of the channel (row -1)
  // goes to its own array
  T* out = fl;
  long long idx = (long long)gx + (long long)gy * g.stride[1] + (long long)gz * g.stride[2];
  long long cs = g.N;
  if (CHAN && DIR == 1 && gy < 0) {
    out = (T*)g.fwall;
    idx = (long long)gx + (long long)gz * g.n[0];
    cs = (long long)g.n[0] * g.n[2];
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int gk = gcomp_local<DIR>(k);
    if (!STAGE2) out[(long long)gk * cs + idx] = T(0.25) * Fs[k];
    out[(long long)(5 + gk) * cs + idx] = T(0.25) * dFs[k];
  }
}

// Waves per SIMD requested from the register allocator for the constant-viscosity
// kernels (the variable-viscosity ones keep the default: capping them spills).
#ifndef HGKS_FLUX_WAVES
#define HGKS_FLUX_WAVES 3
#endif
#ifndef HGKS_FLUX_WAVES_F32
#define HGKS_FLUX_WAVES_F32 4
#endif

template <typename T, int DIR, bool STAGE2, bool OFF32>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? HGKS_FLUX_WAVES : HGKS_FLUX_WAVES_F32)))
flux_fused_kernel(Geo g, const double* __restrict__ q, T* __restrict__ fl, const int* __restrict__ stop, int ntx,
                  int nty, int ntz, int nper) {
  if (*stop) return;
  __shared__ __align__(16) T ff[10 * FusedTile<T, DIR, false>::TG::NFF];
  __shared__ T rowbuf[kRowBuf<T, DIR, false>];
  flux_fused_body<T, DIR, STAGE2, false, false, OFF32>(g, q, fl, ff, rowbuf, ntx, nty, ntz, nper);
}

template <typename T, int DIR, bool OFF32>
__global__ void __launch_bounds__(256) flux_fused_varmu_kernel(Geo g, const double* __restrict__ q,
                                                               T* __restrict__ fl, const int* __restrict__ stop,
                                                               int ntx, int nty, int ntz, int nper) {
  if (*stop) return;
  __shared__ __align__(16) T ff[10 * FusedTile<T, DIR, false>::TG::NFF];
  __shared__ T rowbuf[kRowBuf<T, DIR, false>];
  flux_fused_body<T, DIR, false, true, false, OFF32>(g, q, fl, ff, rowbuf, ntx, nty, ntz, nper);
}

// Channel: walls in y and/or the stretched y mesh (the metric branches are
// uniform over the launch).
template <typename T, int DIR, bool STAGE2, bool VAR_MU>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(VAR_MU ? 1 : (sizeof(T) == 8 ? HGKS_FLUX_WAVES : HGKS_FLUX_WAVES_F32))))
flux_fused_chan_kernel(Geo g, const double* __restrict__ q,
                                                              T* __restrict__ fl, const int* __restrict__ stop,
                                                              int ntx, int nty, int ntz, int nper) {
  if (*stop) return;
  __shared__ T ff[10 * FusedTile<T, DIR, true>::TG::NFF];
  __shared__ T rowbuf[kRowBuf<T, DIR, true>];
  flux_fused_body<T, DIR, STAGE2, VAR_MU, true, false>(g, q, fl, ff, rowbuf, ntx, nty, ntz, nper);
}

template <typename T, int DIR, bool CHAN>
static void tile_grid(const Geo& g, int& ntx, int& nty, int& ntz, int& nper) {
  using TG = typename FusedTile<T, DIR, CHAN>::TG;
  ntx = (g.n[0] + TG::BX - 1) / TG::BX;
  // with walls in y there are ny + 1 rows of y-faces (one tile row each)
  nty = (g.n[1] + (DIR == 1 && g.wall_y ? 1 : 0) + TG::BY - 1) / TG::BY;
  ntz = (g.n[2] + TG::BZ - 1) / TG::BZ;
  nper = (ntx * nty * ntz + 7) / 8;
}

// Boxes of up to 2^29 cells address every field with 32-bit byte offsets.
constexpr long long kOff32MaxCells = 1LL << 29;

template <typename T, int DIR, bool STAGE2, bool VAR_MU>
static void launch_dir(const Geo& g, const double* q, T* fl, const int* stop, hipStream_t st) {
  int ntx, nty, ntz, nper;
  const bool chan = g.wall_y || g.stretch_y;
  if (chan)
    tile_grid<T, DIR, true>(g, ntx, nty, ntz, nper);
  else
    tile_grid<T, DIR, false>(g, ntx, nty, ntz, nper);
  if (chan)
    flux_fused_chan_kernel<T, DIR, STAGE2, VAR_MU><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, fl, stop, ntx,
                                                                                                  nty, ntz, nper);
  else if (g.N <= kOff32MaxCells) {
    if (VAR_MU)
      flux_fused_varmu_kernel<T, DIR, true><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, fl, stop, ntx, nty,
                                                                                           ntz, nper);
    else
      flux_fused_kernel<T, DIR, STAGE2, true><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, fl, stop, ntx, nty,
                                                                                             ntz, nper);
  } else if (VAR_MU) {
    flux_fused_varmu_kernel<T, DIR, false><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, fl, stop, ntx, nty,
                                                                                          ntz, nper);
  } else {
    flux_fused_kernel<T, DIR, STAGE2, false><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, fl, stop, ntx, nty,
                                                                                            ntz, nper);
  }
}

template <typename T, bool STAGE2, bool VAR_MU>
static void launch_any(const Geo& g, int dir, const double* q, T* fl, const int* stop, hipStream_t st) {
  if (dir == 0) launch_dir<T, 0, STAGE2, VAR_MU>(g, q, fl, stop, st);
  else if (dir == 1) launch_dir<T, 1, STAGE2, VAR_MU>(g, q, fl, stop, st);
  else launch_dir<T, 2, STAGE2, VAR_MU>(g, q, fl, stop, st);
}

template <typename T>
static void launch_flux_t(const Geo& g, int dir, bool stage2, const double* q, T* fl, const int* stop, hipStream_t st) {
  const bool var_mu = g.mu_exp != 0.0;
  if (stage2) {
    // the second stage needs dF^n/dt only, which does not involve the viscosity
    launch_any<T, true, false>(g, dir, q, fl, stop, st);
  } else if (var_mu) {
    launch_any<T, false, true>(g, dir, q, fl, stop, st);
  } else {
    launch_any<T, false, false>(g, dir, q, fl, stop, st);
  }
}

void launch_flux_fused(const Geo& g, int dir, bool stage2, const double* q, double* fl, const int* stop,
                       hipStream_t st) {
  launch_flux_t<double>(g, dir, stage2, q, fl, stop, st);
}

void launch_flux_fused(const Geo& g, int dir, bool stage2, const double* q, float* fl, const int* stop,
                       hipStream_t st) {
  launch_flux_t<float>(g, dir, stage2, q, fl, stop, st);
}

}  // namespace hgks
