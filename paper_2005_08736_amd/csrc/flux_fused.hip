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
// Tile shapes keep x, the contiguous axis, fastest in every phase: x-faces use
// 4 x 8 x 8 (halo in y and z), y- and z-faces 32 x 8 along x and the other
// tangential axis.  Tiles are dealt to the eight XCDs in contiguous ranges so
// that neighbouring tiles, which share halo cells, meet in the same L2.
#include "internal.hpp"

namespace hgks {

template <int DIR> struct FluxTile;
template <> struct FluxTile<0> { static constexpr int B[3] = {4, 8, 8}; };
template <> struct FluxTile<1> { static constexpr int B[3] = {32, 1, 8}; };
template <> struct FluxTile<2> { static constexpr int B[3] = {32, 8, 1}; };

template <int DIR>
struct TileGeom {
  static constexpr int BX = FluxTile<DIR>::B[0], BY = FluxTile<DIR>::B[1], BZ = FluxTile<DIR>::B[2];
  static constexpr int HX = DIR == 0 ? 0 : 2, HY = DIR == 1 ? 0 : 2, HZ = DIR == 2 ? 0 : 2;
  static constexpr int FX = BX + 2 * HX, FY = BY + 2 * HY, FZ = BZ + 2 * HZ;
  static constexpr int NFF = FX * FY * FZ;
  static constexpr int S[3] = {1, FX, FX * FY};  // LDS strides of the face-field tile
  static_assert(BX * BY * BZ == 256, "one face per thread");
};

__device__ __forceinline__ int wrapmod(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

template <int DIR>
__device__ __forceinline__ int gcomp_local(int local) {
  return (local == 0 || local == 4) ? local : 1 + (DIR + local - 1) % 3;
}

template <typename T, int DIR, bool STAGE2, bool VAR_MU>
__device__ __forceinline__ void flux_fused_body(const Geo& g, const double* __restrict__ q, T* __restrict__ fl,
                                                int ntx, int nty, int ntz, int nper) {
  using TG = TileGeom<DIR>;
  __shared__ T ff[10 * TG::NFF];
  // XCD-aware tile order: block b runs on XCD b % 8 and takes tile (b % 8) * nper + b / 8
  const int tile = int(blockIdx.x % 8u) * nper + int(blockIdx.x / 8u);
  const int ntiles = ntx * nty * ntz;
  if (tile >= ntiles) return;
  const int x0 = (tile % ntx) * TG::BX;
  const int y0 = ((tile / ntx) % nty) * TG::BY;
  const int z0 = (tile / (ntx * nty)) * TG::BZ;
  const int tid = threadIdx.x;

  // ---- phase 1: face field of the tile and its tangential halo
  const int Nn = g.n[DIR];
  const long long sn = g.stride[DIR];
  for (int e = tid; e < TG::NFF; e += 256) {
    const int ex = e % TG::FX, ey = (e / TG::FX) % TG::FY, ez = e / (TG::FX * TG::FY);
    int c[3] = {wrapmod(x0 + ex - TG::HX, g.n[0]), wrapmod(y0 + ey - TG::HY, g.n[1]),
                wrapmod(z0 + ez - TG::HZ, g.n[2])};
    const int nn = c[DIR];
    const long long base = (long long)c[0] + (long long)c[1] * g.stride[1] + (long long)c[2] * g.stride[2] -
                           (long long)nn * sn;
    long long off[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) off[m] = base + (long long)wrapi(nn - 2 + m, Nn) * sn;
    T Ql[5], Qr[5], Dn[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double* f = q + (long long)gcomp_local<DIR>(k) * g.N;
      const double ref = k == 0 ? g.rho_ref : (k == 4 ? g.E_ref : 0.0);
      T v0 = T(f[off[0]] - ref), v1 = T(f[off[1]] - ref), v2 = T(f[off[2]] - ref);
      T v3 = T(f[off[3]] - ref), v4 = T(f[off[4]] - ref), v5 = T(f[off[5]] - ref);
      Ql[k] = (T(2) * v0 - T(13) * v1 + T(47) * v2 + T(27) * v3 - T(3) * v4) * T(1.0 / 60.0);
      Qr[k] = (T(-3) * v1 + T(27) * v2 + T(47) * v3 - T(13) * v4 + T(2) * v5) * T(1.0 / 60.0);
      Dn[k] = (v1 - T(15) * v2 + T(15) * v3 - v4) * T(g.inv_h[DIR] * (1.0 / 12.0));
    }
    T Q0[5];
    compat_dev(g, Ql, Qr, Q0);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      ff[k * TG::NFF + e] = Q0[k];
      ff[(5 + k) * TG::NFF + e] = Dn[k];
    }
  }
  __syncthreads();

  // ---- phase 2: Gauss-point reconstruction and flux of this thread's face
  const int fx = tid % TG::BX, fy = (tid / TG::BX) % TG::BY, fz = tid / (TG::BX * TG::BY);
  const int gx = x0 + fx, gy = y0 + fy, gz = z0 + fz;
  if (gx >= g.n[0] || gy >= g.n[1] || gz >= g.n[2]) return;
  constexpr int A1 = (DIR + 1) % 3, A2 = (DIR + 2) % 3;
  constexpr int s1 = TG::S[A1], s2 = TG::S[A2];
  const int centre = (fx + TG::HX) + (fy + TG::HY) * TG::FX + (fz + TG::HZ) * TG::FX * TG::FY;
  const int corner = centre - 2 * s1 - 2 * s2;
  const T i1 = T(g.inv_h[A1]), i2 = T(g.inv_h[A2]);
  T Fs[5] = {0, 0, 0, 0, 0}, dFs[5] = {0, 0, 0, 0, 0};
#pragma unroll 1
  for (int m = 0; m < 2; ++m) {  // t1 Gauss point (-, +)
    T Qg[2][5], Dg[2][3][5];
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
        T line[5], lined[5];
#pragma unroll
        for (int a = 0; a < 5; ++a) {
          line[a] = f0[a * s1 + r * s2];
          lined[a] = fn[a * s1 + r * s2];
        }
        T vm, vp, dm, dp, nm, np;
        tang_val(line, vm, vp);
        tang_der(line, dm, dp);
        tang_val(lined, nm, np);
        rv[r] = m ? vp : vm;
        rd[r] = m ? dp : dm;
        rn[r] = m ? np : nm;
      }
      T vm, vp, d2m, d2p, d1m, d1p, nm, np;
      tang_val(rv, vm, vp);
      tang_der(rv, d2m, d2p);
      tang_val(rd, d1m, d1p);
      tang_val(rn, nm, np);
      Qg[0][k] = vm;          Qg[1][k] = vp;
      Dg[0][0][k] = nm;       Dg[1][0][k] = np;
      Dg[0][1][k] = d1m * i1; Dg[1][1][k] = d1p * i1;
      Dg[0][2][k] = d2m * i2; Dg[1][2][k] = d2p * i2;
    }
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      T F[5], dF[5];
      smooth_flux<!STAGE2, VAR_MU>(g, Qg[l], Dg[l], F, dF);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        if (!STAGE2) Fs[k] += F[k];
        dFs[k] += dF[k];
      }
    }
  }
  const long long idx = (long long)gx + (long long)gy * g.stride[1] + (long long)gz * g.stride[2];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int gk = gcomp_local<DIR>(k);
    if (!STAGE2) fl[(long long)gk * g.N + idx] = T(0.25) * Fs[k];
    fl[(long long)(5 + gk) * g.N + idx] = T(0.25) * dFs[k];
  }
}

// Waves per SIMD requested from the register allocator for the constant-viscosity
// kernels (the variable-viscosity ones keep the default: capping them spills).
#ifndef HGKS_FLUX_WAVES
#define HGKS_FLUX_WAVES 3
#endif
#ifndef HGKS_FLUX_WAVES_F32
#define HGKS_FLUX_WAVES_F32 5
#endif

template <typename T, int DIR, bool STAGE2>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? HGKS_FLUX_WAVES : HGKS_FLUX_WAVES_F32)))
flux_fused_kernel(Geo g, const double* __restrict__ q, T* __restrict__ fl, const int* __restrict__ stop, int ntx,
                  int nty, int ntz, int nper) {
  if (*stop) return;
  flux_fused_body<T, DIR, STAGE2, false>(g, q, fl, ntx, nty, ntz, nper);
}

template <typename T, int DIR>
__global__ void __launch_bounds__(256) flux_fused_varmu_kernel(Geo g, const double* __restrict__ q,
                                                               T* __restrict__ fl, const int* __restrict__ stop,
                                                               int ntx, int nty, int ntz, int nper) {
  if (*stop) return;
  flux_fused_body<T, DIR, false, true>(g, q, fl, ntx, nty, ntz, nper);
}

template <typename T, int DIR, bool STAGE2, bool VAR_MU>
static void launch_dir(const Geo& g, const double* q, T* fl, const int* stop, hipStream_t st) {
  using TG = TileGeom<DIR>;
  const int ntx = (g.n[0] + TG::BX - 1) / TG::BX;
  const int nty = (g.n[1] + TG::BY - 1) / TG::BY;
  const int ntz = (g.n[2] + TG::BZ - 1) / TG::BZ;
  const int ntiles = ntx * nty * ntz;
  const int nper = (ntiles + 7) / 8;
  if (VAR_MU)
    flux_fused_varmu_kernel<T, DIR><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, fl, stop, ntx, nty, ntz, nper);
  else
    flux_fused_kernel<T, DIR, STAGE2><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, fl, stop, ntx, nty, ntz, nper);
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
