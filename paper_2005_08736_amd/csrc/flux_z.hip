// Fused face-flux kernel of the WENO-Z / full-flux mode (mode Z), one face
// direction per launch, LDS-tiled for gfx950.
//
// A workgroup of 256 threads owns 8 x 8 faces of direction DIR (one face thick
// along the normal) and works in three phases:
//   1. face field of the tile and a two-face halo in both tangential axes
//      (12 x 12 entries) into LDS: for each conservative component, the WENO-Z
//      values Q_l, Q_r and slopes dQ_l/dn, dQ_r/dn from the six cells along the
//      normal, the equilibrium state Q0 by the compatibility condition and dQ0/dn
//      (Sec. 2.1): 30 fields;
//   2. WENO-Z edge values, along t1, of the middle face of every five-face t1
//      line centred on a tile column (8 x 12 lines per field) into LDS;
//   3. one thread per Gauss point (4 per face): the parabola through each line's
//      average and edge values gives the line's value and t1-derivative at the
//      t1 Gauss point; WENO-Z across the five lines in t2 and a second parabola
//      give the field's value and both tangential derivatives at the Gauss point
//      (60 values), from which the full gas distribution of Eq. (flux), integrated
//      over dt and dt/2, gives F^n and dF^n/dt (Eq. (expansion-1)).  The four
//      Gauss points of a face sit in adjacent lanes and are summed with shuffles.
// Tiles are dealt to the XCDs in contiguous ranges, in the order of
// zflux_tile_origin (ztile.hpp).
#include "internal.hpp"
#include "ztile.hpp"

namespace hgks {

template <typename T, int DIR, bool STAGE2, bool VAR_MU, bool RECOMP>
__device__ __forceinline__ void flux_z_body(const Geo& g, const double* __restrict__ q, T* __restrict__ fl,
                                            const double* __restrict__ dtp, int nt1, int nt2, int nper) {
  using TG = ZTileGeom<DIR>;
  __shared__ T ff[TG::NF * TG::NFF];
  __shared__ T ed[2 * TG::NF * TG::NROW];
  const int tile = tile_of_block(nper);
  const int Nn = g.n[DIR];
  if (tile >= Nn * nt1 * nt2) return;  // whole workgroup leaves together
  int on, o1, o2;
  zflux_tile_origin<DIR>(tile, Nn, nt1, nt2, on, o1, o2);

  zface_field<T, DIR>(g, q, ff, on, o1, o2);
  __syncthreads();
  zrow_edges<T, DIR>(g, ff, ed);
  __syncthreads();

  const int tid = threadIdx.x;
  const int face = tid >> 2, gp = tid & 3;
  const int a = face % TG::B, t = face / TG::B;
  const T sm = (gp & 2) ? T(1) : T(-1);  // t1 Gauss point
  const T sl = (gp & 1) ? T(1) : T(-1);  // t2 Gauss point
  const T dt = T(*dtp);
  const T K = T(g.K);
  T dum, tok = T(0);
  // Values of Q_l, Q_r and Q0 first: the collision time needs them (the two
  // Gauss points with the same t1 point split each pair of WENO-Z edge
  // evaluations between them, zgp_pair).  The sides' values and t2-derivatives
  // are either held from here through the side loop with the three sides'
  // primitive states (RECOMP = false), or evaluated again in each side's trip by
  // the same calls, which give the same bits (RECOMP = true): three more WENO-Z
  // edge evaluations per lane and side for 200 B less scratch per lane.
  T Ql[5], Qr[5], Q0[5], Ql2[5], Qr2[5], Q02[5];
#pragma unroll
  for (int k = 0; k < 5; ++k)
    zgp_pair<T, DIR, false>(g, ff, ed, kZQl + k, kZQr + k, a, t, sm, sl, Ql[k], Ql2[k], Qr[k], Qr2[k], tok);
  zgp_pair<T, DIR, false>(g, ff, ed, kZQ0 + 0, kZQ0 + 1, a, t, sm, sl, Q0[0], Q02[0], Q0[1], Q02[1], tok);
  zgp_pair<T, DIR, false>(g, ff, ed, kZQ0 + 2, kZQ0 + 3, a, t, sm, sl, Q0[2], Q02[2], Q0[3], Q02[3], tok);
  zgp_field<T, DIR, false>(g, ff, ed, kZQ0 + 4, a, t, sm, sl, Q0[4], dum, Q02[4], tok);
  ZFold<T> c;
  zfold_begin<VAR_MU>(g, Q0, Ql, Qr, dt, c);
  const T U0 = c.s0.U, V0 = c.s0.V, W0 = c.s0.W;
  ZOut<T> o;
  // one side per trip of a loop that is not unrolled: the scheduler cannot
  // overlap one side's reconstruction with another side's moments, and a single
  // copy of the side's code holds its temporaries
#pragma unroll 1
  for (int side = 0; side < 3; ++side) {
    // the side's LDS reads wait for the previous side's result
    int aa = a;
    if (side > 0) zdep(aa, o.F[4]);
    const int fd = side == 0 ? kZDn : (side == 1 ? kZDl : kZDr);
    const int fs = side == 0 ? kZQ0 : (side == 1 ? kZQl : kZQr);
    T D[3][5];
    ZPrim<T> sp;
    if (!RECOMP) {
      sp = side == 0 ? c.s0 : (side == 1 ? c.sl : c.sr);
#pragma unroll
      for (int k = 0; k < 5; ++k) D[2][k] = side == 0 ? Q02[k] : (side == 1 ? Ql2[k] : Qr2[k]);
    } else {
      T Qs[5];
      if (side == 0) {
        zgp_pair<T, DIR, false>(g, ff, ed, fs + 0, fs + 1, aa, t, sm, sl, Qs[0], D[2][0], Qs[1], D[2][1], tok);
        zgp_pair<T, DIR, false>(g, ff, ed, fs + 2, fs + 3, aa, t, sm, sl, Qs[2], D[2][2], Qs[3], D[2][3], tok);
        zgp_field<T, DIR, false>(g, ff, ed, fs + 4, aa, t, sm, sl, Qs[4], dum, D[2][4], tok);
      } else {
        // the fifth field pairs with itself: the same row formula as the first pass
#pragma unroll
        for (int k = 0; k < 5; k += 2) {
          const int k2 = k + 1 < 5 ? k + 1 : k;
          T v2, d2;
          zgp_pair<T, DIR, false>(g, ff, ed, fs + k, fs + k2, aa, t, sm, sl, Qs[k], D[2][k], v2, d2, tok);
          if (k + 1 < 5) {
            Qs[k + 1] = v2;
            D[2][k + 1] = d2;
          }
        }
      }
      sp = zprim(g, Qs);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k)
      zgp_pair<T, DIR, true>(g, ff, ed, fd + k, fs + k, aa, t, sm, sl, D[0][k], dum, D[1][k], dum, tok);
    T kF[3], kD[3];
    zfd_coef(dt, c.tau, c.e1, c.eh, side == 0, kF, kD);
    zside_fold(sp, D, side == 0 ? 0 : (side == 1 ? +1 : -1), K, kF, kD, U0, V0, W0, o, side == 0);
  }
  T F[5], dF[5];
  zfold_end(g, o, F, dF);
  // sum of the four Gauss points (adjacent lanes), face average = sum / 4
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    F[k] += __shfl_xor(F[k], 1);
    F[k] += __shfl_xor(F[k], 2);
    dF[k] += __shfl_xor(dF[k], 1);
    dF[k] += __shfl_xor(dF[k], 2);
  }
  int cc[3];
  cc[DIR] = on;
  cc[TG::A1] = o1 + a;
  cc[TG::A2] = o2 + t;
  if (cc[TG::A1] >= g.n[TG::A1] || cc[TG::A2] >= g.n[TG::A2]) return;
  const long long idx = (long long)cc[0] + (long long)cc[1] * g.stride[1] + (long long)cc[2] * g.stride[2];
  // each lane of the face writes every fourth of its ten outputs
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int gk = gcomp_local<DIR>(k);
    if (!STAGE2 && (k & 3) == gp) fl[(long long)gk * g.N + idx] = T(0.25) * F[k];
    if (((k + 5) & 3) == gp) fl[(long long)(5 + gk) * g.N + idx] = T(0.25) * dF[k];
  }
}

#ifndef HGKS_ZWAVES
#define HGKS_ZWAVES 2
#endif

#ifndef HGKS_ZWAVES_F32
#define HGKS_ZWAVES_F32 4
#endif
template <typename T, int DIR, bool STAGE2, bool VAR_MU>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? HGKS_ZWAVES : HGKS_ZWAVES_F32)))
flux_z_kernel(Geo g, const double* __restrict__ q, T* __restrict__ fl, const int* __restrict__ stop,
              const double* __restrict__ dtp, int nt1, int nt2, int nper) {
  if (*stop) return;
  // side values evaluated again in each side's trip: FP64 stage 1 only (measured
  // faster there; slower in the FP64 stage-2 launch and in the FP32 form, whose
  // spills are smaller or cheaper)
  constexpr bool RECOMP = sizeof(T) == 8 && !STAGE2;
  flux_z_body<T, DIR, STAGE2, VAR_MU, RECOMP>(g, q, fl, dtp, nt1, nt2, nper);
}

template <typename T, int DIR, bool STAGE2, bool VAR_MU>
static void launch_z_dir(const Geo& g, const double* q, T* fl, const int* stop, const double* dtp, hipStream_t st) {
  using TG = ZTileGeom<DIR>;
  const int nt1 = (g.n[TG::A1] + TG::B - 1) / TG::B;
  const int nt2 = (g.n[TG::A2] + TG::B - 1) / TG::B;
  const int tiles = g.n[DIR] * nt1 * nt2;
  const int nper = (tiles + 7) / 8;
  flux_z_kernel<T, DIR, STAGE2, VAR_MU><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, fl, stop, dtp, nt1,
                                                                                      nt2, nper);
}

template <typename T, bool STAGE2, bool VAR_MU>
static void launch_z_any(const Geo& g, int dir, const double* q, T* fl, const int* stop, const double* dtp,
                         hipStream_t st) {
  if (dir == 0) launch_z_dir<T, 0, STAGE2, VAR_MU>(g, q, fl, stop, dtp, st);
  else if (dir == 1) launch_z_dir<T, 1, STAGE2, VAR_MU>(g, q, fl, stop, dtp, st);
  else launch_z_dir<T, 2, STAGE2, VAR_MU>(g, q, fl, stop, dtp, st);
}

template <typename T>
static void launch_z_t(const Geo& g, int dir, bool stage2, const double* q, T* fl, const int* stop, const double* dtp,
                       hipStream_t st) {
  const bool var_mu = g.mu_exp != 0.0;
  if (stage2) {
    if (var_mu) launch_z_any<T, true, true>(g, dir, q, fl, stop, dtp, st);
    else launch_z_any<T, true, false>(g, dir, q, fl, stop, dtp, st);
  } else {
    if (var_mu) launch_z_any<T, false, true>(g, dir, q, fl, stop, dtp, st);
    else launch_z_any<T, false, false>(g, dir, q, fl, stop, dtp, st);
  }
}

void launch_flux_z(const Geo& g, int dir, bool stage2, const double* q, double* fl, const int* stop,
                   const double* dtp, hipStream_t st) {
  launch_z_t<double>(g, dir, stage2, q, fl, stop, dtp, st);
}

void launch_flux_z(const Geo& g, int dir, bool stage2, const double* q, float* fl, const int* stop, const double* dtp,
                   hipStream_t st) {
  launch_z_t<float>(g, dir, stage2, q, fl, stop, dtp, st);
}

}  // namespace hgks
