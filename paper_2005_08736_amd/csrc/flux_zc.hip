// Fused face-flux kernel of mode Z with WENO-Z in characteristic variables (the
// Remark of Sec. 2.1 on non-smooth flows: the reconstruction works on
// omega = R^{-1} Q, R the right eigenvectors of the Jacobian of the face-normal
// Euler flux, and returns to Q by R), one face direction per launch, for gfx950.
//
// Eigenvectors.  Normal reconstruction of a face: at the mean of the face's two
// cells.  Tangential reconstruction of a face: at the face's own equilibrium
// state Q0, shared by its four Gauss points and by every field group (Q0, dQ0/dn,
// Q_l, Q_r and the normal slopes of Q_l, Q_r).
//
// A workgroup of 256 threads owns 8 x 8 faces of direction DIR:
//   1. face field of the tile and a two-face halo (12 x 12 entries, 30 fields)
//      into LDS, the normal WENO-Z done on the six cells' characteristic
//      variables;
//   2. per field group, for every face of the tile and every one of its five t2
//      rows: the five t1-neighbours projected with the face's left eigenvectors,
//      and the WENO-Z edge values of each characteristic component's line, into
//      LDS (the projection depends on the face, so lines are not shared between
//      faces);
//   3. per Gauss point (four lanes per face): parabolas through each line's
//      average and edges at the t1 point, WENO-Z across the five rows in t2 and a
//      second parabola, back to conservative variables with the face's right
//      eigenvectors; the full flux of Eq. (flux) follows as in mode Z.
// The field groups are reconstructed in the order the flux consumes them (the
// three states, then each side's slopes just before that side), one LDS pass
// each.
#include "internal.hpp"
#include "ztile.hpp"

namespace hgks {

// Eigen-structure of the normal Euler-flux Jacobian at a local-frame state given
// as a deviation from the reference state.  With q^2 = u^2 + v^2 + w^2,
// b1 = (gamma - 1)/c^2, b2 = q^2 b1 / 2, the left eigenvectors (rows of R^{-1})
// applied to x give, with s = b1 (u x1 + v x2 + w x3 - x4) and d = (u x0 - x1)/c,
//   w0 = (b2 x0 - s + d)/2,  w1 = (1 - b2) x0 + s,  w2 = x2 - v x0,
//   w3 = x3 - w x0,          w4 = (b2 x0 - s - d)/2,
// and the right eigenvectors (columns for u - c, u, u, u, u + c) map back:
//   x0 = w0 + w1 + w4,  x1 = u x0 - c (w0 - w4),  x2 = v x0 + w2,  x3 = w x0 + w3,
//   x4 = H (w0 + w4) - u c (w0 - w4) + q^2/2 w1 + v w2 + w w3.
template <typename T>
struct ZEig {
  T u, v, w, c, ic, H, b1, b2, hq2;
};

template <typename T>
__device__ __forceinline__ ZEig<T> zeig(const Geo& g, const T* dQ) {
  ZEig<T> e;
  const T rho = T(g.rho_ref) + dQ[0];
  const T ir = recip(rho);
  e.u = dQ[1] * ir;
  e.v = dQ[2] * ir;
  e.w = dQ[3] * ir;
  e.hq2 = T(0.5) * (e.u * e.u + e.v * e.v + e.w * e.w);
  const T p = T(g.p_ref) + T(g.gm1) * (dQ[4] - rho * e.hq2);
  const T c2 = T(g.gamma) * p * ir;
  e.c = sqrt(c2);
  e.ic = recip(e.c);
  e.H = (T(g.E_ref) + dQ[4] + p) * ir;
  e.b1 = T(g.gm1) * recip(c2);
  e.b2 = e.hq2 * e.b1;
  return e;
}

template <typename T>
__device__ __forceinline__ void zleft(const ZEig<T>& e, const T* x, T* w) {
  const T s = e.b1 * (e.u * x[1] + e.v * x[2] + e.w * x[3] - x[4]);
  const T d = (e.u * x[0] - x[1]) * e.ic;
  const T b = e.b2 * x[0] - s;
  w[0] = T(0.5) * (b + d);
  w[1] = x[0] - e.b2 * x[0] + s;
  w[2] = x[2] - e.v * x[0];
  w[3] = x[3] - e.w * x[0];
  w[4] = T(0.5) * (b - d);
}

template <typename T>
__device__ __forceinline__ void zright(const ZEig<T>& e, const T* w, T* x) {
  const T sum = w[0] + w[4], dif = w[0] - w[4];
  const T x0 = sum + w[1];
  x[0] = x0;
  x[1] = e.u * x0 - e.c * dif;
  x[2] = e.v * x0 + w[2];
  x[3] = e.w * x0 + w[3];
  x[4] = e.H * sum - e.u * e.c * dif + e.hq2 * w[1] + e.v * w[2] + e.w * w[3];
}

// The eigen-structure of each of the tile's 64 faces, kept in LDS (nine values a
// face) once phase 1 has written Q0: every line job of phase 2 reads its face's.
constexpr int kZEigVals = 9;
template <typename T>
__device__ __forceinline__ void zeig_store(const ZEig<T>& e, T* p) {
  p[0] = e.u; p[1] = e.v; p[2] = e.w; p[3] = e.c; p[4] = e.ic; p[5] = e.H; p[6] = e.b1; p[7] = e.b2; p[8] = e.hq2;
}
template <typename T>
__device__ __forceinline__ ZEig<T> zeig_load(const T* p) {
  ZEig<T> e;
  e.u = p[0]; e.v = p[1]; e.w = p[2]; e.c = p[3]; e.ic = p[4]; e.H = p[5]; e.b1 = p[6]; e.b2 = p[7]; e.hq2 = p[8];
  return e;
}

// The WENO-Z exponent: WP when it is fixed at compile time (the usual p = 2: 6%
// faster, its kernels carry no branch on the exponent), else the run's parameter.
template <int WP>
__device__ __forceinline__ int zexp(const Geo& g) {
  return WP > 0 ? WP : g.weno_p;
}

// Phase 1: face-field entries; the normal WENO-Z on characteristic variables.
template <typename T, int DIR, int WP>
__device__ __forceinline__ void zcface_field(const Geo& g, const double* __restrict__ q, T* ff, int on, int o1,
                                             int o2) {
  using TG = ZTileGeom<DIR>;
  const int wp = zexp<WP>(g);
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
    T v[6][5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double* f = q + (long long)gcomp_local<DIR>(k) * g.N;
      const double ref = k == 0 ? g.rho_ref : (k == 4 ? g.E_ref : 0.0);
#pragma unroll
      for (int m = 0; m < 6; ++m) v[m][k] = T(f[base + (long long)wrapi(on - 2 + m, Nn) * sn] - ref);
    }
    T Dn[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) Dn[k] = (v[1][k] - T(15) * v[2][k] + T(15) * v[3][k] - v[4][k]) * ih12;
    ZEig<T> ez;
    {
      T mid[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) mid[k] = T(0.5) * (v[2][k] + v[3][k]);
      ez = zeig(g, mid);
    }
    T w[6][5];
#pragma unroll
    for (int m = 0; m < 6; ++m) zleft(ez, v[m], w[m]);
    T wl[5], wr[5], sl[5], sr[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      T line[5] = {w[0][k], w[1][k], w[2][k], w[3][k], w[4][k]};
      weno_z_right(line, eps, wp, wl[k], sl[k]);
      T rline[5] = {w[5][k], w[4][k], w[3][k], w[2][k], w[1][k]};
      weno_z_right(rline, eps, wp, wr[k], sr[k]);
    }
    T Ql[5], Qr[5], Dl[5], Dr[5];
    zright(ez, wl, Ql);
    zright(ez, wr, Qr);
    zright(ez, sl, Dl);
    zright(ez, sr, Dr);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      Dl[k] = Dl[k] * ih;
      Dr[k] = -Dr[k] * ih;
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

// Layout of the per-group line buffer: for face f (t1 fastest) of the tile, t2 row
// r and characteristic component k, the line's middle value and its two WENO-Z
// edge values.
constexpr int kZcLines = 64 * 5 * 5;
__device__ __forceinline__ int zc_line(int face, int r, int k) { return (face * 5 + r) * 5 + k; }

// Phase 2 for one field group (first LDS field f0): lines of the five
// t1-neighbours of every face's five t2 rows, in that face's characteristic
// variables, into lb (320 jobs: two rounds of 256 threads, the second a quarter
// full).  Building two or three groups per pass fills the rounds better but needs
// a line buffer per group; with one buffer the FP64 kernel fits two workgroups
// per CU at two waves per SIMD, which measured 12% faster.
template <typename T, int DIR, int WP>
__device__ __forceinline__ void zc_group_lines(const Geo& g, const T* ff, const T* eg, int f0, T* lb) {
  using TG = ZTileGeom<DIR>;
  const int wp = zexp<WP>(g);
  const T eps = T(g.weno_eps);
  for (int jj = threadIdx.x; jj < 64 * 5; jj += 256) {
    const int face = jj / 5, r = jj % 5;
    const int a = face % TG::B, t = face / TG::B;
    const ZEig<T> ez = zeig_load(eg + face * kZEigVals);
    T w[5][5];  // [t1 position s][component]
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      T x[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) x[k] = ff[(f0 + k) * TG::NFF + (t + r) * TG::P + a + s];
      zleft(ez, x, w[s]);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      T line[5] = {w[0][k], w[1][k], w[2][k], w[3][k], w[4][k]};
      T ea, eb;
      weno_z_edges(line, eps, wp, ea, eb);
      const int li = zc_line(face, r, k);
      lb[3 * li] = w[2][k];
      lb[3 * li + 1] = ea;
      lb[3 * li + 2] = eb;
    }
  }
}

// Phase 3 for one field group at this lane's Gauss point: value, t2-derivative
// and (with T1DER) t1-derivative, in conservative variables.
//
// The WENO-Z edges across the five t2 rows depend on the t1 Gauss point only,
// so the two lanes of a face with the same t1 point (adjacent lanes, sl = -1 and
// +1) split them: of the group's jobs (the five components' value rows, and with
// T1DER their t1-derivative rows) each lane evaluates every other one and the
// pair swaps edges with a lane shuffle.  The arithmetic of each job is the same
// on either lane, so the results do not depend on the split.
template <typename T, int DIR, bool T1DER, int WP>
__device__ __forceinline__ void zc_group_gp(const Geo& g, const T* lb, const ZEig<T>& ez, int face, T sm, T sl,
                                            T* val, T* d1, T* d2) {
  using TG = ZTileGeom<DIR>;
  const int wp = zexp<WP>(g);
  const T eps = T(g.weno_eps);
  constexpr int J = T1DER ? 10 : 5;  // job j: component j % 5, t1-derivative rows if j >= 5
  const int mine = sl > T(0) ? 1 : 0;
  // row r of job j at this lane's t1 point
  auto row = [&](int j, int r) {
    const int li = zc_line(face, r, j % 5);
    const T m = lb[3 * li], ea = lb[3 * li + 1], eb = lb[3 * li + 2];
    return j >= 5 ? zpar_der(m, ea, eb, sm) : zpar_val(m, ea, eb, sm);
  };
  T wv[5], w1[5], w2[5];
#pragma unroll
  for (int s2 = 0; s2 < (J + 1) / 2; ++s2) {
    const int j0 = 2 * s2, j1 = (2 * s2 + 1 < J) ? 2 * s2 + 1 : 2 * s2;  // an odd count repeats the last job
    const int jo = mine ? j1 : j0;                                       // this lane's job
    T rv[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) rv[r] = row(jo, r);
    T ea, eb;
    weno_z_edges(rv, eps, wp, ea, eb);
    const T pa = __shfl_xor(ea, 1), pb = __shfl_xor(eb, 1);
    // edges of j0 and j1 on both lanes
    const T ea0 = mine ? pa : ea, eb0 = mine ? pb : eb;
    const T ea1 = mine ? ea : pa, eb1 = mine ? eb : pb;
    const T m0 = row(j0, 2), m1 = row(j1, 2);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int jj = h ? j1 : j0;
      if (h && j1 == j0) continue;
      const T m = h ? m1 : m0, a = h ? ea1 : ea0, b = h ? eb1 : eb0;
      if (jj < 5) {
        wv[jj] = zpar_val(m, a, b, sl);
        w2[jj] = zpar_der(m, a, b, sl);
      } else {
        w1[jj - 5] = zpar_val(m, a, b, sl);
      }
    }
  }
  zright(ez, wv, val);
  zright(ez, w2, d2);
  const T i2 = T(g.inv_h[TG::A2]);
#pragma unroll
  for (int k = 0; k < 5; ++k) d2[k] = d2[k] * i2;
  if (T1DER) {
    zright(ez, w1, d1);
    const T i1 = T(g.inv_h[TG::A1]);
#pragma unroll
    for (int k = 0; k < 5; ++k) d1[k] = d1[k] * i1;
  }
}

template <typename T, int DIR, bool STAGE2, bool VAR_MU, int WP>
__device__ __forceinline__ void flux_zc_body(const Geo& g, const double* __restrict__ q, T* __restrict__ fl,
                                             const double* __restrict__ dtp, int nt1, int nt2, int nper) {
  using TG = ZTileGeom<DIR>;
  static_assert(TG::B * TG::B * 4 == 256, "four lanes per face");
  // one field group's lines per pass (a single line buffer): 76 KB of LDS in
  // FP64, two workgroups per CU; 39 KB in FP32, three
  __shared__ T ff[TG::NF * TG::NFF];
  __shared__ T lb[3 * kZcLines];
  __shared__ T eg[64 * kZEigVals];
  const int tile = tile_of_block(nper);
  const int Nn = g.n[DIR];
  if (tile >= Nn * nt1 * nt2) return;  // whole workgroup leaves together
  int on, o1, o2;
  zflux_tile_origin<DIR>(tile, Nn, nt1, nt2, on, o1, o2);

  zcface_field<T, DIR, WP>(g, q, ff, on, o1, o2);
  __syncthreads();

  const int tid = threadIdx.x;
  const int face = tid >> 2, gp = tid & 3;
  const int a = face % TG::B, t = face / TG::B;
  const T sm = (gp & 2) ? T(1) : T(-1);  // t1 Gauss point
  const T sl = (gp & 1) ? T(1) : T(-1);  // t2 Gauss point
  const T dt = T(*dtp);
  const T K = T(g.K);
  ZEig<T> ez;
  {
    T q0[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) q0[k] = ff[(kZQ0 + k) * TG::NFF + (t + 2) * TG::P + a + 2];
    ez = zeig(g, q0);
    if (gp == 0) zeig_store(ez, eg + face * kZEigVals);
  }
  __syncthreads();
  // the three states first (the collision time needs them); each side's
  // tangential derivatives are reconstructed again just before that side, which
  // keeps fewer values live than holding them from the first pass
  ZFold<T> c;
  {
    T Ql[5], Qr[5], Q0[5], unused[5];
    const int fs[3] = {kZQl, kZQr, kZQ0};
    T* out[3] = {Ql, Qr, Q0};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (i > 0) __syncthreads();  // the previous group's lines have been read
      zc_group_lines<T, DIR, WP>(g, ff, eg, fs[i], lb);
      __syncthreads();
      zc_group_gp<T, DIR, false, WP>(g, lb, ez, face, sm, sl, out[i], unused, unused);
    }
    zfold_begin<VAR_MU>(g, Q0, Ql, Qr, dt, c);
  }
  ZOut<T> o;
#pragma unroll 1
  for (int side = 0; side < 3; ++side) {
    const int fs = side == 0 ? kZQ0 : (side == 1 ? kZQl : kZQr);
    const int fd = side == 0 ? kZDn : (side == 1 ? kZDl : kZDr);
    T D[3][5], unused[5];
    __syncthreads();  // the previous pass's lines have been read
    zc_group_lines<T, DIR, WP>(g, ff, eg, fs, lb);
    __syncthreads();
    zc_group_gp<T, DIR, true, WP>(g, lb, ez, face, sm, sl, unused, D[1], D[2]);
    __syncthreads();
    zc_group_lines<T, DIR, WP>(g, ff, eg, fd, lb);
    __syncthreads();
    zc_group_gp<T, DIR, false, WP>(g, lb, ez, face, sm, sl, D[0], unused, unused);
    zfold_side(c, side, D, K, dt, o);
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
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int gk = gcomp_local<DIR>(k);
    if (!STAGE2 && (k & 3) == gp) fl[(long long)gk * g.N + idx] = T(0.25) * F[k];
    if (((k + 5) & 3) == gp) fl[(long long)(5 + gk) * g.N + idx] = T(0.25) * dF[k];
  }
}

// FP64 runs two waves per SIMD (256 VGPRs, with spills): 12% faster at 256^3 than
// one wave per SIMD holding three line buffers and spilling into AGPRs; the FP32
// form fits three
#ifndef HGKS_ZCWAVES_F64
#define HGKS_ZCWAVES_F64 2
#endif
#ifndef HGKS_ZCWAVES_F32
#define HGKS_ZCWAVES_F32 3
#endif
// WP: the WENO-Z exponent fixed at compile time (2), or 0 for the run's parameter
template <typename T, int DIR, bool STAGE2, bool VAR_MU, int WP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? HGKS_ZCWAVES_F64 : HGKS_ZCWAVES_F32)))
flux_zc_kernel(Geo g, const double* __restrict__ q, T* __restrict__ fl, const int* __restrict__ stop,
               const double* __restrict__ dtp, int nt1, int nt2, int nper) {
  if (*stop) return;
  flux_zc_body<T, DIR, STAGE2, VAR_MU, WP>(g, q, fl, dtp, nt1, nt2, nper);
}

template <typename T, int DIR, bool STAGE2, bool VAR_MU>
static void launch_zc_dir(const Geo& g, const double* q, T* fl, const int* stop, const double* dtp, hipStream_t st) {
  using TG = ZTileGeom<DIR>;
  const int nt1 = (g.n[TG::A1] + TG::B - 1) / TG::B;
  const int nt2 = (g.n[TG::A2] + TG::B - 1) / TG::B;
  const int tiles = g.n[DIR] * nt1 * nt2;
  const int nper = (tiles + 7) / 8;
  if (g.weno_p == 2)
    flux_zc_kernel<T, DIR, STAGE2, VAR_MU, 2><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, fl, stop, dtp,
                                                                                             nt1, nt2, nper);
  else
    flux_zc_kernel<T, DIR, STAGE2, VAR_MU, 0><<<dim3(unsigned(8 * nper)), dim3(256), 0, st>>>(g, q, fl, stop, dtp,
                                                                                             nt1, nt2, nper);
}

template <typename T, bool STAGE2, bool VAR_MU>
static void launch_zc_any(const Geo& g, int dir, const double* q, T* fl, const int* stop, const double* dtp,
                          hipStream_t st) {
  if (dir == 0) launch_zc_dir<T, 0, STAGE2, VAR_MU>(g, q, fl, stop, dtp, st);
  else if (dir == 1) launch_zc_dir<T, 1, STAGE2, VAR_MU>(g, q, fl, stop, dtp, st);
  else launch_zc_dir<T, 2, STAGE2, VAR_MU>(g, q, fl, stop, dtp, st);
}

template <typename T>
static void launch_zc_t(const Geo& g, int dir, bool stage2, const double* q, T* fl, const int* stop,
                        const double* dtp, hipStream_t st) {
  const bool var_mu = g.mu_exp != 0.0;
  if (stage2) {
    if (var_mu) launch_zc_any<T, true, true>(g, dir, q, fl, stop, dtp, st);
    else launch_zc_any<T, true, false>(g, dir, q, fl, stop, dtp, st);
  } else {
    if (var_mu) launch_zc_any<T, false, true>(g, dir, q, fl, stop, dtp, st);
    else launch_zc_any<T, false, false>(g, dir, q, fl, stop, dtp, st);
  }
}

void launch_flux_zc(const Geo& g, int dir, bool stage2, const double* q, double* fl, const int* stop,
                    const double* dtp, hipStream_t st) {
  launch_zc_t<double>(g, dir, stage2, q, fl, stop, dtp, st);
}

void launch_flux_zc(const Geo& g, int dir, bool stage2, const double* q, float* fl, const int* stop,
                    const double* dtp, hipStream_t st) {
  launch_zc_t<float>(g, dir, stage2, q, fl, stop, dtp, st);
}

}  // namespace hgks
