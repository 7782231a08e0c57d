// Stage kernels of the HGKS update for gfx950: the divergence of the face fluxes
// (Eq. (finite)), the two-stage formula of Eq. (two-stage), the CFL speed
// reduction and the physicality check of each new state.  The face fluxes come
// from flux_fused.hip.
#include "internal.hpp"

namespace hgks {

template <int DIR>
__device__ __forceinline__ void cell_coords(const Geo& g, long long idx, int* c) {
  c[0] = int(idx % g.n[0]);
  long long r = idx / g.n[0];
  c[1] = int(r % g.n[1]);
  c[2] = int(r / g.n[1]);
}

// ---------------------------------------------------------------------------
// Stage updates.
// ---------------------------------------------------------------------------
// 1/width of row j along y (the row height on a stretched mesh)
__device__ __forceinline__ double inv_width_y(const Geo& g, int j) {
  return g.stretch_y ? ym_inv_dy(g, j) : g.inv_h[1];
}

// max over axes of (|U_d| + c)/dx_d of a cell in row j, and whether the state is physical
__device__ __forceinline__ double cell_speed(const Geo& g, const double* Q, int j, bool& ok) {
  double ir = 1.0 / Q[0];
  double U = Q[1] * ir, V = Q[2] * ir, W = Q[3] * ir;
  double p = g.gm1 * (Q[4] - 0.5 * Q[0] * (U * U + V * V + W * W));
  ok = (Q[0] > 0.0) && (p > 0.0) && isfinite(p) && isfinite(Q[0]);
  double c = sqrt(g.gamma * p * ir);
  double s = (fabs(U) + c) * g.inv_h[0];
  s = fmax(s, (fabs(V) + c) * inv_width_y(g, j));
  s = fmax(s, (fabs(W) + c) * g.inv_h[2]);
  return s;
}

// face below cell c along direction d: its array and index (the bottom wall face
// of the channel lives in its own array, component stride nx nz)
template <typename TF>
__device__ __forceinline__ const TF* lower_face(const Geo& g, const TF* F, long long idx, const int* c, int d,
                                                long long& lo, long long& cs) {
  cs = g.N;
  if (c[d] > 0) {
    lo = idx - g.stride[d];
    return F;
  }
  if (d == 1 && g.wall_y) {
    lo = (long long)c[0] + (long long)c[2] * g.n[0];
    cs = (long long)g.n[0] * g.n[2];
    return static_cast<const TF*>(g.fwall);
  }
  lo = idx + (long long)(g.n[d] - 1) * g.stride[d];
  return F;
}

// block maximum of v (256 threads) written to part[blockIdx.x]
__device__ __forceinline__ void block_max_speed(double v, double* part) {
  __shared__ double wmax[4];
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
}

// -(1/|Omega|) sum_p F_p for component k (Eq. (finite)) from the face averages of
// the three directions (face n+1/2 stored at cell n), and the same for dF/dt.
__device__ __forceinline__ void divergence(const Geo& g, const double* fl, long long idx, const int* c, int k,
                                           double* L, double* dL) {
  double l = 0.0, dl = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double* F = fl + (long long)d * 10 * g.N;
    long long lo, cs;
    const double* Fl = lower_face(g, F, idx, c, d, lo, cs);
    const double ih = d == 1 ? inv_width_y(g, c[1]) : g.inv_h[d];
    if (L) l -= (F[(long long)k * g.N + idx] - Fl[(long long)k * cs + lo]) * ih;
    dl -= (F[(long long)(5 + k) * g.N + idx] - Fl[(long long)(5 + k) * cs + lo]) * ih;
  }
  if (L) *L = l;
  *dL = dl;
}

// FP32 face fluxes (FP32-flux form): each difference of two neighbouring faces
// and its scaling by 1/h are split exactly into FP32 pieces (TwoSum for the
// difference, an FMA for the product's rounding error), and the pieces of the
// three directions are summed with compensation: every addition is a TwoSum
// whose rounding error is collected in a second FP32 word (the summation of
// Neumaier / Ogita-Rump-Oishi).  The error is then bounded by the precision of
// the result itself, not by the size of the cancelling terms, and the FP64
// update receives hi + lo, so the face contributions telescope over the box.
// Contraction into FMAs is switched off in these helpers: fusing a product into
// the compensated additions would add a value other than the one the error
// terms account for.
struct Kahan {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float t) {
#pragma clang fp contract(off)
    const float u = s + t;
    const float v = u - s;
    c += (s - (u - v)) + (t - v);  // TwoSum error of s + t
    s = u;
  }
  __device__ __forceinline__ double value() const { return double(s) + double(c); }
};

// adds -(a - b) * ih to acc without losing the rounding errors of - and *
__device__ __forceinline__ void add_neg_scaled_diff(Kahan& acc, float a, float b, float ih) {
#pragma clang fp contract(off)
  const float d = a - b;                  // TwoSum of a and -b: a - b = d + e exactly
  const float v = d - a;
  const float e = (a - (d - v)) + (-b - v);
  const float p = d * ih;
  const float pe = fmaf(d, ih, -p);       // d * ih = p + pe exactly
  acc.add(-p);
  acc.add(-pe);
  acc.add(-(e * ih));
}

__device__ __forceinline__ void divergence(const Geo& g, const float* fl, long long idx, const int* c, int k,
                                           double* L, double* dL) {
  Kahan l, dl;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float* F = fl + (long long)d * 10 * g.N;
    long long lo, cs;
    const float* Fl = lower_face(g, F, idx, c, d, lo, cs);
    const float ih = float(d == 1 ? inv_width_y(g, c[1]) : g.inv_h[d]);
    if (L) add_neg_scaled_diff(l, F[(long long)k * g.N + idx], Fl[(long long)k * cs + lo], ih);
    add_neg_scaled_diff(dl, F[(long long)(5 + k) * g.N + idx], Fl[(long long)(5 + k) * cs + lo], ih);
  }
  if (L) *L = l.value();
  *dL = dl.value();
}

// Time step of the step about to start: the maximum of the block maxima of the
// CFL speed left by the previous stage-2 (or state-check) kernel; one block.
__global__ void __launch_bounds__(1024) dt_kernel(Geo g, const double* __restrict__ part, int nparts, Ctrl* ctrl,
                                                  double dt_fixed, int hist) {
  __shared__ double wmax[16];
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 1024) v = fmax(v, part[i]);
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < 16; ++w) m = fmax(m, wmax[w]);
    double dt = dt_fixed > 0.0 ? dt_fixed : g.cfl / m;
    ctrl->maxspeed = m;
    ctrl->dt = dt;
    ctrl->dt_hist[hist] = dt;
  }
}

// Q* = Q^n + dt/2 L + dt^2/8 dL ; R = Q^n + dt L + dt^2/6 dL
template <typename TF>
__global__ void __launch_bounds__(256) stage1_kernel(Geo g, const double* __restrict__ qn, const TF* __restrict__ fl,
                                                     double* __restrict__ qs, double* __restrict__ rr, Ctrl* ctrl,
                                                     int step) {
  if (ctrl->flag) return;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const double dt = ctrl->dt;
  if (idx >= g.N) return;
  int c[3];
  cell_coords<0>(g, idx, c);
  double Qs[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double L, dL;
    divergence(g, fl, idx, c, k, &L, &dL);
    double q0 = qn[(long long)k * g.N + idx];
    Qs[k] = q0 + 0.5 * dt * L + 0.125 * dt * dt * dL;
    qs[(long long)k * g.N + idx] = Qs[k];
    rr[(long long)k * g.N + idx] = q0 + dt * L + (dt * dt / 6.0) * dL;
  }
  bool ok;
  (void)cell_speed(g, Qs, c[1], ok);
  if (!ok) {
    ctrl->fail_step = step;
    ctrl->flag = 1;
  }
}

// fixed-order sums of three values over a 256-thread block, left in out[0..2]
// (LDS or global) by thread 0
__device__ __forceinline__ void block_sums3(double a, double b, double c, double* out) {
  __shared__ double red[3][256];
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
    out[2] = red[2][0];
  }
}

__device__ __forceinline__ double cell_volume(const Geo& g, int j) {
  return g.h[0] * g.h[2] * (g.stretch_y ? ym_dy(g, j) : g.h[1]);
}

// Q^{n+1} = R + dt^2/3 dL(Q*); then the channel's constant body force f_x
// (Sec. 3.3), with the trapezoidal rule over the step:
//   (rho U)^{n+1} += dt/2 (rho^{n+1} + rho^n) f_x,
//   (rho E)^{n+1} += dt/2 ((rho U)^{n+1} + (rho U)^n) f_x;
// block maxima of the next step's CFL speed.  With BULK (constant bulk momentum)
// the force is left to bulk_force_apply_kernel, and each block writes the sums of
// (rho U)~ V, (rho^n + rho~) V and V over its cells to mpart instead.
template <typename TF, bool BULK>
__global__ void __launch_bounds__(256) stage2_kernel(Geo g, const double* __restrict__ rr, const TF* __restrict__ fl,
                                                     const double* __restrict__ qn, double* __restrict__ qout,
                                                     Ctrl* ctrl, double* __restrict__ part,
                                                     double* __restrict__ mpart, int step) {
  // other blocks of this launch may raise the flag while it runs: the block reads
  // it once, so that all its waves leave together or all reach the reduction
  __shared__ int stop;
  if (threadIdx.x == 0) stop = ctrl->flag;
  __syncthreads();
  if (stop) return;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const double dt = ctrl->dt;
  double speed = 0.0, sm = 0.0, ss = 0.0, sv = 0.0;
  if (idx < g.N) {
    int c[3];
    cell_coords<0>(g, idx, c);
    double Qn[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double dL;
      divergence(g, fl, idx, c, k, nullptr, &dL);
      Qn[k] = rr[(long long)k * g.N + idx] + (dt * dt / 3.0) * dL;
    }
    if (!BULK && g.fx != 0.0) {
      const double mx_old = qn[g.N + idx];
      Qn[1] = Qn[1] + 0.5 * dt * (Qn[0] + qn[idx]) * g.fx;
      Qn[4] = Qn[4] + 0.5 * dt * (Qn[1] + mx_old) * g.fx;
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) qout[(long long)k * g.N + idx] = Qn[k];
    if constexpr (BULK) {
      const double V = cell_volume(g, c[1]);
      sm = Qn[1] * V;
      ss = (qn[idx] + Qn[0]) * V;
      sv = V;
    } else {
      bool ok;
      speed = cell_speed(g, Qn, c[1], ok);
      if (!ok) {
        ctrl->fail_step = step;
        ctrl->flag = 1;
      }
    }
  }
  if constexpr (BULK) block_sums3(sm, ss, sv, mpart + 3 * (long long)blockIdx.x);
  else block_max_speed(speed, part);
}

// The step's force for constant bulk momentum (Sec. 3.3) from the stage-2 block
// sums, combined in a fixed order: f_x = (m_b vol - M~) / (dt/2 S), with M~ the
// box integral of the unforced (rho U)~, S that of rho^n + rho~ and vol the box
// volume.  One block.
__global__ void __launch_bounds__(256) bulk_force_kernel(const double* __restrict__ mpart, int nblocks, Ctrl* ctrl,
                                                         double m_b, double* __restrict__ fx_out) {
  __shared__ double tot[3];
  __shared__ int stop;
  if (threadIdx.x == 0) stop = ctrl->flag;
  __syncthreads();
  if (stop) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += 256) {
    a += mpart[3 * (long long)i];
    b += mpart[3 * (long long)i + 1];
    c += mpart[3 * (long long)i + 2];
  }
  block_sums3(a, b, c, tot);
  __syncthreads();
  if (threadIdx.x == 0) *fx_out = (m_b * tot[2] - tot[0]) / (0.5 * ctrl->dt * tot[1]);
}

// Applies the force by the trapezoidal rule of stage2_kernel to the unforced
// state in qout; physicality and the next step's CFL block maxima as there.
__global__ void __launch_bounds__(256) bulk_force_apply_kernel(Geo g, const double* __restrict__ qn,
                                                               double* __restrict__ qout, Ctrl* ctrl,
                                                               const double* __restrict__ fxp,
                                                               double* __restrict__ part, int step) {
  __shared__ int stop;
  if (threadIdx.x == 0) stop = ctrl->flag;
  __syncthreads();
  if (stop) return;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double speed = 0.0;
  if (idx < g.N) {
    const double dt = ctrl->dt, fx = *fxp;
    double Q[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) Q[k] = qout[(long long)k * g.N + idx];
    const double mx_old = qn[g.N + idx];
    Q[1] = Q[1] + 0.5 * dt * (Q[0] + qn[idx]) * fx;
    Q[4] = Q[4] + 0.5 * dt * (Q[1] + mx_old) * fx;
    qout[g.N + idx] = Q[1];
    qout[4 * g.N + idx] = Q[4];
    int c[3];
    cell_coords<0>(g, idx, c);
    bool ok;
    speed = cell_speed(g, Q, c[1], ok);
    if (!ok) {
      ctrl->fail_step = step;
      ctrl->flag = 1;
    }
  }
  block_max_speed(speed, part);
}

// CFL speed and physicality of the state at the start of a call.
__global__ void __launch_bounds__(256) check_state_kernel(Geo g, const double* __restrict__ q, Ctrl* ctrl,
                                                          double* __restrict__ part, int step) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double speed = 0.0;
  if (idx < g.N) {
    double Q[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) Q[k] = q[(long long)k * g.N + idx];
    int c[3];
    cell_coords<0>(g, idx, c);
    bool ok;
    speed = cell_speed(g, Q, c[1], ok);
    if (!ok) {
      ctrl->fail_step = step;
      ctrl->flag = 1;
    }
  }
  block_max_speed(speed, part);
}

__global__ void reset_ctrl_kernel(Ctrl* ctrl) {
  ctrl->dt = 0.0;
  ctrl->maxspeed = 0.0;
  ctrl->flag = 0;
  ctrl->fail_step = -1;
  ctrl->zero = 0;
}

// L and dL of Eq. (finite) from the face fluxes (parity entry point).
template <typename TF>
__global__ void __launch_bounds__(256) operator_kernel(Geo g, const TF* __restrict__ fl, double* __restrict__ L,
                                                       double* __restrict__ dL) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.N) return;
  int c[3];
  cell_coords<0>(g, idx, c);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double l, dl;
    divergence(g, fl, idx, c, k, &l, &dl);
    L[(long long)k * g.N + idx] = l;
    dL[(long long)k * g.N + idx] = dl;
  }
}

// Face fluxes of one direction as FP64 face averages with the constant reference
// pressure restored in the normal-momentum component (parity entry point).  On a
// stretched y the Gauss points of x- and z-faces carry their shares of the row
// height, so the constant comes back with the same weights.
template <typename TF>
__global__ void __launch_bounds__(256) export_flux_kernel(Geo g, int dir, const TF* __restrict__ fl,
                                                          double* __restrict__ F, double* __restrict__ dF) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.N) return;
  double pref = g.p_ref;
  if (g.stretch_y && dir != 1) {
    int c[3];
    cell_coords<0>(g, idx, c);
    pref = g.p_ref * (0.5 * (ym_gp_w(g, c[1], 0) + ym_gp_w(g, c[1], 1)));
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    F[(long long)k * g.N + idx] = double(fl[(long long)k * g.N + idx]) + (k == 1 + dir ? pref : 0.0);
    dF[(long long)k * g.N + idx] = double(fl[(long long)(5 + k) * g.N + idx]);
  }
}

// Face fluxes of the two wall faces of every (x, z) column of the channel: F and
// dF [2][5][nz][nx], entry 0 the bottom wall face (row -1/2, kept in its own
// array), entry 1 the top wall face (row ny-1/2, stored at the top row's cells);
// face averages in the global frame, the reference pressure restored in the
// normal (y) momentum.
template <typename TF>
__global__ void __launch_bounds__(256) export_wall_flux_kernel(Geo g, const TF* __restrict__ fl,
                                                               double* __restrict__ F, double* __restrict__ dF) {
  const long long m = (long long)g.n[0] * g.n[2];
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m) return;
  const int i = int(idx % g.n[0]), k = int(idx / g.n[0]);
  const TF* bot = static_cast<const TF*>(g.fwall);
  const long long top = (long long)i + (long long)(g.n[1] - 1) * g.stride[1] + (long long)k * g.stride[2];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double pref = c == 2 ? g.p_ref : 0.0;
    F[(long long)c * m + idx] = double(bot[(long long)c * m + idx]) + pref;
    dF[(long long)c * m + idx] = double(bot[(long long)(5 + c) * m + idx]);
    F[(long long)(5 + c) * m + idx] = double(fl[(long long)c * g.N + top]) + pref;
    dF[(long long)(5 + c) * m + idx] = double(fl[(long long)(5 + c) * g.N + top]);
  }
}

__global__ void __launch_bounds__(256) copy_kernel(const double* __restrict__ src, double* __restrict__ dst, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long n) { return unsigned((n + 255) / 256); }

void launch_dt(const Geo& g, const double* part, Ctrl* ctrl, double dt_fixed, int hist, hipStream_t st) {
  dt_kernel<<<1, 1024, 0, st>>>(g, part, int(blocks_for(g.N)), ctrl, dt_fixed, hist);
}

template <typename TF>
void launch_stage1(const Geo& g, const double* qn, const TF* fl, double* qs, double* rr, Ctrl* ctrl, int step,
                   hipStream_t st) {
  stage1_kernel<TF><<<blocks_for(g.N), 256, 0, st>>>(g, qn, fl, qs, rr, ctrl, step);
}
template void launch_stage1<double>(const Geo&, const double*, const double*, double*, double*, Ctrl*, int, hipStream_t);
template void launch_stage1<float>(const Geo&, const double*, const float*, double*, double*, Ctrl*, int, hipStream_t);

template <typename TF>
void launch_stage2(const Geo& g, const double* rr, const TF* fl, const double* qn, double* qout, Ctrl* ctrl,
                   double* part, double* mpart, int step, hipStream_t st) {
  if (mpart)
    stage2_kernel<TF, true><<<blocks_for(g.N), 256, 0, st>>>(g, rr, fl, qn, qout, ctrl, part, mpart, step);
  else
    stage2_kernel<TF, false><<<blocks_for(g.N), 256, 0, st>>>(g, rr, fl, qn, qout, ctrl, part, nullptr, step);
}
template void launch_stage2<double>(const Geo&, const double*, const double*, const double*, double*, Ctrl*, double*,
                                    double*, int, hipStream_t);
template void launch_stage2<float>(const Geo&, const double*, const float*, const double*, double*, Ctrl*, double*,
                                   double*, int, hipStream_t);

// mflux holds 3 * blocks_for(N) block sums, then the force
void launch_bulk_force(const Geo& g, const double* qn, double* qout, Ctrl* ctrl, double* mflux, double m_b,
                       double* part, int step, hipStream_t st) {
  const unsigned nb = blocks_for(g.N);
  double* fx = mflux + 3 * size_t(nb);
  bulk_force_kernel<<<1, 256, 0, st>>>(mflux, int(nb), ctrl, m_b, fx);
  bulk_force_apply_kernel<<<nb, 256, 0, st>>>(g, qn, qout, ctrl, fx, part, step);
}

void launch_check_state(const Geo& g, const double* q, Ctrl* ctrl, double* part, int step, hipStream_t st) {
  check_state_kernel<<<blocks_for(g.N), 256, 0, st>>>(g, q, ctrl, part, step);
}

size_t speed_partials(const Geo& g) { return size_t(blocks_for(g.N)); }

void launch_reset_ctrl(Ctrl* ctrl, hipStream_t st) { reset_ctrl_kernel<<<1, 1, 0, st>>>(ctrl); }

template <typename TF>
void launch_operator(const Geo& g, const TF* fl, double* L, double* dL, hipStream_t st) {
  operator_kernel<TF><<<blocks_for(g.N), 256, 0, st>>>(g, fl, L, dL);
}
template void launch_operator<double>(const Geo&, const double*, double*, double*, hipStream_t);
template void launch_operator<float>(const Geo&, const float*, double*, double*, hipStream_t);

template <typename TF>
void launch_export_flux(const Geo& g, int dir, const TF* fl, double* F, double* dF, hipStream_t st) {
  export_flux_kernel<TF><<<blocks_for(g.N), 256, 0, st>>>(g, dir, fl, F, dF);
}
template void launch_export_flux<double>(const Geo&, int, const double*, double*, double*, hipStream_t);
template void launch_export_flux<float>(const Geo&, int, const float*, double*, double*, hipStream_t);

template <typename TF>
void launch_export_wall_flux(const Geo& g, const TF* fl, double* F, double* dF, hipStream_t st) {
  export_wall_flux_kernel<TF><<<blocks_for((long long)g.n[0] * g.n[2]), 256, 0, st>>>(g, fl, F, dF);
}
template void launch_export_wall_flux<double>(const Geo&, const double*, double*, double*, hipStream_t);
template void launch_export_wall_flux<float>(const Geo&, const float*, double*, double*, hipStream_t);

void launch_copy(const double* src, double* dst, long long n, hipStream_t st) {
  long long b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  copy_kernel<<<unsigned(b), 256, 0, st>>>(src, dst, n);
}

}  // namespace hgks
