// Global diagnostics of Sec. 3.1 and Sec. 3.4 in FP64 with a fixed reduction
// order (each block owns a fixed set of cells; blocks are combined serially),
// so repeated calls are bitwise identical.
#include "internal.hpp"

namespace hgks {

constexpr int kDiagBlocks = 512;
constexpr int kDiagThreads = 256;
constexpr int kNDiag = 34;

// accumulator slots (those with derived outputs are filled by the final kernel)
enum {
  A_TOT = 0, A_KE = 5, A_ENS = 6, A_EPS1 = 7, A_EPS2 = 8, A_EPS3 = 9, A_VAR = 10, A_U2 = 11,
  A_MINR = 13, A_MINP = 14, A_EPSS = 16, A_EPSD = 17, A_PTH = 18, A_RHO = 19, A_G2 = 20, A_G3 = 23,
  A_G4 = 26, A_C = 31, A_VOL = 32, A_MAXS = 33
};

__device__ __forceinline__ bool is_min_slot(int s) { return s == A_MINR || s == A_MINP; }
__device__ __forceinline__ bool is_max_slot(int s) { return s == A_MAXS; }

__device__ __forceinline__ double vel(const Geo& g, const double* q, long long i, int comp) {
  return q[(long long)(1 + comp) * g.N + i] / q[i];
}

// pass 0: all sums; pass 1: sum (rho - mean)^2 V with the mean from pass 0
__global__ void __launch_bounds__(kDiagThreads) diag_partial_kernel(Geo g, const double* __restrict__ q,
                                                                    double* __restrict__ part, int pass,
                                                                    const double* __restrict__ out) {
  __shared__ double red[kDiagThreads];
  double acc[kNDiag];
#pragma unroll
  for (int s = 0; s < kNDiag; ++s) acc[s] = is_min_slot(s) ? 1e300 : 0.0;
  const double Vu = g.h[0] * g.h[1] * g.h[2];
  const double mean_rho = pass == 1 ? out[19] : 0.0;
  const double c6[3] = {45.0 / 60.0, -9.0 / 60.0, 1.0 / 60.0};  // antisymmetric weights at offsets 1, 2, 3
  for (long long idx = (long long)blockIdx.x * kDiagThreads + threadIdx.x; idx < g.N;
       idx += (long long)kDiagBlocks * kDiagThreads) {
    double Q[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) Q[k] = q[(long long)k * g.N + idx];
    int c[3];
    c[0] = int(idx % g.n[0]);
    long long r = idx / g.n[0];
    c[1] = int(r % g.n[1]);
    c[2] = int(r / g.n[1]);
    // cell volume (row height on a stretched mesh)
    const double V = g.stretch_y ? g.h[0] * g.h[2] * ym_dy(g, c[1]) : Vu;
    if (pass == 1) {
      double dr = Q[0] - mean_rho;
      acc[A_VAR] += dr * dr * V;
      continue;
    }
    double ir = 1.0 / Q[0];
    double U[3] = {Q[1] * ir, Q[2] * ir, Q[3] * ir};
    double u2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    double p = g.gm1 * (Q[4] - 0.5 * Q[0] * u2);
    double T = p * ir;
    double mu = g.mu_ref;
    if (g.mu_exp != 0.0) mu *= pow(T / g.T_ref, g.mu_exp);
    double cs = sqrt(g.gamma * p * ir);
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[A_TOT + k] += Q[k] * V;
    acc[A_KE] += 0.5 * Q[0] * u2 * V;
    acc[A_RHO] += Q[0] * V;
    acc[A_U2] += u2 / 3.0 * V;
    acc[A_C] += cs * V;
    acc[A_VOL] += V;
    acc[A_MINR] = fmin(acc[A_MINR], Q[0]);
    acc[A_MINP] = fmin(acc[A_MINP], p);
    double sp = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      sp = fmax(sp, (fabs(U[a]) + cs) * (a == 1 && g.stretch_y ? ym_inv_dy(g, c[1]) : g.inv_h[a]));
    acc[A_MAXS] = fmax(acc[A_MAXS], sp);
    // the derivative diagnostics need a uniform mesh
    if (g.stretch_y) continue;
    // velocity gradient gr[a][k] = dU_k/dx_a by the sixth-order central difference
    double gr[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const long long base = idx - (long long)c[a] * g.stride[a];
      double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int o = 1; o <= 3; ++o) {
        if (a == 1 && g.wall_y && (c[1] - o < 0 || c[1] + o >= g.n[1])) {
          // a wall within reach: neighbours beyond it are wall ghosts
          double Qp[5], Qm[5];
          load_cell_wall(g, q, c[0], c[1] + o, c[2], Qp);
          load_cell_wall(g, q, c[0], c[1] - o, c[2], Qm);
#pragma unroll
          for (int k = 0; k < 3; ++k) s[k] += c6[o - 1] * (Qp[1 + k] / Qp[0] - Qm[1 + k] / Qm[0]);
          continue;
        }
        long long ip = base + (long long)wrapi(c[a] + o, g.n[a]) * g.stride[a];
        long long im = base + (long long)wrapi(c[a] - o, g.n[a]) * g.stride[a];
        double irp = 1.0 / q[ip], irm = 1.0 / q[im];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          s[k] += c6[o - 1] * (q[(long long)(1 + k) * g.N + ip] * irp - q[(long long)(1 + k) * g.N + im] * irm);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) gr[a][k] = s[k] * g.inv_h[a];
    }
    double wx = gr[1][2] - gr[2][1], wy = gr[2][0] - gr[0][2], wz = gr[0][1] - gr[1][0];
    double w2 = wx * wx + wy * wy + wz * wz;
    double th = gr[0][0] + gr[1][1] + gr[2][2];
    double SS = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double S = 0.5 * (gr[a][k] + gr[k][a]) - (a == k ? th / 3.0 : 0.0);
        SS += S * S;
      }
    double mub = (g.mub_m23 + 2.0 / 3.0) * mu;
    acc[A_ENS] += 0.5 * Q[0] * w2 * V;
    acc[A_EPS1] += 2.0 * mu * SS * V;
    acc[A_EPS2] += mub * th * th * V;
    acc[A_EPS3] += -p * th * V;
    acc[A_EPSS] += mu * w2 * V;
    acc[A_EPSD] += 4.0 / 3.0 * mu * th * th * V;
    acc[A_PTH] += p * th * V;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double x = gr[a][a];
      acc[A_G2 + a] += x * x * V;
      acc[A_G3 + a] += x * x * x * V;
      acc[A_G4 + a] += x * x * x * x * V;
    }
  }
  // fixed-order tree reduction of each slot over the block
  for (int s = 0; s < kNDiag; ++s) {
    if (pass == 1 && s != A_VAR) continue;
    red[threadIdx.x] = acc[s];
    __syncthreads();
    for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        double a = red[threadIdx.x], b = red[threadIdx.x + w];
        red[threadIdx.x] = is_min_slot(s) ? fmin(a, b) : (is_max_slot(s) ? fmax(a, b) : a + b);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)blockIdx.x * kNDiag + s] = red[0];
    __syncthreads();
  }
}

// serial combination of the block partials and the derived quantities
__global__ void diag_final_kernel(const double* __restrict__ part, double* __restrict__ out, int pass, double rho0) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc[kNDiag];
  for (int s = 0; s < kNDiag; ++s) {
    double v = is_min_slot(s) ? 1e300 : 0.0;
    if (pass == 1 && s != A_VAR) continue;
    for (int b = 0; b < kDiagBlocks; ++b) {
      double x = part[(long long)b * kNDiag + s];
      v = is_min_slot(s) ? fmin(v, x) : (is_max_slot(s) ? fmax(v, x) : v + x);
    }
    acc[s] = v;
  }
  if (pass == 1) {
    out[10] = sqrt(acc[A_VAR] / out[32]);
    return;
  }
  const double vol = acc[A_VOL];
  for (int k = 0; k < 5; ++k) out[k] = acc[A_TOT + k];
  out[5] = acc[A_KE] / (rho0 * vol);
  out[6] = acc[A_ENS] / (rho0 * vol);
  out[7] = acc[A_EPS1] / (rho0 * vol);
  out[8] = acc[A_EPS2] / (rho0 * vol);
  out[9] = acc[A_EPS3] / (rho0 * vol);
  out[10] = 0.0;
  out[11] = sqrt(acc[A_U2] / vol);
  out[31] = acc[A_C] / vol;
  out[12] = sqrt(3.0) * out[11] / out[31];
  out[13] = acc[A_MINR];
  out[14] = acc[A_MINP];
  out[15] = acc[A_KE] / vol;
  out[16] = acc[A_EPSS] / vol;
  out[17] = acc[A_EPSD] / vol;
  out[18] = acc[A_PTH] / vol;
  out[19] = acc[A_RHO] / vol;
  double Su = 0.0, Fu = 0.0;
  for (int a = 0; a < 3; ++a) {
    double m2 = acc[A_G2 + a] / vol, m3 = acc[A_G3 + a] / vol, m4 = acc[A_G4 + a] / vol;
    out[20 + a] = m2;
    out[23 + a] = m3;
    out[26 + a] = m4;
    if (m2 > 0.0) {
      Su += m3 / pow(m2, 1.5);
      Fu += m4 / (m2 * m2);
    }
  }
  out[29] = Su;
  out[30] = Fu;
  out[32] = vol;
  out[33] = acc[A_MAXS];
}

size_t diag_partial_doubles() { return size_t(kDiagBlocks) * kNDiag; }

// ---- normalized dilatation theta / theta_rms (Sec. 3.4, the dilation contours
// of the isotropic cases: shocklets where it is at most -3, strong expansion where
// it is at least 2).  theta = div U by the same sixth-order central difference as
// the diagnostics, recomputed in both passes rather than stored.  The partial
// buffer holds the block sums of theta^2 in its first kDiagBlocks entries,
// theta_rms at kDiagBlocks, then the nbins + 2 counts as 64-bit integers.
static_assert(size_t(kDiagBlocks) + 1 + kPdfMaxBins + 2 <= size_t(kDiagBlocks) * kNDiag,
              "the counts fit in the partial buffer");
// 1024 threads per block (four waves per SIMD at 98 VGPRs, against two with 256
// threads): 17% faster at 256^3; the z-neighbour planes' re-reads remain
constexpr int kDilThreads = 1024;

__device__ __forceinline__ double dilatation_at(const Geo& g, const double* __restrict__ q, long long idx,
                                                const int* c) {
  const double c6[3] = {45.0 / 60.0, -9.0 / 60.0, 1.0 / 60.0};
  double th = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const long long base = idx - (long long)c[a] * g.stride[a];
    double s = 0.0;
#pragma unroll
    for (int o = 1; o <= 3; ++o) {
      if (a == 1 && g.wall_y && (c[1] - o < 0 || c[1] + o >= g.n[1])) {
        double Qp[5], Qm[5];
        load_cell_wall(g, q, c[0], c[1] + o, c[2], Qp);
        load_cell_wall(g, q, c[0], c[1] - o, c[2], Qm);
        s += c6[o - 1] * (Qp[1 + a] / Qp[0] - Qm[1 + a] / Qm[0]);
        continue;
      }
      const long long ip = base + (long long)wrapi(c[a] + o, g.n[a]) * g.stride[a];
      const long long im = base + (long long)wrapi(c[a] - o, g.n[a]) * g.stride[a];
      s += c6[o - 1] * (q[(long long)(1 + a) * g.N + ip] / q[ip] - q[(long long)(1 + a) * g.N + im] / q[im]);
    }
    th += s * g.inv_h[a];
  }
  return th;
}

__device__ __forceinline__ void cell_coords(const Geo& g, long long idx, int* c) {
  c[0] = int(idx % g.n[0]);
  const long long r = idx / g.n[0];
  c[1] = int(r % g.n[1]);
  c[2] = int(r / g.n[1]);
}

// block sums of theta^2 in a fixed order
__global__ void __launch_bounds__(kDilThreads) dil_sum_kernel(Geo g, const double* __restrict__ q,
                                                               double* __restrict__ part) {
  __shared__ double red[kDilThreads];
  double acc = 0.0;
  for (long long idx = (long long)blockIdx.x * kDilThreads + threadIdx.x; idx < g.N;
       idx += (long long)kDiagBlocks * kDilThreads) {
    int c[3];
    cell_coords(g, idx, c);
    const double th = dilatation_at(g, q, idx, c);
    acc += th * th;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kDilThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// theta_rms from the block sums (serial), and the global counts cleared
__global__ void dil_rms_kernel(Geo g, double* __restrict__ part, int nslots) {
  unsigned long long* counts = reinterpret_cast<unsigned long long*>(part + kDiagBlocks + 1);
  for (int i = threadIdx.x; i < nslots; i += blockDim.x) counts[i] = 0ull;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < kDiagBlocks; ++b) s += part[b];
    part[kDiagBlocks] = sqrt(s / double(g.N));
  }
}

// histogram of r = theta / theta_rms (r = 0 where theta_rms = 0, i.e. every theta
// is zero): slot 0 for r < lo, 1 + floor((r - lo) * scale) for lo <= r < hi (the
// last bin also takes the rounding of values just below hi), nbins + 1 for r >= hi
// and for non-finite r.  Counts are integers, so their order of addition is
// immaterial.
__global__ void __launch_bounds__(kDilThreads) dil_hist_kernel(Geo g, const double* __restrict__ q,
                                                                double* __restrict__ part, int nbins, double lo,
                                                                double hi, double scale) {
  __shared__ unsigned int hist[kPdfMaxBins + 2];
  const int nslots = nbins + 2;
  for (int i = threadIdx.x; i < nslots; i += kDilThreads) hist[i] = 0u;
  __syncthreads();
  const double rms = part[kDiagBlocks];
  for (long long idx = (long long)blockIdx.x * kDilThreads + threadIdx.x; idx < g.N;
       idx += (long long)kDiagBlocks * kDilThreads) {
    int c[3];
    cell_coords(g, idx, c);
    const double th = dilatation_at(g, q, idx, c);
    const double r = rms > 0.0 ? th / rms : 0.0;
    int slot;
    if (r < lo) {
      slot = 0;
    } else if (r >= hi || !(r == r)) {
      slot = nbins + 1;
    } else {
      const int b = int(floor((r - lo) * scale));
      slot = 1 + (b < nbins - 1 ? b : nbins - 1);
    }
    atomicAdd(&hist[slot], 1u);
  }
  __syncthreads();
  unsigned long long* counts = reinterpret_cast<unsigned long long*>(part + kDiagBlocks + 1);
  for (int i = threadIdx.x; i < nslots; i += kDilThreads)
    if (hist[i]) atomicAdd(&counts[i], (unsigned long long)hist[i]);
}

void launch_dilatation_pdf(const Geo& g, const double* q, double* part, int nbins, double lo, double hi,
                           hipStream_t st) {
  dil_sum_kernel<<<kDiagBlocks, kDilThreads, 0, st>>>(g, q, part);
  dil_rms_kernel<<<1, 256, 0, st>>>(g, part, nbins + 2);
  dil_hist_kernel<<<kDiagBlocks, kDilThreads, 0, st>>>(g, q, part, nbins, lo, hi, double(nbins) / (hi - lo));
}

// theta / theta_rms on the plane `index` of `axis` (the slices whose contours
// Sec. 3.4 shows), rms from the partial buffer; out holds the plane's cells with
// the two remaining axes in state order (slower first, faster fastest)
__global__ void __launch_bounds__(256) dil_slice_kernel(Geo g, const double* __restrict__ q,
                                                        const double* __restrict__ part, int axis, int index,
                                                        double* __restrict__ out) {
  const int fa = axis == 0 ? 1 : 0;  // faster remaining axis
  const int sa = axis == 2 ? 1 : 2;  // slower remaining axis
  const long long m = (long long)blockIdx.x * 256 + threadIdx.x;
  if (m >= (long long)g.n[fa] * g.n[sa]) return;
  int c[3];
  c[axis] = index;
  c[fa] = int(m % g.n[fa]);
  c[sa] = int(m / g.n[fa]);
  const long long idx = (long long)c[0] + (long long)c[1] * g.stride[1] + (long long)c[2] * g.stride[2];
  const double rms = part[kDiagBlocks];
  const double th = dilatation_at(g, q, idx, c);
  out[m] = rms > 0.0 ? th / rms : 0.0;
}

void launch_dilatation_slice(const Geo& g, const double* q, double* part, int axis, int index, double* out,
                             hipStream_t st) {
  dil_sum_kernel<<<kDiagBlocks, kDilThreads, 0, st>>>(g, q, part);
  dil_rms_kernel<<<1, 256, 0, st>>>(g, part, 0);
  const int fa = axis == 0 ? 1 : 0, sa = axis == 2 ? 1 : 2;
  const long long cells = (long long)g.n[fa] * g.n[sa];
  dil_slice_kernel<<<unsigned((cells + 255) / 256), 256, 0, st>>>(g, q, part, axis, index, out);
}

// ---- plane-averaged profiles per y row (Sec. 3.3: mean velocity, velocity
// fluctuations and Reynolds stress of the channel).  One block per row; Reynolds
// averages over the row's nx * nz cells, the second moments about the row means
// in a second pass over the row.  Fixed reduction order.
constexpr int kProfThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kProfThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

__device__ __forceinline__ void row_cell(const Geo& g, const double* __restrict__ q, int j, long long m, double& rho,
                                         double* U, double& p) {
  const int x = int(m % g.n[0]);
  const long long z = m / g.n[0];
  const long long idx = (long long)x + (long long)j * g.stride[1] + z * g.stride[2];
  rho = q[idx];
  const double ir = 1.0 / rho;
#pragma unroll
  for (int k = 0; k < 3; ++k) U[k] = q[(long long)(1 + k) * g.N + idx] * ir;
  const double u2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
  p = g.gm1 * (q[4 * g.N + idx] - 0.5 * rho * u2);
}

__global__ void __launch_bounds__(kProfThreads) profile_kernel(Geo g, const double* __restrict__ q,
                                                               double* __restrict__ out) {
  __shared__ double red[kProfThreads];
  const int j = blockIdx.x;
  const long long nxz = (long long)g.n[0] * g.n[2];
  double s[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // rho, U, V, W, p, T, rho U
  for (long long m = threadIdx.x; m < nxz; m += kProfThreads) {
    double rho, U[3], p;
    row_cell(g, q, j, m, rho, U, p);
    s[0] += rho;
    s[1] += U[0];
    s[2] += U[1];
    s[3] += U[2];
    s[4] += p;
    s[5] += p / rho;
    s[6] += rho * U[0];
  }
  double mean[7];
#pragma unroll 1
  for (int k = 0; k < 7; ++k) mean[k] = block_sum(s[k], red) / double(nxz);
  double c[4] = {0.0, 0.0, 0.0, 0.0};  // u'u', v'v', w'w', u'v'
  for (long long m = threadIdx.x; m < nxz; m += kProfThreads) {
    double rho, U[3], p;
    row_cell(g, q, j, m, rho, U, p);
    const double du = U[0] - mean[1], dv = U[1] - mean[2], dw = U[2] - mean[3];
    c[0] += du * du;
    c[1] += dv * dv;
    c[2] += dw * dw;
    c[3] += du * dv;
  }
  double cov[4];
#pragma unroll 1
  for (int k = 0; k < 4; ++k) cov[k] = block_sum(c[k], red) / double(nxz);
  if (threadIdx.x == 0) {
    double* o = out + (long long)j * kNProfile;
    for (int k = 0; k < 6; ++k) o[k] = mean[k];
    for (int k = 0; k < 4; ++k) o[6 + k] = cov[k];
    o[10] = mean[6];
  }
}

void launch_plane_profiles(const Geo& g, const double* q, double* out, hipStream_t st) {
  profile_kernel<<<g.n[1], kProfThreads, 0, st>>>(g, q, out);
}

size_t dilatation_pdf_rms_offset() { return kDiagBlocks; }
size_t dilatation_pdf_counts_offset() { return kDiagBlocks + 1; }

void launch_diagnostics(const Geo& g, const double* q, double* part, double* out, hipStream_t st) {
  diag_partial_kernel<<<kDiagBlocks, kDiagThreads, 0, st>>>(g, q, part, 0, out);
  diag_final_kernel<<<1, 64, 0, st>>>(part, out, 0, 1.0);
  diag_partial_kernel<<<kDiagBlocks, kDiagThreads, 0, st>>>(g, q, part, 1, out);
  diag_final_kernel<<<1, 64, 0, st>>>(part, out, 1, 1.0);
}

}  // namespace hgks
