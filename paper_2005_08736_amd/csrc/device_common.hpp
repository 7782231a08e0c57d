// Device-side building blocks of the HGKS stage update for gfx950 (CDNA4).
//
// Scheme: Cao, Pan & Xu, arXiv:2005.08736, Sec. 2.1.  The state is FP64
// structure-of-arrays q[5][nz][ny][nx]; every kernel maps one thread to one
// face or cell with x fastest, so each wavefront's loads and stores of a field
// are 64 consecutive doubles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace hgks {

// Grid and gas constants, passed to every kernel by value.
struct Geo {
  int n[3];              // cells along x, y, z
  long long N;           // total cells
  long long stride[3];   // 1, nx, nx*ny
  double h[3];           // cell widths
  double inv_h[3];
  double gamma, gm1, inv_gm1;
  double cp;             // gamma / (gamma - 1) with R = 1
  double inv_pr;         // 1 / Pr
  double pr_fix;         // 1 / Pr - 1 (heat-flux correction of the BGK model)
  double mub_m23;        // mu_b/mu - 2/3 with mu_b/mu = 2K/(3(K+3))
  double K;              // internal degrees of freedom
  double mu_ref, T_ref, mu_exp;
  double cfl;
  // constant reference state (rho_ref, U = 0, p_ref): the flux arithmetic works on
  // deviations from it, and the constant p_ref is left out of the normal-momentum
  // face flux (a constant flux has no divergence)
  double rho_ref, p_ref, E_ref, H_ref;  // E_ref = p_ref/(gamma-1), H_ref = gamma p_ref/(gamma-1)
  // WENO-Z / full-flux mode: Z-weight epsilon and exponent, artificial collision-time coefficient
  double weno_eps, c_art;
  int weno_p;
  // channel (Sec. 3.3): isothermal no-slip walls at both ends of y, the tanh
  // mesh in y (metric tables in device memory, see ym_* below), and the
  // constant streamwise body force
  int wall_y, stretch_y;
  double T_wall, fx;
  const double* ym;        // metric tables (stretched y only)
  const void* fwall;       // face fluxes of the bottom wall faces (walls only), [10][nz][nx]
};

// ---------------------------------------------------------------------------
// Stretched wall-normal mesh y(eta), eta uniform with spacing h[1] (Sec. 3.3).
// Tables of 7 ny + 1 doubles, computed on the host at init:
//   [0, ny)          1 / dy_j            (dy_j: height of row j)
//   [ny, 2ny)        dy_j
//   [2ny, 3ny+1)     1 / (y'(eta_f) h)   at the faces eta_f = f h, f = 0..ny
//   [3ny+1, 5ny+1)   1 / (y'(eta) h)     at the two Gauss points of row j (2j + m)
//   [5ny+1, 7ny+1)   y'(eta) h / dy_j    the Gauss points' share of the row height
// A derivative per unit eta-width times 1/(y' h) is the physical derivative; the
// face average of a face with y as a tangential axis weights its Gauss points
// by their share of the row height (the two shares sum to 2 up to the
// quadrature error of the two-point rule).
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ double ym_inv_dy(const Geo& g, int j) { return g.ym[j]; }
__host__ __device__ __forceinline__ double ym_dy(const Geo& g, int j) { return g.ym[g.n[1] + j]; }
__host__ __device__ __forceinline__ double ym_face_inv(const Geo& g, int f) { return g.ym[2 * g.n[1] + f]; }
__host__ __device__ __forceinline__ double ym_gp_inv(const Geo& g, int j, int m) { return g.ym[3 * g.n[1] + 1 + 2 * j + m]; }
__host__ __device__ __forceinline__ double ym_gp_w(const Geo& g, int j, int m) { return g.ym[5 * g.n[1] + 1 + 2 * j + m]; }
constexpr int kYmTableDoubles = 7;  // per row, plus one

// Ghost state behind an isothermal no-slip wall from its mirror cell Q (global
// frame, full conservative variables): velocity reversed, equal pressure,
// temperature reflected about the wall temperature, T_g = 2 T_w - T, held at
// T_w / 2 or above.
__host__ __device__ __forceinline__ void wall_ghost(const Geo& g, double* Q) {
  const double rho = Q[0];
  const double U = Q[1] / rho, V = Q[2] / rho, W = Q[3] / rho;
  const double p = g.gm1 * (Q[4] - 0.5 * (Q[1] * Q[1] + Q[2] * Q[2] + Q[3] * Q[3]) / rho);
  double Tg = 2.0 * g.T_wall - p / rho;
  if (Tg < 0.5 * g.T_wall) Tg = 0.5 * g.T_wall;
  const double rg = p / Tg;
  Q[0] = rg;
  Q[1] = rg * -U;
  Q[2] = rg * -V;
  Q[3] = rg * -W;
  Q[4] = p / g.gm1 + 0.5 * rg * (U * U + V * V + W * W);
}

// Row of the cell that supplies row y when walls bound y: rows outside [0, ny)
// are ghosts of their mirror rows (-1 - y below, 2 ny - 1 - y above).  Rows more
// than three beyond a wall only feed faces outside the grid, whose results are
// discarded; they are clamped into the grid so that every read stays in bounds.
__host__ __device__ __forceinline__ int wall_row(const Geo& g, int y, bool& ghost) {
  ghost = y < 0 || y >= g.n[1];
  int ym = y < 0 ? -1 - y : (y >= g.n[1] ? 2 * g.n[1] - 1 - y : y);
  ym = ym < 0 ? 0 : (ym >= g.n[1] ? g.n[1] - 1 : ym);
  return ym;
}

// The conservative variables of cell (x, y, z), global frame, with walls in y
// (see wall_row); x and z are in range.
__host__ __device__ __forceinline__ void load_cell_wall(const Geo& g, const double* q, int x, int y, int z,
                                                        double* Q) {
  bool ghost;
  const int ym = wall_row(g, y, ghost);
  const long long idx = (long long)x + (long long)ym * g.stride[1] + (long long)z * g.stride[2];
#pragma unroll
  for (int k = 0; k < 5; ++k) Q[k] = q[(long long)k * g.N + idx];
  if (ghost) wall_ghost(g, Q);
}

// Control block at the head of the workspace.
constexpr int kDtHist = 1024;
struct Ctrl {
  double dt;                       // time step of the current step
  double maxspeed;                 // max over cells and axes of (|U_d|+c)/h_d of the step's start state
  int flag;                        // set to 1 when a non-physical state appears
  int fail_step;                   // step index that produced it
  int zero;                        // always 0: "never stop" for the parity entry points
  int pad;
  double dt_hist[kDtHist];         // time step of each step of the current call
};

// Value-dependency barrier: x is treated as recomputed from `after`, so work that
// uses x cannot be scheduled before `after` is available.  Used to keep
// independent stages of a long computation from being interleaved by the
// scheduler (which would keep both stages' temporaries live at once).
template <typename T, typename U>
__host__ __device__ __forceinline__ void zdep(T& x, const U& after) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(x) : "v"(after));
#else
  (void)after;
#endif
}

// 1/a without the scaling steps of IEEE division, for a whose reciprocal is a
// normal number (densities, sound speeds, sums of positive weights).  FP64: the
// hardware estimate refined by two Newton steps r <- r + r (1 - a r), within
// about an ulp of the rounded quotient; FP32: the hardware estimate (1 ulp).
// Other arithmetic types (the forward tangents of the mode-Z adjoint) divide.
template <typename T>
__host__ __device__ __forceinline__ T recip(T a) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (std::is_same<T, double>::value) {
    double r = __builtin_amdgcn_rcp(a);
    r = fma(r, fma(-a, r, 1.0), r);
    return fma(r, fma(-a, r, 1.0), r);
  } else if constexpr (std::is_same<T, float>::value) {
    return __builtin_amdgcn_rcpf(a);
  } else {
    return T(1) / a;
  }
#else
  return T(1) / a;
#endif
}

// 1/sqrt(a) in FP64 for positive normal a whose result is normal (squared sound
// speeds): the hardware estimate refined by two Newton steps
// y <- y + y (1/2 - (a/2) y^2), within about an ulp of the rounded result.
__host__ __device__ __forceinline__ double rsqrt_refined(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double h = 0.5 * a;
  double y = __builtin_amdgcn_rsq(a);
  y = fma(y, fma(-h, y * y, 0.5), y);
  return fma(y, fma(-h, y * y, 0.5), y);
#else
  return 1.0 / sqrt(a);
#endif
}

__host__ __device__ __forceinline__ int wrapi(int i, int n) {
  i = i < 0 ? i + n : i;
  return i >= n ? i - n : i;
}

// ---------------------------------------------------------------------------
// Reconstruction coefficients.
//
// Normal direction (face between cells 0 and 1, stencils of cell averages):
//   left  value: ( 2, -13, 47, 27, -3)/60 on cells -2..2  (fifth-order upwind
//                 = WENO5 with its optimal linear weights)
//   right value: mirror image on cells -1..3
//   derivative : ( 1, -15, 15, -1)/12 on cells -1..2 (derivative at the face of
//                 the cubic through four averages; adding the face value Q0 as a
//                 fifth condition leaves it unchanged)
// Tangential direction: the quartic matching five face averages j-2..j+2,
// evaluated at the Gauss points s = +-1/(2 sqrt 3) of the middle face.  Written
// as even/odd parts about the middle so that both Gauss points come from one
// set of sums:  value(+-) = E +- O,  derivative(+-) = A +- S.
// ---------------------------------------------------------------------------
constexpr double kS3 = 1.7320508075688772935;  // sqrt(3)
// value at s = +1/(2 sqrt 3): even part (centre, +-1, +-2) and odd part (+1, +2)
constexpr double kVe0 = 719.0 / 720.0;
constexpr double kVe1 = 1.0 / 1080.0;
constexpr double kVe2 = -1.0 / 4320.0;
constexpr double kVo1 = 25.0 * kS3 / 216.0;
constexpr double kVo2 = -7.0 * kS3 / 432.0;
// derivative (per unit width) at s = +1/(2 sqrt 3): symmetric part S and antisymmetric part A
constexpr double kDs0 = -4.0 * kS3 / 9.0;
constexpr double kDs1 = 13.0 * kS3 / 54.0;
constexpr double kDs2 = -kS3 / 54.0;
constexpr double kDa1 = 2.0 / 3.0;
constexpr double kDa2 = -1.0 / 12.0;

// Tangential reconstruction of one field along a line of five face values f[0..4]
// (f[2] the middle face): values and derivatives at the -/+ Gauss points.
template <typename T>
__host__ __device__ __forceinline__ void tang_val(const T* f, T& vm, T& vp) {
  T e = T(kVe0) * f[2] + T(kVe1) * (f[1] + f[3]) + T(kVe2) * (f[0] + f[4]);
  T o = T(kVo1) * (f[3] - f[1]) + T(kVo2) * (f[4] - f[0]);
  vm = e - o;
  vp = e + o;
}
template <typename T>
__host__ __device__ __forceinline__ void tang_der(const T* f, T& dm, T& dp) {
  T s = T(kDs0) * f[2] + T(kDs1) * (f[1] + f[3]) + T(kDs2) * (f[0] + f[4]);
  T a = T(kDa1) * (f[3] - f[1]) + T(kDa2) * (f[4] - f[0]);
  dm = a - s;
  dp = a + s;
}

// ---------------------------------------------------------------------------
// Equilibrium state at the interface from the two reconstructed states: the
// compatibility condition of Sec. 2.1 integrates the left Maxwellian over u>0
// and the right one over u<0.  With lambda = rho/(2p), x = sqrt(lambda) U and
// the half-space moments of the normal velocity
//   a0 = erfc(-x)/2 = 1/2 + erf(x)/2,  a1 = U a0 + exp(-x^2)/(2 sqrt(pi lambda)),
//   a2 = U a1 + a0/(2 lambda)
// (for u<0: b0 = 1/2 - erf(x)/2, b1 = U b0 - exp(-x^2)/(2 sqrt(pi lambda))), the
// psi-moments are (a0, a1, V a0, W a0, (a2 + a0 (V^2 + W^2 + (K+2)/(2 lambda)))/2),
// whose energy moment times rho equals rho U a1/2 + rho a0 (V^2+W^2)/2 + a0 p/(gamma-1).
// Inputs and output are deviations from the reference state (rho_ref, 0, p_ref),
// arranged so that no large quantity is formed and then cancelled: this keeps the
// FP32 form accurate.  Local frame: component 1 is the face-normal momentum.
// ---------------------------------------------------------------------------
template <typename T>
struct Side {
  T rho, U, V, W, p, dp, h, th;  // h = erf(x)/2, th = exp(-x^2)/(2 sqrt(pi lambda))
};

template <typename T>
__host__ __device__ __forceinline__ Side<T> side_state(const Geo& g, const T* dQ) {
  Side<T> s;
  s.rho = T(g.rho_ref) + dQ[0];
  T ir = recip(s.rho);
  s.U = dQ[1] * ir;
  s.V = dQ[2] * ir;
  s.W = dQ[3] * ir;
  s.dp = T(g.gm1) * (dQ[4] - T(0.5) * s.rho * (s.U * s.U + s.V * s.V + s.W * s.W));
  s.p = T(g.p_ref) + s.dp;
  // c = 1/sqrt(lambda) = sqrt(2 p / rho): x = U / c, th = c exp(-x^2) / (2 sqrt(pi));
  // in FP64 one refined reciprocal square root gives both c and 1/c (1% faster
  // smooth-mode flux launches); the FP32 form keeps the square root and the
  // reciprocal estimate, which measured faster there
  const T c2 = T(2) * s.p * ir;
  T c, x;
  if constexpr (std::is_same<T, double>::value) {
    const T rc = rsqrt_refined(c2);
    c = c2 * rc;
    x = s.U * rc;
  } else {
    c = sqrt(c2);
    x = s.U * recip(c);
  }
  s.h = T(0.5) * erf(x);
  s.th = T(0.28209479177387814347) * exp(-x * x) * c;
  return s;
}

template <typename T>
__host__ __device__ __forceinline__ void compat_dev(const Geo& g, const T* dQl, const T* dQr, T* dQ0) {
  Side<T> l = side_state(g, dQl), r = side_state(g, dQr);
  T a0 = T(0.5) + l.h, b0 = T(0.5) - r.h;
  T a1 = l.U * a0 + l.th, b1 = r.U * b0 - r.th;
  dQ0[0] = T(0.5) * (dQl[0] + dQr[0]) + (l.rho * l.h - r.rho * r.h);
  dQ0[1] = l.rho * a1 + r.rho * b1;
  dQ0[2] = l.rho * l.V * a0 + r.rho * r.V * b0;
  dQ0[3] = l.rho * l.W * a0 + r.rho * r.W * b0;
  dQ0[4] = T(0.5) * (l.rho * (l.U * a1 + a0 * (l.V * l.V + l.W * l.W)) +
                     r.rho * (r.U * b1 + b0 * (r.V * r.V + r.W * r.W))) +
           (T(0.5) * (l.dp + r.dp) + (l.h * l.p - r.h * r.p)) * T(g.inv_gm1);
}

// ---------------------------------------------------------------------------
// Smooth gas-kinetic flux at one Gauss point.
//
// With a continuous equilibrium g0 on both sides, Eq. (flux) becomes
//   f = g0 [1 - tau (a_n u + a_t1 v + a_t2 w + A) + t A]
// and the psi-moments of u f are evaluated here in closed form, taking every
// moment about the interface velocity (odd central Gaussian moments vanish):
//   * <u psi> g0           -> the Euler flux of Q0;
//   * -tau <u (a.u + A) psi> g0 with the slopes a from <a psi> = dQ0/rho0 and A
//     from <a.u + A> = 0   -> the Newtonian stress with mu = tau p and bulk
//     viscosity 2K/(3(K+3)) mu, and the Fourier heat flux c_p mu dT (R = 1);
//   * <u A psi> g0         -> d/dt of the Euler flux along the Euler time
//     derivative of Q0, i.e. the flux Jacobian times dQ0/dt.
// The Prandtl-number correction adds (1/Pr - 1) times the heat flux, taken
// about the interface velocity, of each part of f: -c_p mu dT/dn for the
// tau-part and c_p p dU_n/dt for the t-part.
// Inputs (local frame, index 0 = normal): the deviation dQ of Q0 from the
// reference state and the derivatives D[a][k] = dQ0_k/dx_a along (n, t1, t2).
// F gets F^n without the constant p_ref in its normal-momentum component, dF gets
// dF^n/dt (Eq. (expansion-1)).
// VAR_MU selects mu(T) = mu_ref (T/T_ref)^mu_exp; otherwise mu = mu_ref (a
// separate instantiation keeps the power function's registers out of the
// constant-viscosity kernels).
// ---------------------------------------------------------------------------
template <bool NEED_F, bool VAR_MU, typename T>
__host__ __device__ __forceinline__ void smooth_flux(const Geo& g, const T* dQ, const T (*D)[5], T* F, T* dF) {
  const T gm1 = T(g.gm1);
  T rho = T(g.rho_ref) + dQ[0];
  T ir = recip(rho);
  T U0 = dQ[1] * ir, U1 = dQ[2] * ir, U2 = dQ[3] * ir;
  T ke = T(0.5) * (U0 * U0 + U1 * U1 + U2 * U2);
  T dp = gm1 * (dQ[4] - rho * ke);
  T p = T(g.p_ref) + dp;
  T H = T(g.H_ref) + dQ[4] + dp;  // E + p
  // velocity gradient gu[a][c] = dU_c/dx_a and pressure gradient
  T gu[3][3], gp[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gu[a][0] = (D[a][1] - U0 * D[a][0]) * ir;
    gu[a][1] = (D[a][2] - U1 * D[a][0]) * ir;
    gu[a][2] = (D[a][3] - U2 * D[a][0]) * ir;
    gp[a] = gm1 * (D[a][4] - (U0 * D[a][1] + U1 * D[a][2] + U2 * D[a][3]) + ke * D[a][0]);
  }
  T theta = gu[0][0] + gu[1][1] + gu[2][2];
  // Euler time derivatives of rho, U, p
  T rho_t = -(U0 * D[0][0] + U1 * D[1][0] + U2 * D[2][0] + rho * theta);
  T u_t[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) u_t[c] = -(U0 * gu[0][c] + U1 * gu[1][c] + U2 * gu[2][c] + gp[c] * ir);
  T p_t = -(U0 * gp[0] + U1 * gp[1] + U2 * gp[2] + T(g.gamma) * p * theta);
  T E_t = p_t * T(g.inv_gm1) + ke * rho_t + rho * (U0 * u_t[0] + U1 * u_t[1] + U2 * u_t[2]);
  T m0 = dQ[1];
  dF[0] = rho_t * U0 + rho * u_t[0];
  dF[1] = rho_t * U0 * U0 + T(2) * m0 * u_t[0] + p_t;
  dF[2] = rho_t * U0 * U1 + rho * (u_t[0] * U1 + U0 * u_t[1]);
  dF[3] = rho_t * U0 * U2 + rho * (u_t[0] * U2 + U0 * u_t[2]);
  dF[4] = u_t[0] * H + U0 * (E_t + p_t) + T(g.pr_fix * g.cp) * p * u_t[0];
  if (NEED_F) {
    T T0 = p * ir;
    T mu = T(g.mu_ref);
    if (VAR_MU) mu = mu * pow(T0 / T(g.T_ref), T(g.mu_exp));
    T s0 = mu * (T(2) * gu[0][0] + T(g.mub_m23) * theta);
    T s1 = mu * (gu[0][1] + gu[1][0]);
    T s2 = mu * (gu[0][2] + gu[2][0]);
    T dTn = (gp[0] - T0 * D[0][0]) * ir;
    F[0] = m0;
    F[1] = m0 * U0 + dp - s0;
    F[2] = m0 * U1 - s1;
    F[3] = m0 * U2 - s2;
    F[4] = U0 * H - (U0 * s0 + U1 * s1 + U2 * s2) - T(g.cp * g.inv_pr) * mu * dTn;
  }
}

}  // namespace hgks
