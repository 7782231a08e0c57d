// Reverse-mode (vector-Jacobian) counterparts of the device building blocks in
// device_common.hpp, written by hand statement by statement: each function
// recomputes the forward intermediates it needs and then accumulates the
// cotangents of its inputs in reverse order.  Used by the adjoint of the
// two-stage step (adjoint.hip).
#pragma once

#include "device_common.hpp"

namespace hgks {

// ---------------------------------------------------------------------------
// Adjoint of smooth_flux (device_common.hpp).  Given cotangents Fb (of F^n, may
// be ignored when NEED_F is false) and dFb (of dF^n/dt), accumulates the
// cotangents dQb of the deviation state and Db of its derivatives.
// ---------------------------------------------------------------------------
template <bool NEED_F, bool VAR_MU, typename T>
__host__ __device__ __forceinline__ void smooth_flux_vjp(const Geo& g, const T* dQ, const T (*D)[5], const T* Fb, const T* dFb,
                                                T* dQb, T (*Db)[5]) {
  const T gm1 = T(g.gm1);
  const T gam = T(g.gamma);
  // ---- forward
  T rho = T(g.rho_ref) + dQ[0];
  T ir = T(1) / rho;
  T U[3] = {dQ[1] * ir, dQ[2] * ir, dQ[3] * ir};
  T ke = T(0.5) * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
  T dp = gm1 * (dQ[4] - rho * ke);
  T p = T(g.p_ref) + dp;
  T H = T(g.H_ref) + dQ[4] + dp;
  T gu[3][3], gp[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int c = 0; c < 3; ++c) gu[a][c] = (D[a][1 + c] - U[c] * D[a][0]) * ir;
    gp[a] = gm1 * (D[a][4] - (U[0] * D[a][1] + U[1] * D[a][2] + U[2] * D[a][3]) + ke * D[a][0]);
  }
  T theta = gu[0][0] + gu[1][1] + gu[2][2];
  T rho_t = -(U[0] * D[0][0] + U[1] * D[1][0] + U[2] * D[2][0] + rho * theta);
  T u_t[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) u_t[c] = -(U[0] * gu[0][c] + U[1] * gu[1][c] + U[2] * gu[2][c] + gp[c] * ir);
  T p_t = -(U[0] * gp[0] + U[1] * gp[1] + U[2] * gp[2] + gam * p * theta);
  T Uut = U[0] * u_t[0] + U[1] * u_t[1] + U[2] * u_t[2];
  T E_t = p_t * T(g.inv_gm1) + ke * rho_t + rho * Uut;
  T m0 = dQ[1];
  const T PF = T(g.pr_fix * g.cp);

  // ---- reverse
  T rho_b = T(0), ir_b = T(0), ke_b = T(0), dp_b = T(0), p_b = T(0), H_b = T(0), m0_b = T(0);
  T U_b[3] = {T(0), T(0), T(0)};
  T gu_b[3][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
  T gp_b[3] = {T(0), T(0), T(0)};
  T theta_b = T(0), rho_t_b = T(0), p_t_b = T(0), E_t_b = T(0);
  T u_t_b[3] = {T(0), T(0), T(0)};

  if (NEED_F) {
    T T0 = p * ir;
    T mu = T(g.mu_ref);
    if (VAR_MU) mu = mu * pow(T0 / T(g.T_ref), T(g.mu_exp));
    const T B = T(g.mub_m23);
    T s0 = mu * (T(2) * gu[0][0] + B * theta);
    T s1 = mu * (gu[0][1] + gu[1][0]);
    T s2 = mu * (gu[0][2] + gu[2][0]);
    T dTn = (gp[0] - T0 * D[0][0]) * ir;
    const T CK = T(g.cp * g.inv_pr);
    // F[0] = m0; F[1] = m0 U0 + dp - s0; F[2] = m0 U1 - s1; F[3] = m0 U2 - s2;
    // F[4] = U0 H - (U0 s0 + U1 s1 + U2 s2) - CK mu dTn
    m0_b += Fb[0] + Fb[1] * U[0] + Fb[2] * U[1] + Fb[3] * U[2];
    U_b[0] += Fb[1] * m0 + Fb[4] * (H - s0);
    U_b[1] += Fb[2] * m0 - Fb[4] * s1;
    U_b[2] += Fb[3] * m0 - Fb[4] * s2;
    dp_b += Fb[1];
    T s0_b = -Fb[1] - Fb[4] * U[0];
    T s1_b = -Fb[2] - Fb[4] * U[1];
    T s2_b = -Fb[3] - Fb[4] * U[2];
    H_b += Fb[4] * U[0];
    T mu_b = -CK * dTn * Fb[4];
    T dTn_b = -CK * mu * Fb[4];
    // dTn = (gp0 - T0 D00) ir
    gp_b[0] += dTn_b * ir;
    T T0_b = -dTn_b * D[0][0] * ir;
    Db[0][0] += -dTn_b * T0 * ir;
    ir_b += dTn_b * (gp[0] - T0 * D[0][0]);
    // stresses
    gu_b[0][0] += T(2) * mu * s0_b;
    theta_b += B * mu * s0_b;
    mu_b += s0_b * (T(2) * gu[0][0] + B * theta);
    gu_b[0][1] += mu * s1_b;
    gu_b[1][0] += mu * s1_b;
    mu_b += s1_b * (gu[0][1] + gu[1][0]);
    gu_b[0][2] += mu * s2_b;
    gu_b[2][0] += mu * s2_b;
    mu_b += s2_b * (gu[0][2] + gu[2][0]);
    // mu = mu_ref (T0/T_ref)^omega
    if (VAR_MU) T0_b += mu_b * T(g.mu_exp) * mu / T0;
    // T0 = p ir
    p_b += T0_b * ir;
    ir_b += T0_b * p;
  }
  // dF[4] = u_t0 H + U0 (E_t + p_t) + PF p u_t0
  u_t_b[0] += dFb[4] * (H + PF * p);
  H_b += dFb[4] * u_t[0];
  U_b[0] += dFb[4] * (E_t + p_t);
  E_t_b += dFb[4] * U[0];
  p_t_b += dFb[4] * U[0];
  p_b += dFb[4] * PF * u_t[0];
  // dF[3] = rho_t U0 U2 + rho (u_t0 U2 + U0 u_t2)
  rho_t_b += dFb[3] * U[0] * U[2];
  U_b[0] += dFb[3] * (rho_t * U[2] + rho * u_t[2]);
  U_b[2] += dFb[3] * (rho_t * U[0] + rho * u_t[0]);
  rho_b += dFb[3] * (u_t[0] * U[2] + U[0] * u_t[2]);
  u_t_b[0] += dFb[3] * rho * U[2];
  u_t_b[2] += dFb[3] * rho * U[0];
  // dF[2] = rho_t U0 U1 + rho (u_t0 U1 + U0 u_t1)
  rho_t_b += dFb[2] * U[0] * U[1];
  U_b[0] += dFb[2] * (rho_t * U[1] + rho * u_t[1]);
  U_b[1] += dFb[2] * (rho_t * U[0] + rho * u_t[0]);
  rho_b += dFb[2] * (u_t[0] * U[1] + U[0] * u_t[1]);
  u_t_b[0] += dFb[2] * rho * U[1];
  u_t_b[1] += dFb[2] * rho * U[0];
  // dF[1] = rho_t U0^2 + 2 m0 u_t0 + p_t
  rho_t_b += dFb[1] * U[0] * U[0];
  U_b[0] += dFb[1] * T(2) * rho_t * U[0];
  m0_b += dFb[1] * T(2) * u_t[0];
  u_t_b[0] += dFb[1] * T(2) * m0;
  p_t_b += dFb[1];
  // dF[0] = rho_t U0 + rho u_t0
  rho_t_b += dFb[0] * U[0];
  U_b[0] += dFb[0] * rho_t;
  rho_b += dFb[0] * u_t[0];
  u_t_b[0] += dFb[0] * rho;
  // m0 = dQ[1]
  dQb[1] += m0_b;
  // E_t = p_t/(gamma-1) + ke rho_t + rho sum_c U_c u_t_c
  p_t_b += E_t_b * T(g.inv_gm1);
  ke_b += E_t_b * rho_t;
  rho_t_b += E_t_b * ke;
  rho_b += E_t_b * Uut;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    U_b[c] += E_t_b * rho * u_t[c];
    u_t_b[c] += E_t_b * rho * U[c];
  }
  // p_t = -(sum_a U_a gp_a + gamma p theta)
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    U_b[a] -= p_t_b * gp[a];
    gp_b[a] -= p_t_b * U[a];
  }
  p_b -= p_t_b * gam * theta;
  theta_b -= p_t_b * gam * p;
  // u_t_c = -(sum_a U_a gu_ac + gp_c ir)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      U_b[a] -= u_t_b[c] * gu[a][c];
      gu_b[a][c] -= u_t_b[c] * U[a];
    }
    gp_b[c] -= u_t_b[c] * ir;
    ir_b -= u_t_b[c] * gp[c];
  }
  // rho_t = -(sum_a U_a D_a0 + rho theta)
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    U_b[a] -= rho_t_b * D[a][0];
    Db[a][0] -= rho_t_b * U[a];
  }
  rho_b -= rho_t_b * theta;
  theta_b -= rho_t_b * rho;
  // theta = sum_a gu_aa
#pragma unroll
  for (int a = 0; a < 3; ++a) gu_b[a][a] += theta_b;
  // gp_a = (gamma-1)(D_a4 - sum_c U_c D_a(1+c) + ke D_a0)
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T w = gm1 * gp_b[a];
    Db[a][4] += w;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Db[a][1 + c] -= w * U[c];
      U_b[c] -= w * D[a][1 + c];
    }
    ke_b += w * D[a][0];
    Db[a][0] += w * ke;
  }
  // gu_ac = (D_a(1+c) - U_c D_a0) ir
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T w = gu_b[a][c];
      Db[a][1 + c] += w * ir;
      U_b[c] -= w * D[a][0] * ir;
      Db[a][0] -= w * U[c] * ir;
      ir_b += w * (D[a][1 + c] - U[c] * D[a][0]);
    }
  // H = H_ref + dQ4 + dp ; p = p_ref + dp
  dQb[4] += H_b;
  dp_b += H_b + p_b;
  // dp = (gamma-1)(dQ4 - rho ke)
  dQb[4] += gm1 * dp_b;
  rho_b -= gm1 * dp_b * ke;
  ke_b -= gm1 * dp_b * rho;
  // ke = |U|^2/2 ; U_c = dQ_(1+c) ir
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    U_b[c] += ke_b * U[c];
    dQb[1 + c] += U_b[c] * ir;
    ir_b += U_b[c] * dQ[1 + c];
  }
  // ir = 1/rho ; rho = rho_ref + dQ0
  rho_b -= ir_b * ir * ir;
  dQb[0] += rho_b;
}

// ---------------------------------------------------------------------------
// Adjoint of compat_dev: given the cotangent Q0b of the interface equilibrium
// state, accumulates the cotangents of the two reconstructed states.
// ---------------------------------------------------------------------------
template <typename T>
struct SideB {
  T rho, U, V, W, p, dp, h, th;
};

template <typename T>
__host__ __device__ __forceinline__ void side_state_vjp(const Geo& g, const T* dQ, const Side<T>& s, const SideB<T>& b,
                                               T* dQb) {
  const T kInvSqrtPi = T(0.56418958354775628695);
  T ir = T(1) / s.rho;
  T lam = T(0.5) * s.rho / s.p;
  T sl = sqrt(lam);
  T x = sl * s.U;
  T ex = exp(-x * x);
  T rho_b = b.rho, U_b = b.U, V_b = b.V, W_b = b.W, p_b = b.p, dp_b = b.dp;
  // th = kInvSqrtPi exp(-x^2) / (2 sl) ; h = erf(x)/2
  T x_b = b.th * s.th * (T(-2) * x) + b.h * kInvSqrtPi * ex;
  T sl_b = -b.th * s.th / sl;
  // x = sl U
  sl_b += x_b * s.U;
  U_b += x_b * sl;
  // sl = sqrt(lam) ; lam = rho / (2 p)
  T lam_b = sl_b * T(0.5) / sl;
  rho_b += lam_b * T(0.5) / s.p;
  p_b -= lam_b * lam / s.p;
  // p = p_ref + dp ; dp = (gamma-1)(dQ4 - rho |U|^2/2)
  dp_b += p_b;
  const T gm1 = T(g.gm1);
  dQb[4] += gm1 * dp_b;
  rho_b -= gm1 * dp_b * T(0.5) * (s.U * s.U + s.V * s.V + s.W * s.W);
  U_b -= gm1 * dp_b * s.rho * s.U;
  V_b -= gm1 * dp_b * s.rho * s.V;
  W_b -= gm1 * dp_b * s.rho * s.W;
  // U = dQ1 ir, V = dQ2 ir, W = dQ3 ir ; ir = 1/rho ; rho = rho_ref + dQ0
  dQb[1] += U_b * ir;
  dQb[2] += V_b * ir;
  dQb[3] += W_b * ir;
  T ir_b = U_b * dQ[1] + V_b * dQ[2] + W_b * dQ[3];
  rho_b -= ir_b * ir * ir;
  dQb[0] += rho_b;
}

template <typename T>
__host__ __device__ __forceinline__ void compat_dev_vjp(const Geo& g, const T* dQl, const T* dQr, const T* Q0b, T* dQlb,
                                               T* dQrb) {
  Side<T> l = side_state(g, dQl), r = side_state(g, dQr);
  T a0 = T(0.5) + l.h, b0 = T(0.5) - r.h;
  T a1 = l.U * a0 + l.th, b1 = r.U * b0 - r.th;
  SideB<T> lb = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
  SideB<T> rb = lb;
  T a0_b = T(0), a1_b = T(0), b0_b = T(0), b1_b = T(0);
  const T ig = T(g.inv_gm1);
  // Q0[4] = (rho_l (U_l a1 + a0 (V_l^2+W_l^2)) + rho_r (U_r b1 + b0 (V_r^2+W_r^2)))/2
  //         + ((dp_l + dp_r)/2 + h_l p_l - h_r p_r)/(gamma-1)
  {
    T e = Q0b[4];
    T vwl = l.V * l.V + l.W * l.W, vwr = r.V * r.V + r.W * r.W;
    lb.rho += T(0.5) * e * (l.U * a1 + a0 * vwl);
    lb.U += T(0.5) * e * l.rho * a1;
    a1_b += T(0.5) * e * l.rho * l.U;
    a0_b += T(0.5) * e * l.rho * vwl;
    lb.V += e * l.rho * a0 * l.V;
    lb.W += e * l.rho * a0 * l.W;
    rb.rho += T(0.5) * e * (r.U * b1 + b0 * vwr);
    rb.U += T(0.5) * e * r.rho * b1;
    b1_b += T(0.5) * e * r.rho * r.U;
    b0_b += T(0.5) * e * r.rho * vwr;
    rb.V += e * r.rho * b0 * r.V;
    rb.W += e * r.rho * b0 * r.W;
    lb.dp += T(0.5) * e * ig;
    rb.dp += T(0.5) * e * ig;
    lb.h += e * l.p * ig;
    lb.p += e * l.h * ig;
    rb.h -= e * r.p * ig;
    rb.p -= e * r.h * ig;
  }
  // Q0[3] = rho_l W_l a0 + rho_r W_r b0 ; Q0[2] likewise with V
  {
    T e = Q0b[3];
    lb.rho += e * l.W * a0;
    lb.W += e * l.rho * a0;
    a0_b += e * l.rho * l.W;
    rb.rho += e * r.W * b0;
    rb.W += e * r.rho * b0;
    b0_b += e * r.rho * r.W;
    e = Q0b[2];
    lb.rho += e * l.V * a0;
    lb.V += e * l.rho * a0;
    a0_b += e * l.rho * l.V;
    rb.rho += e * r.V * b0;
    rb.V += e * r.rho * b0;
    b0_b += e * r.rho * r.V;
  }
  // Q0[1] = rho_l a1 + rho_r b1
  lb.rho += Q0b[1] * a1;
  a1_b += Q0b[1] * l.rho;
  rb.rho += Q0b[1] * b1;
  b1_b += Q0b[1] * r.rho;
  // Q0[0] = (dQl0 + dQr0)/2 + rho_l h_l - rho_r h_r
  dQlb[0] += T(0.5) * Q0b[0];
  dQrb[0] += T(0.5) * Q0b[0];
  lb.rho += Q0b[0] * l.h;
  lb.h += Q0b[0] * l.rho;
  rb.rho -= Q0b[0] * r.h;
  rb.h -= Q0b[0] * r.rho;
  // a1 = U_l a0 + th_l ; b1 = U_r b0 - th_r ; a0 = 1/2 + h_l ; b0 = 1/2 - h_r
  lb.U += a1_b * a0;
  a0_b += a1_b * l.U;
  lb.th += a1_b;
  rb.U += b1_b * b0;
  b0_b += b1_b * r.U;
  rb.th -= b1_b;
  lb.h += a0_b;
  rb.h -= b0_b;
  side_state_vjp(g, dQl, l, lb, dQlb);
  side_state_vjp(g, dQr, r, rb, dQrb);
}

// Cotangent accumulation: LDS (one workgroup) and device memory (all of them).
template <typename T>
__device__ __forceinline__ void lds_add(T* p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void global_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace hgks
