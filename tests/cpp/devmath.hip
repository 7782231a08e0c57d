// Host build of the library's scalar device math (the same headers the kernels
// use), so that the tests can check it on the CPU: forward Gauss-point flux and
// compatibility state against the oracle, and each hand-written vector-Jacobian
// product against central differences of its forward function.
#include <cmath>

#include "../../paper_2005_08736_amd/csrc/adjoint_common.hpp"
#include "../../paper_2005_08736_amd/csrc/zadjoint_common.hpp"
#include "../../paper_2005_08736_amd/csrc/zflux.hpp"

using namespace hgks;

static Geo make(double gamma, double prandtl, double mu, double rho_ref, double p_ref) {
  Geo g{};
  g.gamma = gamma;
  g.gm1 = gamma - 1.0;
  g.inv_gm1 = 1.0 / g.gm1;
  g.cp = gamma / (gamma - 1.0);
  g.inv_pr = 1.0 / prandtl;
  g.pr_fix = 1.0 / prandtl - 1.0;
  g.K = (5.0 - 3.0 * gamma) / (gamma - 1.0);
  g.mub_m23 = 2.0 * g.K / (3.0 * (g.K + 3.0)) - 2.0 / 3.0;
  g.mu_ref = mu;
  g.T_ref = 1.0;
  g.mu_exp = 0.0;
  g.rho_ref = rho_ref;
  g.p_ref = p_ref;
  g.E_ref = p_ref / g.gm1;
  g.H_ref = gamma * p_ref / g.gm1;
  return g;
}

extern "C" {

// Q: full state (local frame), D[15]: derivatives; F excludes p_ref in F[1]
int dm_smooth_flux(const double* Q, const double* D, double gamma, double prandtl, double mu, double rho_ref,
                   double p_ref, double* F, double* dF) {
  Geo g = make(gamma, prandtl, mu, rho_ref, p_ref);
  double dQ[5] = {Q[0] - rho_ref, Q[1], Q[2], Q[3], Q[4] - g.E_ref};
  double d[3][5];
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 5; ++k) d[a][k] = D[a * 5 + k];
  smooth_flux<true, false>(g, dQ, d, F, dF);
  return 0;
}

int dm_smooth_flux_vjp(const double* Q, const double* D, double gamma, double prandtl, double mu, double rho_ref,
                       double p_ref, const double* Fb, const double* dFb, double* Qb, double* Db) {
  Geo g = make(gamma, prandtl, mu, rho_ref, p_ref);
  double dQ[5] = {Q[0] - rho_ref, Q[1], Q[2], Q[3], Q[4] - g.E_ref};
  double d[3][5], db[3][5] = {};
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 5; ++k) d[a][k] = D[a * 5 + k];
  double qb[5] = {0, 0, 0, 0, 0};
  smooth_flux_vjp<true, false>(g, dQ, d, Fb, dFb, qb, db);
  for (int k = 0; k < 5; ++k) Qb[k] = qb[k];
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 5; ++k) Db[a * 5 + k] = db[a][k];
  return 0;
}

int dm_compat(const double* Ql, const double* Qr, double gamma, double rho_ref, double p_ref, double* Q0) {
  Geo g = make(gamma, 1.0, 0.0, rho_ref, p_ref);
  double l[5] = {Ql[0] - rho_ref, Ql[1], Ql[2], Ql[3], Ql[4] - g.E_ref};
  double r[5] = {Qr[0] - rho_ref, Qr[1], Qr[2], Qr[3], Qr[4] - g.E_ref};
  double q0[5];
  compat_dev(g, l, r, q0);
  Q0[0] = q0[0] + rho_ref;
  for (int k = 1; k < 4; ++k) Q0[k] = q0[k];
  Q0[4] = q0[4] + g.E_ref;
  return 0;
}

int dm_compat_vjp(const double* Ql, const double* Qr, double gamma, double rho_ref, double p_ref, const double* Q0b,
                  double* Qlb, double* Qrb) {
  Geo g = make(gamma, 1.0, 0.0, rho_ref, p_ref);
  double l[5] = {Ql[0] - rho_ref, Ql[1], Ql[2], Ql[3], Ql[4] - g.E_ref};
  double r[5] = {Qr[0] - rho_ref, Qr[1], Qr[2], Qr[3], Qr[4] - g.E_ref};
  double lb[5] = {0, 0, 0, 0, 0}, rb[5] = {0, 0, 0, 0, 0};
  compat_dev_vjp(g, l, r, Q0b, lb, rb);
  for (int k = 0; k < 5; ++k) { Qlb[k] = lb[k]; Qrb[k] = rb[k]; }
  return 0;
}

// WENO-Z value and slope at the right edge of the middle of v[0..4]
int dm_weno_z_right(const double* v, double eps, int p, double* val, double* slope) {
  weno_z_right(v, eps, p, *val, *slope);
  return 0;
}

// WENO-Z edge values of the middle of v[0..4]
int dm_weno_z_edges(const double* v, double eps, int p, double* ea, double* eb) {
  weno_z_edges(v, eps, p, *ea, *eb);
  return 0;
}

// Full flux at one Gauss point with a given collision time; states are full
// (local frame), derivatives D[a*5+k]; F excludes p_ref in F[1]
int dm_full_flux(const double* Ql, const double* Dl, const double* Qr, const double* Dr, const double* Q0,
                 const double* D0, double tau, double dt, double gamma, double prandtl, double rho_ref, double p_ref,
                 double* F, double* dF) {
  Geo g = make(gamma, prandtl, 0.0, rho_ref, p_ref);
  auto dev = [&](const double* Q, double* d) {
    d[0] = Q[0] - rho_ref;
    d[1] = Q[1];
    d[2] = Q[2];
    d[3] = Q[3];
    d[4] = Q[4] - g.E_ref;
  };
  double l[5], r[5], z[5], dl[3][5], dr[3][5], dz[3][5];
  dev(Ql, l);
  dev(Qr, r);
  dev(Q0, z);
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 5; ++k) {
      dl[a][k] = Dl[a * 5 + k];
      dr[a][k] = Dr[a * 5 + k];
      dz[a][k] = D0[a * 5 + k];
    }
  full_flux_tau(g, z, dz, l, dl, r, dr, tau, dt, F, dF);
  return 0;
}

// Mode-Z Gauss-point flux of the 60 deviation inputs X (Q0, Q_l, Q_r, then D0,
// D_l, D_r each [3][5]) with tau = mu(T0)/p0 + c_art |p_l - p_r|/(p_l + p_r) dt,
// mu(T) = mu (T/T_ref)^mu_exp; and the transpose of its Jacobian applied to the
// cotangents (Fb, dFb), from forward tangents.
static Geo make_z(double gamma, double prandtl, double mu, double T_ref, double mu_exp, double c_art, double rho_ref,
                  double p_ref) {
  Geo g = make(gamma, prandtl, mu, rho_ref, p_ref);
  g.T_ref = T_ref;
  g.mu_exp = mu_exp;
  g.c_art = c_art;
  return g;
}

int dm_zgp_flux(const double* X, double dt, double gamma, double prandtl, double mu, double T_ref, double mu_exp,
                double c_art, double rho_ref, double p_ref, double* F, double* dF) {
  Geo g = make_z(gamma, prandtl, mu, T_ref, mu_exp, c_art, rho_ref, p_ref);
  if (mu_exp != 0.0) zgp_flux<true>(g, X, dt, F, dF);
  else zgp_flux<false>(g, X, dt, F, dF);
  return 0;
}

int dm_zflux_jt(const double* X, double dt, double gamma, double prandtl, double mu, double T_ref, double mu_exp,
                double c_art, double rho_ref, double p_ref, const double* Fb, const double* dFb, double* Xb) {
  Geo g = make_z(gamma, prandtl, mu, T_ref, mu_exp, c_art, rho_ref, p_ref);
  for (int c0 = 0; c0 < kXN; c0 += kZTan) {
    if (mu_exp != 0.0) zflux_jt_columns<true>(g, X, c0, dt, Fb, dFb, Xb);
    else zflux_jt_columns<false>(g, X, c0, dt, Fb, dFb, Xb);
  }
  return 0;
}

// The same by the kernel's hand-written reverse sweep
int dm_zflux_vjp(const double* X, double dt, double gamma, double prandtl, double mu, double T_ref, double mu_exp,
                 double c_art, double rho_ref, double p_ref, const double* Fb, const double* dFb, double* Xb) {
  Geo g = make_z(gamma, prandtl, mu, T_ref, mu_exp, c_art, rho_ref, p_ref);
  if (mu_exp != 0.0) zflux_jt_all<true>(g, X, dt, Fb, dFb, Xb);
  else zflux_jt_all<false>(g, X, dt, Fb, dFb, Xb);
  return 0;
}

// The hand-written reverses of the WENO-Z edge pair and right-edge value/slope:
// vb = J^T (cotangents)
int dm_wze_vjp(const double* v, double eps, int p, double eab, double ebb, double* vb) {
  for (int i = 0; i < 5; ++i) vb[i] = 0.0;
  weno_z_edges_vjp(v, eps, p, eab, ebb, vb);
  return 0;
}
int dm_wzr_vjp(const double* v, double eps, int p, double valb, double slopeb, double* vb) {
  for (int i = 0; i < 5; ++i) vb[i] = 0.0;
  weno_z_right_vjp(v, eps, p, valb, slopeb, vb);
  return 0;
}

// Jacobians of the WENO-Z edge pair (J[2][5]) and of the right-edge value and
// slope (Jv[5], Js[5]) of a five-value line
int dm_wze_jac(const double* v, double eps, int p, double* J) {
  wze_jac(v, eps, p, reinterpret_cast<double(*)[5]>(J));
  return 0;
}

int dm_wzr_jac(const double* v, double eps, int p, double* Jv, double* Js) {
  wzr_jac(v, eps, p, Jv, Js);
  return 0;
}

}  // extern "C"
