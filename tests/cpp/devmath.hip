// Host build of the library's scalar device math (the same headers the kernels
// use), so that the tests can check it on the CPU: forward Gauss-point flux and
// compatibility state against the oracle, and each hand-written vector-Jacobian
// product against central differences of its forward function.
#include <cmath>

#include "../../paper_2005_08736_amd/csrc/adjoint_common.hpp"

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

}  // extern "C"
