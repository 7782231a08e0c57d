"""Pins of the oracle's kinetic building blocks (Sec. 2.1 of the paper) against
independent mathematics: numerical quadrature of Maxwellian moments, the Euler
flux and its Jacobians (complex-step differentiation of a flux written here),
the Navier-Stokes stress and Fourier heat flux, Gauss-Legendre integration in
time, and kinetic flux-vector splitting."""
import math

import numpy as np
import pytest

from tests import quadrature as Qd

GAMMA = 1.4
K = (5 - 3 * GAMMA) / (GAMMA - 1)
rng = np.random.default_rng(20050873)


def cons(r, u, v, w, p, g=GAMMA):
    return np.array([r, r * u, r * v, r * w, p / (g - 1) + 0.5 * r * (u * u + v * v + w * w)])


def prim(Q, g=GAMMA):
    r = Q[0]
    U = Q[1:4] / r
    p = (g - 1) * (Q[4] - 0.5 * np.dot(Q[1:4], Q[1:4]) / r)
    return r, U, p


def flux_d(Q, d, g=GAMMA):
    r = Q[0]
    U = Q[1:4] / r
    p = (g - 1) * (Q[4] - 0.5 * (Q[1] ** 2 + Q[2] ** 2 + Q[3] ** 2) / r)
    out = np.empty(5, dtype=Q.dtype)
    out[0] = r * U[d]
    out[1:4] = r * U[d] * U
    out[1 + d] += p
    out[4] = U[d] * (Q[4] + p)
    return out


def jacobian(Q, d):
    J = np.zeros((5, 5))
    for k in range(5):
        e = np.zeros(5, dtype=complex)
        e[k] = 1e-30j
        J[:, k] = flux_d(Q.astype(complex) + e, d).imag / 1e-30
    return J


def random_state():
    r = 0.5 + rng.random()
    U = rng.normal(size=3)
    p = 0.5 + rng.random()
    return cons(r, *U, p)


# ---------------------------------------------------------------------------
def test_moments_full_and_half_match_quadrature(oracle_mod):
    for _ in range(5):
        U, lam = rng.normal(), 0.3 + 2 * rng.random()
        full, plus = oracle_mod.moments_1d(U, lam)
        for n in range(7):
            ref_full = Qd.expect(lambda u, v, w, x: u ** n, U, 0.0, 0.0, lam)
            ref_plus = Qd.expect(lambda u, v, w, x: u ** n, U, 0.0, 0.0, lam, half=+1)
            assert abs(full[n] - ref_full) <= 1e-13 * max(1.0, abs(ref_full))
            assert abs(plus[n] - ref_plus) <= 1e-12 * max(1.0, abs(ref_plus))


@pytest.mark.parametrize("half", [0, 1, -1])
def test_psi_moments_match_quadrature(oracle_mod, half):
    for _ in range(3):
        U, V, W = rng.normal(size=3)
        lam = 0.4 + rng.random()
        X = rng.normal(size=5)
        for (a, b, c) in [(0, 0, 0), (1, 0, 0), (2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 0), (0, 0, 1)]:
            got = oracle_mod.psimom(U, V, W, lam, K, half, a, b, c, X)
            for k in range(5):
                ref = Qd.expect(lambda u, v, w, x: u ** a * v ** b * w ** c * Qd.phi(X, u, v, w, x)
                                * Qd.psi(u, v, w, x)[k], U, V, W, lam, half=half)
                assert abs(got[k] - ref) <= 2e-12 * max(1.0, abs(ref)), (a, b, c, k, got[k], ref)


def test_microslope_solves_moment_system(oracle_mod):
    for _ in range(5):
        U, V, W = rng.normal(size=3)
        lam = 0.3 + rng.random()
        b = rng.normal(size=5)
        a = oracle_mod.microslope(b, U, V, W, lam, K)
        for k in range(5):
            ref = Qd.expect(lambda u, v, w, x: Qd.phi(a, u, v, w, x) * Qd.psi(u, v, w, x)[k], U, V, W, lam)
            assert abs(ref - b[k]) <= 1e-12 * max(1.0, abs(b[k]))


def test_compat_identity_and_half_space_quadrature(oracle_mod):
    for _ in range(5):
        Q = random_state()
        assert np.allclose(oracle_mod.compat(Q, Q, GAMMA), Q, rtol=1e-15, atol=1e-15)
    Ql, Qr = random_state(), random_state()
    Q0 = oracle_mod.compat(Ql, Qr, GAMMA)
    rl, Ul, pl = prim(Ql)
    rr, Ur, pr = prim(Qr)
    for k in range(5):
        ref = rl * Qd.expect(lambda u, v, w, x: Qd.psi(u, v, w, x)[k], *Ul, rl / (2 * pl), half=+1) + \
              rr * Qd.expect(lambda u, v, w, x: Qd.psi(u, v, w, x)[k], *Ur, rr / (2 * pr), half=-1)
        assert abs(Q0[k] - ref) <= 1e-12 * max(1.0, abs(ref))


# ---------------------------------------------------------------------------
def test_smooth_flux_euler_limit(oracle_mod):
    for _ in range(5):
        Q = random_state()
        F0, F1 = oracle_mod.gp_flux_smooth(Q, np.zeros(15), 0.0, GAMMA, 0.72)
        assert np.allclose(F0, flux_d(Q, 0), rtol=1e-14, atol=1e-14)
        assert np.allclose(F1, 0.0, atol=1e-14)


def test_smooth_flux_time_derivative_is_jacobian_times_euler_dqdt(oracle_mod):
    for _ in range(5):
        Q = random_state()
        dQ = rng.normal(size=(3, 5)) * 0.3
        _, F1 = oracle_mod.gp_flux_smooth(Q, dQ.ravel(), 0.01, GAMMA, 1.0)
        dtQ = -sum(jacobian(Q, d) @ dQ[d] for d in range(3))
        ref = jacobian(Q, 0) @ dtQ
        assert np.allclose(F1, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def ns_flux(Q, dQ, mu, prandtl, g=GAMMA):
    """Navier-Stokes normal flux with Stokes stress, bulk viscosity
    mu_b = 2K/(3(K+3)) mu (Sec. 3.1) and Fourier heat flux c_p mu / Pr (R = 1)."""
    r, U, p = prim(Q, g)
    T = p / r
    Kd = (5 - 3 * g) / (g - 1)
    gU = np.array([(dQ[a][1:4] - U * dQ[a][0]) / r for a in range(3)])  # gU[a][c] = dU_c/dx_a
    dp = np.array([(g - 1) * (dQ[a][4] - U @ dQ[a][1:4] + 0.5 * (U @ U) * dQ[a][0]) for a in range(3)])
    dT = (dp - T * dQ[:, 0]) / r
    th = np.trace(gU)
    mub = 2 * Kd / (3 * (Kd + 3)) * mu
    sig = mu * (gU + gU.T - 2.0 / 3.0 * th * np.eye(3)) + mub * th * np.eye(3)
    cp = g / (g - 1)
    F = flux_d(Q, 0, g).copy()
    F[1:4] -= sig[0]
    F[4] -= U @ sig[0] + cp * mu / prandtl * dT[0]
    return F


@pytest.mark.parametrize("prandtl", [1.0, 0.72])
@pytest.mark.parametrize("gamma", [GAMMA, 5.0 / 3.0, 1.3])
def test_smooth_flux_is_navier_stokes(oracle_mod, prandtl, gamma):
    """For every gamma, K = (5 - 3 gamma)/(gamma - 1) internal degrees of freedom:
    the monatomic gas (K = 0) has no bulk viscosity, K = 2 (gamma = 1.4) gives
    4/15 mu, K = 11/3 (gamma = 1.3) 11/30 mu."""
    for _ in range(5):
        r, U, pr = 0.5 + rng.random(), rng.normal(size=3), 0.5 + rng.random()
        Q = cons(r, *U, pr, g=gamma)
        dQ = rng.normal(size=(3, 5)) * 0.3
        tau = 0.02 * rng.random()
        F0, _ = oracle_mod.gp_flux_smooth(Q, dQ.ravel(), tau, gamma, prandtl)
        _, _, p = prim(Q, gamma)
        ref = ns_flux(Q, dQ, tau * p, prandtl, gamma)
        assert np.allclose(F0, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_prandtl_fix_on_time_derivative(oracle_mod):
    # The heat flux about the interface velocity of g0 * Abar is d/dt of the heat
    # flux of a Maxwellian whose velocity moves away from U0: c_p p dU_n/dt (R = 1).
    Q = random_state()
    dQ = rng.normal(size=(3, 5)) * 0.3
    _, F1a = oracle_mod.gp_flux_smooth(Q, dQ.ravel(), 0.01, GAMMA, 1.0)
    _, F1b = oracle_mod.gp_flux_smooth(Q, dQ.ravel(), 0.01, GAMMA, 0.72)
    r, U, p = prim(Q)
    dtQ = -sum(jacobian(Q, d) @ dQ[d] for d in range(3))
    dUn = (dtQ[1] - U[0] * dtQ[0]) / r
    cp = GAMMA / (GAMMA - 1)
    assert np.allclose(F1b[:4], F1a[:4], rtol=0, atol=0)
    assert abs((F1b[4] - F1a[4]) - (1 / 0.72 - 1) * cp * p * dUn) <= 1e-12 * abs(F1a[4])


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("gamma", [GAMMA, 5.0 / 3.0, 1.3])
def test_full_flux_reduces_to_smooth_for_continuous_data(oracle_mod, gamma):
    for _ in range(4):
        r, U, pr = 0.5 + rng.random(), rng.normal(size=3), 0.5 + rng.random()
        Q = cons(r, *U, pr, g=gamma)
        dQ = rng.normal(size=(3, 5)) * 0.3
        tau, dt = 0.003 + 0.01 * rng.random(), 0.01 + 0.02 * rng.random()
        F, dF = oracle_mod.gp_flux_full(Q, dQ.ravel(), Q, dQ.ravel(), Q, dQ.ravel(), tau, dt, gamma, 0.72)
        F0, F1 = oracle_mod.gp_flux_smooth(Q, dQ.ravel(), tau, gamma, 0.72)
        assert np.allclose(F, F0, rtol=1e-12, atol=1e-12 * np.abs(F0).max())
        assert np.allclose(dF, F1, rtol=1e-9, atol=1e-9 * np.abs(F1).max())


def test_full_flux_time_integrals_match_gauss_legendre(oracle_mod):
    x, w = np.polynomial.legendre.leggauss(64)
    for _ in range(3):
        Ql, Qr = random_state(), random_state()
        Q0 = oracle_mod.compat(Ql, Qr, GAMMA)
        dl, dr, d0 = (rng.normal(size=15) * 0.3 for _ in range(3))
        tau = 0.002 + 0.01 * rng.random()
        delta = 0.004 + 0.02 * rng.random()
        I, _ = oracle_mod.gp_flux_full_parts(Ql, dl, Qr, dr, Q0, d0, tau, delta, 0.0, GAMMA, 1.0)
        ref = np.zeros(5)
        for xi, wi in zip(x, w):
            t = 0.5 * delta * (xi + 1)
            _, Ft = oracle_mod.gp_flux_full_parts(Ql, dl, Qr, dr, Q0, d0, tau, delta, t, GAMMA, 1.0)
            ref += 0.5 * delta * wi * Ft
        assert np.allclose(I, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_full_flux_initial_value_is_kinetic_flux_vector_splitting(oracle_mod):
    Ql, Qr = random_state(), random_state()
    Q0 = oracle_mod.compat(Ql, Qr, GAMMA)
    z = np.zeros(15)
    _, F_t0 = oracle_mod.gp_flux_full_parts(Ql, z, Qr, z, Q0, z, 0.01, 0.01, 0.0, GAMMA, 1.0)
    rl, Ul, pl = prim(Ql)
    rr, Ur, pr = prim(Qr)
    for k in range(5):
        ref = rl * Qd.expect(lambda u, v, w, x: u * Qd.psi(u, v, w, x)[k], *Ul, rl / (2 * pl), half=+1) + \
              rr * Qd.expect(lambda u, v, w, x: u * Qd.psi(u, v, w, x)[k], *Ur, rr / (2 * pr), half=-1)
        assert abs(F_t0[k] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_full_flux_supersonic_upwinding(oracle_mod):
    # flow to the right at Mach ~ 8 with small tau: the interface flux is the
    # Euler flux of the left state (the g_l half space carries all particles)
    Ql = cons(1.0, 8.0, 0.1, -0.2, 1.0 / GAMMA)
    Qr = cons(0.5, 7.0, 0.0, 0.3, 0.8 / GAMMA)
    Q0 = oracle_mod.compat(Ql, Qr, GAMMA)
    z = np.zeros(15)
    F, _ = oracle_mod.gp_flux_full(Ql, z, Qr, z, Q0, z, 1e-8, 1e-3, GAMMA, 1.0)
    ref = flux_d(Ql, 0)
    assert np.allclose(F, ref, rtol=1e-6)


# ---------------------------------------------------------------------------
def _cell_avg_monomial(m, j):
    a, b = j - 0.5, j + 0.5
    return (b ** (m + 1) - a ** (m + 1)) / (m + 1)


def test_reconstruction_weights_exact_on_polynomials(oracle_mod):
    W = oracle_mod.weights()
    s = 1 / (2 * math.sqrt(3))
    for m in range(5):  # exact for degree <= 4
        avgs = np.array([_cell_avg_monomial(m, j) for j in (-2, -1, 0, 1, 2)])
        for gp, x0 in enumerate((-s, s)):
            assert abs(W["tan_val"][gp] @ avgs - x0 ** m) < 1e-14
            assert abs(W["tan_der"][gp] @ avgs - (m * x0 ** (m - 1) if m else 0.0)) < 1e-13
        # normal derivative at x = 1/2 from cells -1..2 and the point value there
        a4 = np.array([_cell_avg_monomial(m, j) for j in (-1, 0, 1, 2)] + [0.5 ** m])
        assert abs(W["dn"] @ a4 - (m * 0.5 ** (m - 1) if m else 0.0)) < 1e-13
    # the printed (sympy-free) fact: the Q0 weight of the normal derivative vanishes
    assert abs(W["dn"][4]) < 1e-14


def test_weno5_linear_exact_and_z_weights_behave(oracle_mod):
    for m in range(5):
        avgs = np.array([_cell_avg_monomial(m, j) for j in (-2, -1, 0, 1, 2)])
        val, slope = oracle_mod.weno5(avgs, linear=True)
        assert abs(val - 0.5 ** m) < 1e-13
        if m <= 2:
            assert abs(slope - (m * 0.5 ** (m - 1) if m else 0.0)) < 1e-13
    # WENO-Z on smooth data is close to the linear value; across a step it picks the smooth side
    v = np.sin(0.3 * np.arange(5))
    lin, _ = oracle_mod.weno5(v, linear=True)
    z, _ = oracle_mod.weno5(v, linear=False)
    assert abs(z - lin) < 1e-4
    step = np.array([0.0, 0.0, 0.0, 1.0, 1.0])
    z, _ = oracle_mod.weno5(step, linear=False)
    assert abs(z) < 0.05


def test_oracle_rounding_bound_at_low_mach(oracle_mod):
    """Measures the FP64 rounding error of the oracle's moment algebra at the
    Taylor-Green conditions (T = p/rho ~ 71): moments about u = 0 grow like T^3
    and cancel, so F1 carries up to a few 1e-12 relative error.  This bound sets
    the tolerance of the GPU parity checks on dF and dL."""
    rng2 = np.random.default_rng(7)
    worst0 = worst1 = 0.0
    for _ in range(200):
        r = 1 + 0.01 * rng2.normal()
        U = rng2.normal(size=3)
        p = 71.4 + 0.2 * rng2.normal()
        Q = cons(r, *U, p)
        dQ = rng2.normal(size=15)
        tau = (1 / 1600) / p
        F0, F1 = oracle_mod.gp_flux_smooth(Q, dQ, tau, GAMMA, 0.72)
        E0, E1 = oracle_mod.gp_flux_smooth_ext(Q, dQ, tau, GAMMA, 0.72)
        worst0 = max(worst0, np.abs(F0 - E0).max() / np.abs(E0).max())
        worst1 = max(worst1, np.abs(F1 - E1).max() / np.abs(E1).max())
    assert worst0 < 1e-13, worst0
    assert worst1 < 5e-12, worst1
    # at unit temperature the same algebra is accurate to round-off
    Q = cons(1.0, 0.3, -0.2, 0.1, 1.0)
    dQ = rng2.normal(size=15)
    F0, F1 = oracle_mod.gp_flux_smooth(Q, dQ, 0.01, GAMMA, 0.72)
    E0, E1 = oracle_mod.gp_flux_smooth_ext(Q, dQ, 0.01, GAMMA, 0.72)
    assert np.abs(F1 - E1).max() <= 1e-14 * np.abs(E1).max()
