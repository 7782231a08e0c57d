"""CPU checks of the library's scalar device math, built for the host from the
same headers the kernels use: the Gauss-point flux and compatibility state
against the oracle, and the hand-written vector-Jacobian products against
central differences of the forward functions (no GPU needed)."""
import zlib

import numpy as np
import pytest

from tests import devmath

GAMMA = 1.4
rng = np.random.default_rng(11)


@pytest.fixture(autouse=True)
def _seed_per_test(request):
    """Each test draws from its own stream, seeded by its id, so that its inputs
    do not depend on which tests ran before it in the same process."""
    global rng
    rng = np.random.default_rng(zlib.crc32(request.node.nodeid.encode()))


def cons(r, U, p, g=GAMMA):
    return np.array([r, r * U[0], r * U[1], r * U[2], p / (g - 1) + 0.5 * r * (U @ U)])


def states(p_level):
    r = 1 + 0.05 * rng.normal()
    return cons(r, rng.normal(size=3), p_level * (1 + 0.01 * rng.normal()))


@pytest.mark.parametrize("p_level", [1.0, 71.4])
def test_device_flux_and_compat_match_oracle(oracle_mod, p_level):
    rho_ref, p_ref = 1.0, p_level
    for _ in range(20):
        Q = states(p_level)
        D = rng.normal(size=15)
        mu = 1e-3
        F, dF = devmath.smooth_flux(Q, D, GAMMA, 0.72, mu, rho_ref, p_ref)
        F[1] += p_ref
        r = Q[0]
        p = (GAMMA - 1) * (Q[4] - 0.5 * (Q[1:4] @ Q[1:4]) / r)
        F0, F1 = oracle_mod.gp_flux_smooth(Q, D, mu / p, GAMMA, 0.72)
        assert np.abs(F - F0).max() <= 1e-13 * np.abs(F0).max()
        # the oracle's F1 carries up to ~2e-12 relative rounding at p ~ 71
        assert np.abs(dF - F1).max() <= 5e-12 * np.abs(F1).max()
        Ql, Qr = states(p_level), states(p_level)
        Q0 = devmath.compat(Ql, Qr, GAMMA, rho_ref, p_ref)
        assert np.abs(Q0 - oracle_mod.compat(Ql, Qr, GAMMA)).max() <= 1e-13 * np.abs(Q0).max()


def _fd_check(f, x, v, wb, h):
    """<wb, J v> by central differences of f at x along v, Richardson-extrapolated
    over steps h and h/2 (truncation error O(h^4))."""
    def cd(hh):
        return float(wb @ ((f(x + hh * v) - f(x - hh * v)) / (2 * hh)))
    return (4 * cd(h / 2) - cd(h)) / 3


@pytest.mark.parametrize("p_level", [1.0, 71.4])
def test_smooth_flux_vjp_matches_central_differences(p_level):
    rho_ref, p_ref = 1.0, p_level
    for _ in range(10):
        Q = states(p_level)
        D = rng.normal(size=15)
        Fb, dFb = rng.normal(size=5), rng.normal(size=5)

        def f(x):
            F, dF = devmath.smooth_flux(x[:5], x[5:], GAMMA, 0.72, 2e-3, rho_ref, p_ref)
            return np.concatenate([F, dF])

        x = np.concatenate([Q, D])
        v = rng.normal(size=20)
        Qb, Db = devmath.smooth_flux_vjp(Q, D, GAMMA, 0.72, 2e-3, rho_ref, p_ref, Fb, dFb)
        lhs = float(np.concatenate([Qb, Db]) @ v)
        rhs = _fd_check(f, x, v, np.concatenate([Fb, dFb]), 1e-6 * max(1.0, np.abs(x).max()))
        assert abs(lhs - rhs) <= 1e-7 * max(1.0, abs(rhs)), (lhs, rhs)


@pytest.mark.parametrize("p_level", [1.0, 71.4])
def test_compat_vjp_matches_central_differences(p_level):
    rho_ref, p_ref = 1.0, p_level
    for _ in range(10):
        Ql, Qr = states(p_level), states(p_level)
        Q0b = rng.normal(size=5)

        def f(x):
            return devmath.compat(x[:5], x[5:], GAMMA, rho_ref, p_ref)

        x = np.concatenate([Ql, Qr])
        v = rng.normal(size=10)
        Qlb, Qrb = devmath.compat_vjp(Ql, Qr, GAMMA, rho_ref, p_ref, Q0b)
        lhs = float(np.concatenate([Qlb, Qrb]) @ v)
        rhs = _fd_check(f, x, v, Q0b, 1e-6 * max(1.0, np.abs(x).max()))
        assert abs(lhs - rhs) <= 1e-7 * max(1.0, abs(rhs)), (lhs, rhs)


def test_device_weno_z_matches_oracle(oracle_mod):
    """WENO-Z value/slope and both edge values against the oracle's WENO5 with Z
    weights: smooth, steep and discontinuous lines, exponents 1 and 2."""
    lines = [rng.normal(size=5) for _ in range(30)]
    lines += [np.array([1.0, 1.0, 1.0, 0.0, 0.0]), np.array([0.0, 0.0, 5.0, 5.0, 5.0]),
              1.0 + 1e-4 * np.sin(0.3 * np.arange(5)), np.full(5, 2.5)]
    for v in lines:
        for p in (1, 2):
            val, slope = devmath.weno_z_right(v, 1e-6, p)
            rv, rs = oracle_mod.weno5(v, False, 1e-6, p)
            sc = np.abs(v).max()
            assert abs(val - rv) <= 1e-14 * sc and abs(slope - rs) <= 1e-13 * sc
            ea, eb = devmath.weno_z_edges(v, 1e-6, p)
            assert abs(eb - rv) <= 1e-14 * sc
            assert abs(ea - oracle_mod.weno5(v[::-1].copy(), False, 1e-6, p)[0]) <= 1e-14 * sc


@pytest.mark.parametrize("p_level", [1.0, 2.86, 71.4])
def test_device_full_flux_matches_oracle(oracle_mod, p_level):
    """The full flux (three Maxwellians, time integrals over dt and dt/2, Prandtl
    correction) against the oracle at random states and slopes, dt/tau from
    0.05 to 20."""
    rho_ref, p_ref = 1.0, p_level
    for i in range(24):
        Ql, Qr = states(p_level), states(p_level)
        Q0 = 0.5 * (Ql + Qr)
        Dl, Dr, D0 = rng.normal(size=15), rng.normal(size=15), rng.normal(size=15)
        tau = 1e-3 * (1 + rng.random())
        dt = tau * [0.05, 1.0, 5.0, 20.0][i % 4]
        F, dF = devmath.full_flux(Ql, Dl, Qr, Dr, Q0, D0, tau, dt, GAMMA, 0.72, rho_ref, p_ref)
        F[1] += p_ref
        rF, rdF = oracle_mod.gp_flux_full(Ql, Dl, Qr, Dr, Q0, D0, tau, dt, GAMMA, 0.72)
        assert np.abs(F - rF).max() <= 2e-13 * np.abs(rF).max(), (F, rF)
        # dF is a second difference of the time integrals: both sides round at
        # ~1e-16 |I| / (dt |dF|) relative
        assert np.abs(dF - rdF).max() <= 1e-10 * np.abs(rdF).max(), (dF, rdF)


def test_wenoz_jacobians_match_central_differences():
    """The forward-tangent Jacobians of the WENO-Z edge pair and of the right-edge
    value and slope (used by the mode-Z adjoint) against central differences, on
    smooth, steep and near-discontinuous lines, exponents 1 and 2."""
    lines = [rng.normal(size=5) for _ in range(20)]
    lines += [np.array([1.0, 1.02, 1.1, 0.1, 0.0]), 1.0 + 1e-3 * np.sin(0.7 * np.arange(5) + 0.2)]
    for v in lines:
        for p in (1, 2):
            J = devmath.wze_jac(v, 1e-6, p)
            Jv, Js = devmath.wzr_jac(v, 1e-6, p)
            # the Z weights vary on the scale of the line's own variation (and of eps)
            h = 1e-4 * max(np.ptp(v), 1e-3)
            for i in range(5):
                e = np.zeros(5)
                e[i] = 1.0

                def edges(x):
                    return np.array(devmath.weno_z_edges(x, 1e-6, p))

                def right(x):
                    return np.array(devmath.weno_z_right(x, 1e-6, p))

                for f, col in ((edges, J[:, i]), (right, np.array([Jv[i], Js[i]]))):
                    fd = np.array([_fd_check(f, v, e, w, h) for w in np.eye(2)])
                    assert np.abs(col - fd).max() <= 1e-6 * max(np.abs(fd).max(), 1.0), (v, p, i, col, fd)


def test_wenoz_hand_reverses_match_tangent_jacobians():
    """The hand-written reverses of the WENO-Z edge pair and of the right-edge
    value and slope (the mode-Z adjoint's line transposes) equal the transposed
    forward-tangent Jacobians applied to random cotangents, exponents 1 to 4, on
    smooth, steep, near-discontinuous and exactly symmetric lines (b0 = b2)."""
    lines = [rng.normal(size=5) for _ in range(30)]
    lines += [np.array([1.0, 1.02, 1.1, 0.1, 0.0]), 1.0 + 1e-3 * np.sin(0.7 * np.arange(5) + 0.2),
              np.array([0.3, -0.1, 0.5, -0.1, 0.3])]
    for v in lines:
        for p in (1, 2, 3, 4):
            J = devmath.wze_jac(v, 1e-6, p)
            Jv, Js = devmath.wzr_jac(v, 1e-6, p)
            for _ in range(3):
                ab, bb = rng.normal(size=2)
                got = devmath.wze_vjp(v, 1e-6, p, ab, bb)
                want = J[0] * ab + J[1] * bb
                assert np.abs(got - want).max() <= 1e-12 * max(np.abs(want).max(), 1.0), (v, p, got, want)
                got = devmath.wzr_vjp(v, 1e-6, p, ab, bb)
                want = Jv * ab + Js * bb
                assert np.abs(got - want).max() <= 1e-12 * max(np.abs(want).max(), 1.0), (v, p, got, want)


def _z_inputs(p_level, rho_ref, p_ref):
    """60 mode-Z Gauss-point inputs: deviations of Q0, Q_l, Q_r from the reference
    state, then the three slope sets [3][5]."""
    E_ref = p_ref / (GAMMA - 1)
    ref = np.array([rho_ref, 0.0, 0.0, 0.0, E_ref])
    Ql, Qr = states(p_level), states(p_level)
    Q0 = 0.5 * (Ql + Qr) + 0.01 * p_level * rng.normal(size=5) * np.array([0, 0, 0, 0, 1])
    slopes = rng.normal(size=45) * np.tile(np.array([0.1, 0.3, 0.3, 0.3, p_level]), 9)
    return np.concatenate([Q0 - ref, Ql - ref, Qr - ref, slopes])


def test_zflux_reverse_without_viscosity_is_finite_and_matches_central_differences():
    """With mu = 0 and no artificial term the collision time is exactly zero and
    exp(-dt/tau) underflows to 0; the reverse sweep takes the limit 0 of its tau
    derivative there (tau is constant, so that term carries no cotangent), and
    J^T (Fb, dFb) still matches central differences of the forward flux."""
    rho_ref, p_ref = 1.0, 1.0
    args_base = (GAMMA, 0.72, 0.0, 1.0, 0.0, 0.0, rho_ref, p_ref)
    for i in range(4):
        X = _z_inputs(1.0, rho_ref, p_ref)
        dt = [1e-3, 1e-2][i % 2]
        args = (dt,) + args_base
        Fb, dFb = rng.normal(size=5), rng.normal(size=5)
        Xs = devmath.zflux_vjp(X, *args, Fb, dFb)
        assert np.all(np.isfinite(Xs))

        def f(x):
            F, dF = devmath.zgp_flux(x, *args)
            return np.concatenate([F, dF])

        wb = np.concatenate([Fb, dFb])
        for _ in range(3):
            v = rng.normal(size=60) * np.abs(X).clip(1e-2)
            fd = _fd_check(f, X, v, wb, 1e-5)
            got = float(Xs @ v)
            sc = sum(abs(_fd_check(f, X, v * (np.arange(60) == j), wb, 1e-5)) for j in range(0, 60, 7)) + abs(fd)
            assert abs(got - fd) <= 1e-6 * sc, (i, got, fd, sc)


@pytest.mark.parametrize("p_level,mu_exp", [(1.0, 0.0), (2.86, 0.76), (71.4, 0.0)])
def test_zflux_jacobian_transpose_matches_central_differences(p_level, mu_exp):
    """J^T (Fb, dFb) of the mode-Z Gauss-point flux (full distribution, time
    integrals, collision time with the |p_l - p_r| term, mu(T)) from forward
    tangents against central differences of <Fb, F> + <dFb, dF> along random
    directions, dt/tau from 0.05 to 20."""
    rho_ref, p_ref = 1.0, p_level
    mu, c_art = 1e-3, 1.0
    for i in range(8):
        X = _z_inputs(p_level, rho_ref, p_ref)
        dt = mu / p_level * [0.05, 1.0, 5.0, 20.0][i % 4]
        Fb, dFb = rng.normal(size=5), rng.normal(size=5)
        args = (dt, GAMMA, 0.72, mu, 1.0, mu_exp, c_art, rho_ref, p_ref)
        Xb = devmath.zflux_jt(X, *args, Fb, dFb)
        # the kernel's hand-written reverse sweep gives the same transpose
        Xs = devmath.zflux_vjp(X, *args, Fb, dFb)
        assert np.abs(Xs - Xb).max() <= 1e-12 * np.abs(Xb).max(), np.abs(Xs - Xb).max()

        def f(x):
            F, dF = devmath.zgp_flux(x, *args)
            return np.concatenate([F, dF])

        wb = np.concatenate([Fb, dFb])
        for _ in range(3):
            v = rng.normal(size=60) * np.abs(X).clip(1e-2)
            fd = _fd_check(f, X, v, wb, 1e-5)
            got = float(Xb @ v)
            sc = sum(abs(_fd_check(f, X, v * (np.arange(60) == j), wb, 1e-5)) for j in range(0, 60, 7)) + abs(fd)
            assert abs(got - fd) <= 1e-6 * sc, (i, got, fd, sc)
