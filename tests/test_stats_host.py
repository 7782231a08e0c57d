"""CPU checks of the host post-processing in paper_2005_08736_amd.stats: the
three-point derivative is exact on quadratics at any spacing and second order on
a smooth decay; the total-stress balance of laminar Poiseuille flow, which is
linear and exactly 1 - Y+/Re_tau, has zero residual with the exact u_tau."""
import math

import numpy as np
import pytest

from paper_2005_08736_amd import stats


def test_time_derivative_exact_on_quadratics_nonuniform():
    rng = np.random.default_rng(3)
    t = np.cumsum(rng.uniform(0.5, 1.5, size=9))
    f = 2.0 - 0.7 * t + 0.3 * t * t
    assert np.allclose(stats.derivative(t, f), -0.7 + 0.6 * t, rtol=1e-12, atol=1e-12)


def test_time_derivative_second_order():
    errs = []
    for n in (21, 41):
        t = np.linspace(0.0, 1.0, n) ** 1.2  # nonuniform
        errs.append(np.abs(stats.derivative(t, np.exp(-2 * t)) + 2 * np.exp(-2 * t)).max())
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_time_derivative_rejects_bad_histories():
    with pytest.raises(ValueError):
        stats.derivative([0.0, 1.0], [1.0, 2.0])
    with pytest.raises(ValueError):
        stats.derivative([0.0, 2.0, 1.0], [1.0, 2.0, 3.0])


@pytest.mark.parametrize("stretched", [False, True])
def test_total_stress_of_laminar_poiseuille_is_exact(stretched):
    """U = U_c (1 - y^2) at the row centres, no fluctuations: tau_w = 2 U_c mu,
    dU+/dY+ = -y = 1 - Y+/Re_tau."""
    from paper_2005_08736_amd import cases
    ny, Uc, mu, rho = 24, 1.5, 3e-4, 1.1
    if stretched:
        _, y = cases.channel_y(ny, 2.0)
    else:
        y = -1.0 + (np.arange(ny) + 0.5) * 2.0 / ny
    P = np.zeros((ny, 11))
    P[:, 0] = rho
    P[:, 1] = Uc * (1 - y * y)
    r = stats.total_stress(P, {"mu_ref": mu}, y)
    u_tau = math.sqrt(2 * Uc * mu / rho)
    assert r["u_tau"] == pytest.approx(u_tau, rel=1e-12)
    assert r["Re_tau"] == pytest.approx(rho * u_tau / mu, rel=1e-12)
    assert np.abs(r["residual"]).max() <= 1e-11


def test_total_stress_reynolds_stress_enters_with_its_sign():
    """Adding <u'v'> = -c (1 + y) in the lower half moves the residual by +c/u_tau^2."""
    ny = 16
    y = -1.0 + (np.arange(ny) + 0.5) * 2.0 / ny
    P = np.zeros((ny, 11))
    P[:, 0] = 1.0
    P[:, 1] = 1.5 * (1 - y * y)
    base = stats.total_stress(P, {"mu_ref": 1e-3}, y)
    P[:, 9] = -0.01 * (1 + y)
    r = stats.total_stress(P, {"mu_ref": 1e-3}, y)
    half = y < 0
    assert np.allclose(r["residual"] - base["residual"], 0.01 * (1 + y[half]) / base["u_tau"] ** 2, rtol=1e-12)
