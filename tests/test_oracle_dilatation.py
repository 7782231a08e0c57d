"""CPU pins of the oracle's dilatation theta = div U and of its normalized
histogram (the quantity theta / theta_rms of the isotropic cases, Sec. 3.4).

The sixth-order central difference of Sec. 3.1 maps sin(k x + phi) to
k~ cos(k x + phi) exactly, with the modified wavenumber
k~ = (90 sin(k h) - 18 sin(2 k h) + 2 sin(3 k h)) / (60 h), so a velocity field
built from one sine per axis has a closed-form discrete dilatation.  The density
varies in all three directions, so a missing division by rho fails; the three
axes have different spacings, amplitudes and wavenumbers, so a swapped axis or
spacing fails; a sign error flips theta."""
import math

import numpy as np
import pytest

import oracle
from paper_2005_08736_amd import cases


def ktilde(k, h):
    return (90 * math.sin(k * h) - 18 * math.sin(2 * k * h) + 2 * math.sin(3 * k * h)) / (60 * h)


def sine_box(nx, ny, nz, amps, modes, phases, rho_amp=0.2, p0=3.0):
    """Periodic box of lengths (2, 3, 5): U = A sin(k x + phi_x), V, W likewise in
    y and z, rho = 1 + rho_amp sin(2 pi x/2) cos(2 pi y/3) sin(4 pi z/5), p = p0.
    Returns params, state and the closed-form discrete theta [nz][ny][nx]."""
    L = (2.0, 3.0, 5.0)
    n = (nx, ny, nz)
    p = cases.params(nx=nx, ny=ny, nz=nz, lx=L[0], ly=L[1], lz=L[2], mu_ref=1e-3)
    h = [L[a] / n[a] for a in range(3)]
    xs = [(np.arange(n[a]) + 0.5) * h[a] for a in range(3)]
    k = [2 * math.pi * modes[a] / L[a] for a in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    coords = (X, Y, Z)
    vel = [amps[a] * np.sin(k[a] * coords[a] + phases[a]) for a in range(3)]
    rho = 1.0 + rho_amp * np.sin(2 * math.pi * X / L[0]) * np.cos(2 * math.pi * Y / L[1]) * np.sin(
        4 * math.pi * Z / L[2])
    gamma = p["gamma"]
    q = np.empty((5, nz, ny, nx))
    q[0] = rho
    for a in range(3):
        q[1 + a] = rho * vel[a]
    q[4] = p0 / (gamma - 1) + 0.5 * rho * sum(v * v for v in vel)
    theta = sum(amps[a] * ktilde(k[a], h[a]) * np.cos(k[a] * coords[a] + phases[a]) for a in range(3))
    return p, q, theta


def test_dilatation_closed_form_of_sines():
    p, q, theta = sine_box(18, 12, 10, amps=(0.3, -0.7, 1.1), modes=(1, 2, 1), phases=(0.2, 1.3, -0.4))
    th = oracle.dilatation(p, q)
    scale = np.abs(theta).max()
    assert np.abs(th - theta).max() <= 1e-13 * scale


def test_dilatation_is_sixth_order():
    """Against the exact derivative A k cos(k x): the error falls by 2^6 when h halves."""
    errs = []
    for n in (16, 32):
        p, q, theta = sine_box(n, n, n, amps=(0.4, 0.0, 0.0), modes=(1, 1, 1), phases=(0.3, 0.0, 0.0),
                               rho_amp=0.0)
        x = (np.arange(n) + 0.5) * 2.0 / n
        exact = 0.4 * math.pi * np.cos(math.pi * x + 0.3)
        errs.append(np.abs(oracle.dilatation(p, q)[0, 0] - exact).max())
    assert 2 ** 5.8 < errs[0] / errs[1] < 2 ** 6.2


def test_normalized_dilatation_histogram_counts_by_hand():
    """U = A sin(pi x + 0) on 16 cells per period (one x-mode), V = W = 0: theta /
    theta_rms = sqrt(2) cos(2 pi (i + 1/2) / 16), i.e. +-1.387, +-1.176, +-0.786,
    +-0.276, each twice per row.  On [-2, 2) with 4 bins each bin takes 4 of the 16
    values; on [-1, 1) with 2 bins the 8 with |r| > 1 split between the two outer
    slots."""
    nx, ny, nz = 16, 6, 7
    p, q, theta = sine_box(nx, ny, nz, amps=(0.5, 0.0, 0.0), modes=(1, 1, 1), phases=(0.0, 0.0, 0.0), rho_amp=0.0)
    rows = ny * nz
    counts, rms, r = oracle.dilatation_pdf(p, q, 4, -2.0, 2.0)
    k = math.pi
    assert rms == pytest.approx(0.5 * ktilde(k, 2.0 / nx) / math.sqrt(2), rel=1e-13)
    assert counts.tolist() == [0, 4 * rows, 4 * rows, 4 * rows, 4 * rows, 0]
    counts, _, _ = oracle.dilatation_pdf(p, q, 2, -1.0, 1.0)
    assert counts.tolist() == [4 * rows, 4 * rows, 4 * rows, 4 * rows]
    # shocklet and expansion fractions: none reach -3 or 2
    counts, _, _ = oracle.dilatation_pdf(p, q, 1, -3.0, 2.0)
    assert counts.tolist() == [0, nx * rows, 0]


def test_uniform_flow_has_zero_dilatation():
    p = cases.params(nx=7, ny=6, nz=9, lx=1.0, ly=1.0, lz=1.0)
    q = cases.uniform_state(7, 6, 9)
    counts, rms, r = oracle.dilatation_pdf(p, q, 4, -1.0, 1.0)
    assert rms == 0.0 and np.all(r == 0.0)
    # r = 0 falls in the bin [0, 0.5)
    assert counts.tolist() == [0, 0, 0, 7 * 6 * 9, 0, 0]


def test_dilatation_rms_matches_the_dilatational_dissipation():
    """eps_d = 4/3 <mu theta^2> (constant mu) from the diagnostics."""
    p, q, _ = sine_box(12, 10, 14, amps=(0.3, 0.2, -0.4), modes=(1, 1, 2), phases=(0.1, 0.5, 0.9))
    _, rms, _ = oracle.dilatation_pdf(p, q, 8, -4.0, 4.0)
    d = oracle.diagnostics(p, q)
    assert 0.75 * d["eps_d"] / p["mu_ref"] == pytest.approx(rms ** 2, rel=1e-12)
