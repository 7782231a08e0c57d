"""Pins of the isotropic-turbulence initial field (Sec. 3.4, Eq. (initial
spectrum) and the parameter chain that follows it): the generator in
``cases`` holds inputs only, but every mode-Z workload starts from it, so its
properties are checked here against what the set-up fixes:

* solenoidal: k . u_hat(k) = 0 for every Fourier mode (spectral divergence);
* spectrum shape: the energy of each integer shell of wavenumbers follows
  E(k) = A0 k^4 exp(-2 k^2 / k0^2) spread isotropically over the lattice modes
  of the shell (density E(|k|) / (4 pi |k|^2) per unit k-volume), times the
  squared transfer function prod_d sinc(k_d h / 2) of a cell average, within
  the sampling error of the random phases;
* zero mean velocity; u_rms = sqrt(2 K0 / 3) and Ma_t exact after rescaling;
  uniform density and temperature.
"""
import math

import numpy as np
import pytest

from paper_2005_08736_amd import cases


def _spectrum(k):
    return cases.ISO_A0 * k ** 4 * np.exp(-2 * k ** 2 / cases.ISO_K0 ** 2)


def _wavenumbers(n):
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")  # arrays are [z][y][x]
    return kx, ky, kz


@pytest.mark.parametrize("seed", [0, 1])
def test_generated_field_is_solenoidal(seed):
    n = 32
    u = cases.solenoidal_field(n, seed, _spectrum)
    uh = np.fft.fftn(u, axes=(1, 2, 3))
    kx, ky, kz = _wavenumbers(n)
    div = kx * uh[0] + ky * uh[1] + kz * uh[2]
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    mag = np.sqrt(np.sum(np.abs(uh) ** 2, axis=0))
    assert np.abs(div).max() <= 1e-14 * (kk * mag).max()
    assert np.abs(uh[:, 0, 0, 0]).max() <= 1e-12 * mag.max()  # no mean flow


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_generated_shell_spectrum_follows_the_model(seed):
    n = 32
    h = 2 * math.pi / n
    u = cases.solenoidal_field(n, seed, _spectrum)
    uh = np.fft.fftn(u, axes=(1, 2, 3)) / n ** 3
    energy = 0.5 * np.sum(np.abs(uh) ** 2, axis=0)
    kx, ky, kz = _wavenumbers(n)
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    cell = (np.sinc(kx * h / (2 * math.pi)) * np.sinc(ky * h / (2 * math.pi)) *
            np.sinc(kz * h / (2 * math.pi))) ** 2
    safe = np.maximum(kk, 1e-30)
    model = np.where((kk > 0) & (kk <= n / 2), _spectrum(safe) / (4 * math.pi * safe ** 2) * cell, 0.0)
    shell = np.rint(kk).astype(int).ravel()
    got = np.bincount(shell, energy.ravel())[1:n // 2]
    want = np.bincount(shell, model.ravel())[1:n // 2]
    count = np.bincount(shell)[1:n // 2]
    ratio = got / want
    ratio /= np.sum(got) / np.sum(want)  # overall level: set by the rescaling to u_rms
    # each mode pair (k, -k) carries a random share of its energy (the real part of
    # a field with independent phases at k and -k): relative sampling error of a
    # shell ~ 1 / sqrt(modes in the shell)
    sigma = 1.0 / np.sqrt(count)
    z = (ratio - 1.0) / sigma
    assert np.all(np.abs(z) <= 5.0), np.round(z, 2)
    assert math.sqrt(np.mean(z[3:] ** 2)) <= 2.0, np.round(z, 2)
    # the high shells see the cell average: without it they would be 2x higher
    assert want[-1] / np.bincount(shell, np.where(model > 0, model / cell, 0.0).ravel())[n // 2 - 1] < 0.6


@pytest.mark.parametrize("ma_t", [0.5, 1.0])
def test_isotropic_state_rms_mach_and_uniform_thermodynamics(ma_t):
    n = 32
    c = cases.isotropic_constants()
    q = cases.isotropic_state(n, 0, ma_t)
    p = cases.isotropic_params(n, ma_t)
    rho = q[0]
    U = q[1:4] / rho
    urms = math.sqrt(np.mean(np.sum(U ** 2, axis=0)) / 3.0)
    assert np.all(rho == 1.0)
    assert abs(urms - math.sqrt(2 * c["K0"] / 3)) <= 1e-14
    assert np.abs(U.reshape(3, -1).mean(axis=1)).max() <= 1e-15
    pres = (p["gamma"] - 1) * (q[4] - 0.5 * rho * np.sum(U ** 2, axis=0))
    assert np.abs(pres / pres.mean() - 1).max() <= 1e-13
    cs = math.sqrt(p["gamma"] * pres.mean() / 1.0)
    assert abs(math.sqrt(3) * urms / cs - ma_t) <= 1e-13
    # the temperature is the viscosity law's reference temperature
    assert abs(pres.mean() - p["T_ref"]) <= 1e-13 * p["T_ref"]
