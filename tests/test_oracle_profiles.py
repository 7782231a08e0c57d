"""CPU pins of the oracle's plane-averaged profiles (the channel statistics of
Sec. 3.3: mean velocity, velocity fluctuations, Reynolds stress per y row).

The fields are built so that every plane average has a closed form: on n >= 3
equally spaced points of a full period, cos and sin average to zero, cos^2 to
1/2 and cos sin to zero.  Each column gets a different y-dependence and the
fluctuating parts differ per component, so a swapped column, a missing division
by rho, a wrong sign of the stress or a missing centring fails."""
import math

import numpy as np

import oracle
from paper_2005_08736_amd import cases


def field(nx, ny, nz, gamma=1.4):
    """rho = r(y) (x-z constant), U = f(y) + a(y) cos(kx x), V = b(y) cos(kx x) +
    c(y) sin(kz z), W = e(y) sin(kx x), p = p(y)."""
    p = cases.channel_params(nx, ny, nz, stretch_b=0.0, ly=2.0, gamma=gamma)
    y = -1.0 + (np.arange(ny) + 0.5) * 2.0 / ny
    x = (np.arange(nx) + 0.5) * p["lx"] / nx
    z = (np.arange(nz) + 0.5) * p["lz"] / nz
    cx = np.cos(2 * math.pi * x / p["lx"])[None, None, :]
    sx = np.sin(2 * math.pi * x / p["lx"])[None, None, :]
    sz = np.sin(2 * math.pi * z / p["lz"])[:, None, None]
    r = (1.0 + 0.1 * y)[None, :, None]
    f, a = (1.5 * (1 - y * y))[None, :, None], (0.2 + 0.1 * y)[None, :, None]
    b, c, e = (0.3 * y)[None, :, None], (0.05 + 0.0 * y)[None, :, None], (0.1 - 0.05 * y)[None, :, None]
    pr = (50.0 + y)[None, :, None]
    U = f + a * cx
    V = b * cx + c * sz
    W = e * sx
    q = np.empty((5, nz, ny, nx))
    q[0] = r * np.ones((nz, 1, nx))
    q[1], q[2], q[3] = q[0] * U, q[0] * V, q[0] * W
    q[4] = pr / (gamma - 1) + 0.5 * q[0] * (U * U + V * V + W * W)
    sq = lambda v: v[0, :, 0]
    expect = np.stack([
        sq(r), sq(f), 0 * y, 0 * y, sq(pr), sq(pr / r),
        sq(a) ** 2 / 2, sq(b) ** 2 / 2 + sq(c) ** 2 / 2, sq(e) ** 2 / 2, sq(a) * sq(b) / 2, sq(r) * sq(f),
    ], axis=1)
    return p, q, expect


def test_plane_profiles_closed_form():
    p, q, expect = field(12, 9, 8)
    got = oracle.plane_profiles(p, q)
    # zero-mean columns (<V>, <W>) on the velocity scale 1
    scale = np.maximum(np.abs(expect).max(axis=0), 1.0)
    assert np.all(np.abs(got - expect) <= 1e-13 * scale[None, :]), np.abs(got - expect).max(axis=0) / scale


def test_plane_profiles_bulk_momentum_matches_the_total():
    """sum_j <rho U>_j nx nz dx dz dy_j = the total x-momentum of the diagnostics,
    here on the stretched channel mesh with its seeded initial field."""
    p = cases.channel_params(16, 12, 8)
    q = cases.channel_state(p)
    prof = oracle.plane_profiles(p, q)
    yf, _ = cases.channel_y(p["ny"])
    dx, dz = p["lx"] / p["nx"], p["lz"] / p["nz"]
    total = float(np.sum(prof[:, 10] * np.diff(yf))) * p["nx"] * p["nz"] * dx * dz
    assert abs(total - oracle.diagnostics(p, q)["mom_x"]) <= 1e-13 * abs(total)


def test_plane_profiles_uniform_state():
    p = cases.params(nx=6, ny=7, nz=6, lx=1.0, ly=1.0, lz=1.0)
    q = cases.uniform_state(6, 7, 6, rho=1.3, vel=(0.3, -0.2, 0.1), p=2.0)
    got = oracle.plane_profiles(p, q)
    want = [1.3, 0.3, -0.2, 0.1, 2.0, 2.0 / 1.3, 0.0, 0.0, 0.0, 0.0, 1.3 * 0.3]
    assert np.allclose(got, np.array(want)[None, :], rtol=1e-14, atol=1e-15)
