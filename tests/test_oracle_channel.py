"""Pins of the oracle's channel set-up (Sec. 3.3): isothermal no-slip walls in
y by mirror ghosts, the tanh wall-normal mesh and the constant body force."""
import numpy as np

import oracle
from paper_2005_08736_amd import cases


def test_channel_rest_state_at_wall_temperature_is_steady_bitwise():
    """Fluid at rest at the wall temperature: the ghosts equal the interior, every
    face carries the same pressure flux, and the state cannot change."""
    p = cases.channel_params(8, 16, 6, body_force_x=0.0)
    q = cases.uniform_state(8, 16, 6, rho=1.0, vel=(0.0, 0.0, 0.0), p=p["T_wall"])
    q1, _ = oracle.step(p, q, 3)
    assert np.array_equal(q1, q)


def test_channel_mirror_symmetry_is_kept():
    """The mesh and the wall closure are symmetric about y = 0: a state even in y
    (V odd) stays so to round-off under the forced step."""
    p = cases.channel_params(8, 16, 6)
    q = cases.channel_state(p, seed=1, noise=0.1)
    m = q[:, :, ::-1, :].copy()
    m[2] *= -1
    q = 0.5 * (q + m)
    q1, _ = oracle.step(p, q, 3)
    m1 = q1[:, :, ::-1, :].copy()
    m1[2] *= -1
    for k in (0, 1, 4):
        assert np.abs(q1[k] - m1[k]).max() <= 1e-14 * np.abs(q1[k]).max(), k
    for k in (2, 3):  # small transverse momenta: measured against the streamwise one
        assert np.abs(q1[k] - m1[k]).max() <= 1e-14 * np.abs(q1[1]).max(), k


def test_channel_poiseuille_balance_converges_in_the_interior():
    """Laminar Poiseuille flow U = 1.5 (1 - y^2) with f_x = 3 mu / rho balances the
    viscous stress: the x-momentum tendency L_mx + rho f_x of the operator tends
    to zero with refinement away from the walls.  The reconstruction works in
    eta on cell averages taken in y, so the order is two; the wall rows carry the
    mirror-ghost closure's own O(1) error in the wall shear (not converging)."""
    errs = []
    for ny in (32, 64, 128):
        mu = 1e-2
        p = cases.channel_params(6, ny, 6, mu_ref=mu, body_force_x=3.0 * mu)
        q = cases.channel_state(p, seed=0, noise=0.0)
        L, _ = oracle.operator(p, q)
        e = (L[1] + q[0] * p["body_force_x"])[0, :, 0]
        k = ny // 8  # the same physical distance from the walls at every ny
        errs.append(float(np.abs(e[k:-k]).max()))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.5, errs
    assert errs[2] < 0.01 * 3.0 * 1e-2, errs  # below 1% of the force at ny = 128
