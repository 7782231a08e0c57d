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


def test_constant_bulk_momentum_holds_its_target_every_step():
    """With bulk_momentum = m_b the force of each step (Sec. 3.3) makes the box
    integral of rho U equal m_b |Omega| after the step, whatever the unforced
    update did; a dropped factor 1/2, a wrong sign or the wrong density in the
    force formula leaves a residual of the size of the correction itself.  The
    initial field's total differs from the target by 0.2%."""
    p = cases.channel_params(12, 10, 8, body_force_x=0.0, bulk_momentum=1.0)
    q = cases.channel_state(p)
    vol = p["lx"] * 2.0 * p["lz"]
    target = 1.0 * vol
    m0 = oracle.diagnostics(p, q)["mom_x"]
    assert abs(m0 - target) > 1e-3 * target
    for i in range(3):
        q, _ = oracle.step(p, q, 1)
        m = oracle.diagnostics(p, q)["mom_x"]
        assert abs(m - target) <= 1e-13 * target, (i, m, target)


def test_constant_bulk_momentum_and_a_constant_force_exclude_each_other():
    p = cases.channel_params(8, 8, 8, bulk_momentum=1.0)  # body_force_x = 2.93e-3 by default
    q = cases.channel_state(p)
    try:
        oracle.step(p, q, 1)
    except RuntimeError:
        return
    raise AssertionError("the oracle accepted a constant force together with constant bulk momentum")
