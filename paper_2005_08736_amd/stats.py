"""Host post-processing of the device diagnostics: the kinetic-energy dissipation
history of the Taylor-Green case (Sec. 3.1) and the total-stress balance of the
channel (Sec. 3.3).

The dissipation rate of the resolved kinetic energy is eps(E_k) = -dE_k/dt, taken
from the history of E_k; the physical rate is eps1 + eps2 + eps3 (deviatoric
strain, bulk viscosity, pressure dilatation, from hgks_diagnostics), and the
numerical dissipation of the scheme is their difference,
eps_num = eps(E_k) - (eps1 + eps2 + eps3).  The steps and the diagnostics run on
the device; only the time derivative of the recorded history is formed here."""
from __future__ import annotations

import numpy as np


def derivative(t, f) -> np.ndarray:
    """df/dt at every sample of a history on nonuniform times: the derivative of the
    quadratic through three neighbouring samples (second order), centred inside
    and taken over the first or last three samples at the ends."""
    t = np.asarray(t, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    n = t.size
    if n < 3 or f.shape != t.shape:
        raise ValueError("need at least three samples of matching shape")
    if not np.all(np.diff(t) > 0):
        raise ValueError("times must increase")
    d = np.empty(n)
    for i in range(n):
        j = min(max(i - 1, 0), n - 3)
        t0, t1, t2 = t[j], t[j + 1], t[j + 2]
        x = t[i]
        d[i] = (f[j] * (2 * x - t1 - t2) / ((t0 - t1) * (t0 - t2))
                + f[j + 1] * (2 * x - t0 - t2) / ((t1 - t0) * (t1 - t2))
                + f[j + 2] * (2 * x - t0 - t1) / ((t2 - t0) * (t2 - t1)))
    return d


def dissipation_history(solver, nsteps: int, every: int = 1) -> dict:
    """Advance `solver` (an hgks.Solver) by nsteps CFL steps, recording t, E_k and
    eps1..eps3 at the start and after every `every` steps.  Returns arrays t, E_k,
    eps1, eps2, eps3, eps_Ek = -dE_k/dt and eps_num = eps_Ek - (eps1 + eps2 + eps3)."""
    if nsteps < 2 * every or every < 1:
        raise ValueError("need at least three samples")
    rows = []
    t = 0.0

    def record():
        d = solver.diagnostics()
        rows.append((t, d["E_k"], d["eps1"], d["eps2"], d["eps3"]))

    record()
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        t += float(sum(solver.step(k, return_dt=True)))
        done += k
        record()
    a = np.array(rows)
    out = {name: a[:, i] for i, name in enumerate(("t", "E_k", "eps1", "eps2", "eps3"))}
    out["eps_Ek"] = -derivative(out["t"], out["E_k"])
    out["eps_num"] = out["eps_Ek"] - (out["eps1"] + out["eps2"] + out["eps3"])
    return out


def total_stress(profiles: np.ndarray, params: dict, y_centres) -> dict:
    """Total-stress balance of the channel (Sec. 3.3) in wall units from the plane
    profiles of hgks_plane_profiles (rows from the bottom wall y = -1 to the top
    wall y = 1; y_centres the rows' centres; constant viscosity mu_ref).

    The wall shear stress is mu dU/dy at each wall from the quadratic through the
    wall (U = 0) and the two nearest rows, averaged over the two walls; with rho_w
    the mean density of the two wall rows, u_tau = sqrt(tau_w / rho_w) and
    Re_tau = rho_w u_tau / mu (half-width 1).  Per row of the lower half:
    Y+ = (1 + y) Re_tau, dU+/dY+ = mu/(rho_w u_tau^2) dU/dy (three-point derivative
    over the rows), <uv>+ = <u'v'> / u_tau^2, and the residual
    dU+/dY+ - <uv>+ - (1 - Y+/Re_tau) of the balance, which vanishes for a
    statistically stationary flow."""
    y = np.asarray(y_centres, dtype=np.float64)
    P = np.asarray(profiles, dtype=np.float64)
    ny = y.size
    if P.shape[0] != ny or ny < 4:
        raise ValueError("one profile row per y row, at least four rows")
    mu = float(params["mu_ref"])
    U, uv, rho = P[:, 1], P[:, 9], P[:, 0]

    def wall_slope(yw, y0, y1, u0, u1):
        # derivative at yw of the quadratic through (yw, 0), (y0, u0), (y1, u1)
        return (u0 * (yw - y1) / ((y0 - yw) * (y0 - y1)) + u1 * (yw - y0) / ((y1 - yw) * (y1 - y0)))

    tau_b = mu * wall_slope(-1.0, y[0], y[1], U[0], U[1])
    tau_t = -mu * wall_slope(1.0, y[-1], y[-2], U[-1], U[-2])
    tau_w = 0.5 * (tau_b + tau_t)
    rho_w = 0.5 * (rho[0] + rho[-1])
    u_tau = np.sqrt(tau_w / rho_w)
    re_tau = rho_w * u_tau / mu
    dudy = derivative(y, U)
    half = y < 0.0
    Yp = (1.0 + y[half]) * re_tau
    dUp = mu / (rho_w * u_tau ** 2) * dudy[half]
    uvp = uv[half] / u_tau ** 2
    return {"u_tau": float(u_tau), "Re_tau": float(re_tau), "Y_plus": Yp, "dU_plus": dUp, "uv_plus": uvp,
            "residual": dUp - uvp - (1.0 - Yp / re_tau)}
