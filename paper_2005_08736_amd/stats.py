"""Host post-processing of the device diagnostics: the kinetic-energy dissipation
history of the Taylor-Green case (Sec. 3.1).

The dissipation rate of the resolved kinetic energy is eps(E_k) = -dE_k/dt, taken
from the history of E_k; the physical rate is eps1 + eps2 + eps3 (deviatoric
strain, bulk viscosity, pressure dilatation, from hgks_diagnostics), and the
numerical dissipation of the scheme is their difference,
eps_num = eps(E_k) - (eps1 + eps2 + eps3).  The steps and the diagnostics run on
the device; only the time derivative of the recorded history is formed here."""
from __future__ import annotations

import numpy as np


def time_derivative(t, f) -> np.ndarray:
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
    out["eps_Ek"] = -time_derivative(out["t"], out["E_k"])
    out["eps_num"] = out["eps_Ek"] - (out["eps1"] + out["eps2"] + out["eps3"])
    return out
