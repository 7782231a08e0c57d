"""GPU check of the dissipation history (Sec. 3.1: eps(E_k) = -dE_k/dt and the
numerical dissipation eps_num = eps(E_k) - (eps1 + eps2 + eps3)) on the
Taylor-Green vortex at 32^3, 20 CFL steps sampled every 2: the device steps and
diagnostics through paper_2005_08736_amd.stats against the oracle's steps and
diagnostics differentiated with numpy.gradient (second order at nonuniform
times, the same three-point derivative)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2005_08736_amd import cases, hgks, stats

pytestmark = pytest.mark.gpu


def test_taylor_green_dissipation_history_matches_oracle():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test started without a ROCm device")
    n, nsteps, every = 32, 20, 2
    p = cases.tgv_params(n)
    q0 = cases.tgv_state(n)
    print(f"[gpu-case] Taylor-Green {n}^3 dissipation history, {nsteps} steps every {every}", flush=True)
    s = hgks.Solver(p, torch.from_numpy(q0).to("cuda:0"))
    h = stats.dissipation_history(s, nsteps, every)
    s.close()
    q, t = q0.copy(), 0.0
    rows = []
    d = oracle.diagnostics(p, q)
    rows.append((t, d["E_k"], d["eps1"], d["eps2"], d["eps3"]))
    for _ in range(nsteps // every):
        q, dts = oracle.step(p, q, every)
        t += float(np.sum(dts))
        d = oracle.diagnostics(p, q)
        rows.append((t, d["E_k"], d["eps1"], d["eps2"], d["eps3"]))
    a = np.array(rows)
    eps_ek = -np.gradient(a[:, 1], a[:, 0], edge_order=2)
    eps_num = eps_ek - (a[:, 2] + a[:, 3] + a[:, 4])
    assert np.allclose(h["t"], a[:, 0], rtol=1e-13, atol=0)
    assert np.allclose(h["E_k"], a[:, 1], rtol=1e-12, atol=0)
    for k, name in ((2, "eps1"), (3, "eps2"), (4, "eps3")):
        assert np.abs(h[name] - a[:, k]).max() <= 1e-10 * np.abs(a[:, k]).max(), name
    # the three-point weights sum to at most 4 / min spacing in absolute value, so
    # the E_k tolerance (1e-12 relative) bounds the derivative's difference; the
    # eps terms add their own
    bound_ek = 4.0 / np.diff(a[:, 0]).min() * 1e-12 * np.abs(a[:, 1]).max()
    bound_num = bound_ek + 3e-10 * np.abs(a[:, 2:5]).max()
    err_ek = np.abs(h["eps_Ek"] - eps_ek).max()
    err_num = np.abs(h["eps_num"] - eps_num).max()
    print(f"[gpu-case]   eps(E_k) {h['eps_Ek'][-1]:.6e}, eps_num {h['eps_num'][-1]:.6e} at t = {h['t'][-1]:.4f}; "
          f"differences from the oracle {err_ek:.1e} (bound {bound_ek:.1e}), {err_num:.1e} (bound {bound_num:.1e})",
          flush=True)
    sys.stdout.flush()
    assert err_ek <= bound_ek and err_num <= bound_num
