"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on the
same seeded inputs.  Floating-point tolerance: 1e-12 relative L2 per step for the
state (1e-13 relative for single face fluxes), the contract of the FP64 path."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2005_08736_amd import cases, hgks

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test started without a ROCm device")
    return torch.device("cuda:0")


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(q):
    return torch.from_numpy(np.ascontiguousarray(q)).to(dev())


def rel_l2_fields(a, b):
    """Per-field relative L2 error; the momentum components are normalised by the
    L2 norm of the momentum vector field (one component of the Taylor-Green
    momentum is identically zero at t = 0)."""
    out = []
    mom = math.sqrt(float(np.sum(b[1:4] ** 2)))
    for k in range(5):
        den = mom if 1 <= k <= 3 else float(np.linalg.norm(b[k]))
        out.append(float(np.linalg.norm(a[k] - b[k])) / max(den, 1e-300))
    return out


def smooth_field(nx, ny, nz, seed=0, amp=0.05, gamma=1.4):
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx * 2 * math.pi
    y = (np.arange(ny) + 0.5) / ny * 2 * math.pi
    z = (np.arange(nz) + 0.5) / nz * 2 * math.pi
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")

    def f():
        a = rng.normal(size=6)
        return a[0] * np.sin(X + a[1]) + a[2] * np.cos(Y + 2 * Z + a[3]) + a[4] * np.sin(2 * X - Y + a[5])

    rho = 1.0 + amp * f()
    U, V, W = 0.3 + amp * f(), -0.2 + amp * f(), 0.1 + amp * f()
    p = 1.0 + amp * f()
    q = np.empty((5, nz, ny, nx))
    q[0] = rho
    q[1], q[2], q[3] = rho * U, rho * V, rho * W
    q[4] = p / (gamma - 1) + 0.5 * rho * (U * U + V * V + W * W)
    return q


def ragged_params(q, **kw):
    nz, ny, nx = q.shape[1:]
    base = dict(nx=nx, ny=ny, nz=nz, lx=2 * math.pi, ly=1.3 * math.pi, lz=0.9 * math.pi,
                mu_ref=3e-3, T_ref=0.8, mu_exp=0.76, prandtl=0.7, gamma=1.4)
    base.update(kw)
    return cases.params(**base)


CASES = {
    "tgv32": lambda: (cases.tgv_params(32), cases.tgv_state(32)),
    "ragged13x9x7": lambda: (lambda q: (ragged_params(q), q))(smooth_field(13, 9, 7, seed=11)),
    "min6": lambda: (lambda q: (ragged_params(q), q))(smooth_field(6, 6, 6, seed=12)),
    # a monatomic gas: no internal degrees of freedom (K = 0)
    "ragged13x9x7_monatomic": lambda: (lambda q: (ragged_params(q, gamma=5.0 / 3.0), q))(
        smooth_field(13, 9, 7, seed=13, gamma=5.0 / 3.0)),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("direction", [0, 1, 2])
def test_face_flux_matches_oracle(case, direction):
    announce(f"face_flux {case} dir={direction}")
    p, q = CASES[case]()
    qd = to_dev(q)
    s = hgks.Solver(p, qd)
    F, dF = s.face_flux(direction)
    torch.cuda.synchronize()
    Fr, dFr = oracle.face_flux(p, q, direction)
    # the oracle returns the area-weighted face flux, the library the face average
    area = face_area(p, direction)
    Fr, dFr = Fr / area, dFr / area
    F, dF = F.cpu().numpy(), dF.cpu().numpy()
    # Rounding of a face flux scales with the largest flux component, not with the
    # component itself: the compatibility state sums two half-space thermal
    # fluxes of size rho sqrt(2p/(pi rho)) that cancel where the normal velocity
    # vanishes (Taylor-Green W = 0), and dF holds gamma p div(U) with div(U) ~ 0.
    # The oracle's own FP64 error on dF at these temperatures is up to ~2e-12 of
    # its scale (test_oracle_rounding_bound_at_low_mach), hence 1e-11 for dF.
    scF, scD = np.abs(Fr).max(), np.abs(dFr).max()
    for k in range(5):
        assert np.abs(F[k] - Fr[k]).max() <= 1e-13 * scF, (k, np.abs(F[k] - Fr[k]).max(), scF)
        assert np.abs(dF[k] - dFr[k]).max() <= 1e-11 * scD, (k, np.abs(dF[k] - dFr[k]).max(), scD)


def face_area(p, direction):
    h = [p["lx"] / p["nx"], p["ly"] / p["ny"], p["lz"] / p["nz"]]
    return h[(direction + 1) % 3] * h[(direction + 2) % 3]


@pytest.mark.parametrize("case", sorted(CASES))
def test_operator_matches_oracle(case):
    announce(f"operator {case}")
    p, q = CASES[case]()
    s = hgks.Solver(p, to_dev(q))
    L, dL = s.operator()
    torch.cuda.synchronize()
    Lr, dLr = oracle.operator(p, q)
    # rounding in L is relative to the face fluxes whose differences form it:
    # scale_k = max_d max|F_k,d| / h_d (per unit area), likewise for dL
    h = [p["lx"] / p["nx"], p["ly"] / p["ny"], p["lz"] / p["nz"]]
    scF, scD = np.zeros(5), np.zeros(5)
    for d in range(3):
        Fr, dFr = oracle.face_flux(p, q, d)
        area = face_area(p, d)
        scF = np.maximum(scF, np.abs(Fr / area).reshape(5, -1).max(axis=1) / h[d])
        scD = np.maximum(scD, np.abs(dFr / area).reshape(5, -1).max(axis=1) / h[d])
    # dL inherits the oracle's FP64 error on dF (up to ~2e-12 of the flux scale at
    # Taylor-Green temperatures), hence the looser bound on the second entry
    for A, Ar, sc, tol in ((L.cpu().numpy(), Lr, scF, 1e-13), (dL.cpu().numpy(), dLr, scD, 1e-11)):
        for k in range(5):
            assert np.abs(A[k] - Ar[k]).max() <= tol * sc[k], (k, np.abs(A[k] - Ar[k]).max(), sc[k])


def test_tgv32_twenty_steps_match_oracle_every_step():
    announce("tgv32 20 steps")
    p = cases.tgv_params(32)
    q = cases.tgv_state(32)
    qd = to_dev(q)
    s = hgks.Solver(p, qd)
    qr = q.copy()
    for n in range(20):
        dts = s.step(1, return_dt=True)
        qr, dtr = oracle.step(p, qr, 1)
        assert abs(dts[0] - dtr[0]) <= 1e-14 * dtr[0], (n, dts[0], dtr[0])
        errs = rel_l2_fields(qd.cpu().numpy(), qr)
        assert max(errs) <= 1e-12, (n, errs)
    # fluctuation-relative error of the energy (its mean is ~1000 times its variation)
    e = qd.cpu().numpy()[4]
    er = qr[4]
    fl = np.linalg.norm(e - er) / np.linalg.norm(er - er.mean())
    assert fl <= 1e-10, fl


def test_ragged_box_steps_match_oracle():
    announce("ragged 13x9x7, 4 steps fixed dt")
    q = smooth_field(13, 9, 7, seed=5)
    p = ragged_params(q)
    qd = to_dev(q)
    s = hgks.Solver(p, qd)
    s.step(4, dt=2e-3)
    qr, _ = oracle.step(p, q, 4, dt=2e-3)
    errs = rel_l2_fields(qd.cpu().numpy(), qr)
    assert max(errs) <= 1e-12, errs


def test_diagnostics_match_oracle():
    announce("diagnostics tgv32 after 3 steps")
    p = cases.tgv_params(32)
    q = cases.tgv_state(32)
    qd = to_dev(q)
    s = hgks.Solver(p, qd)
    s.step(3)
    d = s.diagnostics()
    dr = oracle.diagnostics(p, qd.cpu().numpy())
    for name in hgks.DIAG_NAMES:
        a, b = d[name], dr[name]
        scale = {"mom_x": dr["mass"], "mom_y": dr["mass"], "mom_z": dr["mass"], "eps2": dr["eps1"],
                 "eps3": dr["eps1"], "p_theta": dr["eps1"] * 1e3, "S_u": 1.0, "dudx3": dr["dudx2"],
                 "dvdy3": dr["dvdy2"], "dwdz3": dr["dwdz2"]}.get(name, abs(b))
        assert abs(a - b) <= 1e-12 * max(scale, 1e-300), (name, a, b)
    d2 = s.diagnostics()
    assert d2 == d  # fixed reduction order: bitwise repeatable


def test_uniform_flow_preserved_bitwise():
    announce("uniform flow")
    q = cases.uniform_state(16, 8, 12, rho=1.3, vel=(0.4, -0.7, 0.25), p=0.9)
    p = ragged_params(q)
    qd = to_dev(q)
    hgks.Solver(p, qd).step(3)
    assert np.array_equal(qd.cpu().numpy(), q)


def test_conservation_to_roundoff():
    announce("conservation tgv32 10 steps")
    p = cases.tgv_params(32)
    q = cases.tgv_state(32)
    qd = to_dev(q)
    hgks.Solver(p, qd).step(10)
    q1 = qd.cpu().numpy()
    scale = np.abs(q).reshape(5, -1).sum(axis=1)
    scale[1:4] = np.sqrt(np.sum(q[1:4] ** 2, axis=0)).sum()  # momentum: sum of |rho U|
    drift = np.abs(q1.reshape(5, -1).sum(axis=1) - q.reshape(5, -1).sum(axis=1)) / scale
    assert np.all(drift <= 10 * 1e-14), drift


def test_two_runs_bitwise_identical():
    announce("determinism")
    p = cases.tgv_params(32)
    q = cases.tgv_state(32)
    a, b = to_dev(q), to_dev(q)
    hgks.Solver(p, a).step(5)
    hgks.Solver(p, b).step(5)
    assert torch.equal(a, b)


def test_nonphysical_state_reports_and_keeps_last_good():
    announce("non-physical")
    q = cases.uniform_state(8, 8, 8, rho=1.0, vel=(0.1, 0.0, 0.0), p=1.0)
    q[4, 3, 3, 3] = 0.001  # rho E below the kinetic energy 0.005: p < 0 in one cell
    p = ragged_params(q)
    qd = to_dev(q)
    s = hgks.Solver(p, qd)
    st = s.step_status(2, dt=1e-3)
    assert st == hgks.HGKS_E_NONPHYSICAL
    assert np.array_equal(qd.cpu().numpy(), q)  # untouched
    # a state that becomes non-physical during stepping: huge fixed dt
    q = smooth_field(8, 8, 8, seed=3, amp=0.3)
    p = ragged_params(q)
    qd = to_dev(q)
    s = hgks.Solver(p, qd)
    s.step(1, dt=1e-3)
    good = qd.clone()
    st = s.step_status(5, dt=50.0)
    assert st == hgks.HGKS_E_NONPHYSICAL
    assert s.failed_step() >= 1
    k = s.failed_step() - 1  # steps taken before the failure in this call
    ref = good.cpu().numpy()
    if k > 0:
        ref, _ = oracle.step(p, ref, k, dt=50.0)
    assert max(rel_l2_fields(qd.cpu().numpy(), ref)) <= 1e-12


def _window(q, center, w_lo, w_hi):
    nz, ny, nx = q.shape[1:]
    i, j, k = center
    ii = np.arange(i - w_lo, i + w_hi + 1) % nx
    jj = np.arange(j - w_lo, j + w_hi + 1) % ny
    kk = np.arange(k - w_lo, k + w_hi + 1) % nz
    return np.ascontiguousarray(q[:, kk][:, :, jj][:, :, :, ii])


def test_tgv256_full_size_sampled_step():
    """One CFL step of the 256^3 Taylor-Green box (the benchmarked workload) in
    the same kernels and launch shapes the benchmark times.  The oracle checks
    dt on the whole box and Q^{n+1} at sampled cells, each from a 13^3 window
    that holds the cell's whole two-stage dependence (radius 6)."""
    n = 256
    announce("tgv256 sampled step")
    p = cases.tgv_params(n)
    q = cases.tgv_state(n)
    qd = to_dev(q)
    s = hgks.Solver(p, qd)
    dts = s.step(1, return_dt=True)
    dt_ref = oracle.cfl_dt(p, q)
    assert abs(dts[0] - dt_ref) <= 1e-14 * dt_ref
    assert abs(dts[0] - 8.925e-4) <= 0.5e-3 * 8.925e-4  # Table time_table2 (printed)
    q1 = qd.cpu().numpy()
    rng = np.random.default_rng(256)
    pts = [tuple(rng.integers(0, n, size=3)) for _ in range(12)] + [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 3)]
    h = 2 * math.pi / n
    for c in pts:
        win = _window(q, c, 6, 6)
        pw = cases.tgv_params(13, lx=13 * h, ly=13 * h, lz=13 * h)
        qw, _ = oracle.step(pw, win, 1, dt=dts[0])
        got = q1[:, c[2], c[1], c[0]]
        ref = qw[:, 6, 6, 6]
        assert np.all(np.abs(got - ref) <= 1e-13 * np.maximum(np.abs(ref), 1.0)), (c, got - ref)


def test_tgv_early_decay_converges_up_to_256():
    """E_k of the Taylor-Green vortex over t = 0.1433 at 64^3, 128^3 and 256^3
    (the benchmarked size), steps of dt proportional to h.  The decay beyond the
    viscous law E_k(0) exp(-6 nu t) (each initial mode has |k|^2 = 3) holds the
    scheme's numerical dissipation plus the flow's own nonlinear transfer.  E_k
    is evaluated from cell averages, sum (rho U)^2 / (2 rho), a second-order
    approximation of the field's kinetic energy (E_k(0) itself moves by 2.3e-4
    and 5.6e-5 between the three grids); that error dominates the scheme's own
    high-order error here, so the differences between successive grids must
    shrink at least at second order (measured ratio 4.4).  The 64^3 state
    matches the oracle's."""
    nu, T = 1.0 / 1600.0, 0.1433
    rel = {}
    for n, steps in ((64, 40), (128, 80), (256, 160)):
        announce(f"tgv{n} early decay, {steps} steps")
        p = cases.tgv_params(n)
        q = cases.tgv_state(n)
        qd = to_dev(q)
        s = hgks.Solver(p, qd)
        e0 = s.diagnostics()["E_k"]
        s.step(steps, dt=T / steps)
        e1 = s.diagnostics()["E_k"]
        dS = e0 * (math.exp(-6 * nu * T) - 1)
        rel[n] = (e1 - e0 - dS) / dS
        announce(f"  E_k {e0:.12f} -> {e1:.12f}; excess decay / viscous decay {rel[n]:.6e}")
        if n == 64:
            # the state against the oracle's (E_k itself differs between the two
            # by the order of summation over 2.6e5 cells, ~1e-12)
            qr, _ = oracle.step(p, q, steps, dt=T / steps)
            errs = rel_l2_fields(qd.cpu().numpy(), qr)
            announce(f"  64^3 state vs oracle after {steps} steps: rel L2 {max(errs):.2e}")
            assert max(errs) <= 1e-12, errs
        s.close()
    d1, d2 = rel[64] - rel[128], rel[128] - rel[256]
    announce(f"  successive differences {d1:.3e}, {d2:.3e}, ratio {d1 / d2:.1f}")
    assert d1 > 0 and d2 > 0 and d1 / d2 > 3, rel
