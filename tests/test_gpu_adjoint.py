"""GPU tests of the hand-written adjoint (hgks_step_vjp) and of the autograd
wrappers with checkpointing: dot-product tests against the oracle's dual-number
JVP (exact derivative of the same scheme) and central finite differences of the
gradient of the volume-averaged kinetic energy after 100 Taylor-Green steps, in
FP64 and in the FP32-flux form."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2005_08736_amd import autograd as ag
from paper_2005_08736_amd import cases, hgks

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test started without a ROCm device")
    return torch.device("cuda:0")


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


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


def to_dev(q):
    return torch.from_numpy(np.ascontiguousarray(q)).to(dev())


CASES = {
    "ragged12x10x8": lambda: (lambda q: (cases.params(nx=12, ny=10, nz=8, lx=2 * math.pi, ly=1.7 * math.pi,
                                                      lz=1.3 * math.pi, mu_ref=3e-3, prandtl=0.7), q))(
        smooth_field(12, 10, 8, seed=21)),
    "tgv32": lambda: (cases.tgv_params(32), cases.tgv_state(32)),
    # y and z axes of at least 21 cells that are not multiples of the y/z adjoint's
    # 16-face runs: the last run along each is partial (8 and 6 faces), and its
    # directly written cells border cells that take atomic adds
    "ragged14x24x22": lambda: (lambda q: (cases.params(nx=14, ny=24, nz=22, lx=1.1 * math.pi, ly=2 * math.pi,
                                                        lz=1.8 * math.pi, mu_ref=3e-3, prandtl=0.7), q))(
        smooth_field(14, 24, 22, seed=22)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_step_vjp_dot_product_with_oracle_jvp(case):
    """<lambda, J v> (oracle JVP, exact derivative of the same scheme) equals
    <J^T lambda, v> (GPU adjoint) for random lambda, v."""
    announce(f"step vjp dot product {case}")
    p, q = CASES[case]()
    dt = 0.5 * oracle.cfl_dt(p, q)
    rng = np.random.default_rng(3)
    qd = to_dev(q)
    st = ag.Stepper(p, qd)
    for trial in range(3):
        v = rng.normal(size=q.shape) * np.array([1e-2, 1e-2, 1e-2, 1e-2, 1e-1])[:, None, None, None]
        lam = rng.normal(size=q.shape)
        _, jv = oracle.jvp(p, q, v, [dt])
        vjp = st.vjp(qd, dt, to_dev(lam)).cpu().numpy()
        lhs = float(np.sum(lam * jv))
        rhs = float(np.sum(vjp * v))
        scale = math.sqrt(float(np.sum(lam ** 2)) * float(np.sum(jv ** 2)))
        announce(f"  trial {trial}: <lam, Jv> = {lhs:.15e}  <J^T lam, v> = {rhs:.15e}")
        assert abs(lhs - rhs) <= 1e-11 * scale, (lhs, rhs, scale)


@pytest.mark.parametrize("case", sorted(CASES))
def test_fp32_form_step_vjp_against_fp64_and_oracle_jvp(case):
    """The FP32-flux form's step adjoint (forward recompute and reverse in FP32,
    cotangents in FP64) against the FP64 adjoint at the same state, and in the
    dot-product test against the oracle's JVP of the FP64 scheme: the identity part
    of the step Jacobian is exact in both, so the error is measured on the
    operator part, lambda_n - lambda."""
    announce(f"FP32-form step vjp {case}")
    p, q = CASES[case]()
    dt = 0.5 * oracle.cfl_dt(p, q)
    rng = np.random.default_rng(4)
    qd = to_dev(q)
    st64 = ag.Stepper(p, qd)
    p32 = dict(p)
    p32["precision"] = hgks.PREC_F32FLUX
    st32 = ag.Stepper(p32, qd)
    for trial in range(2):
        v = rng.normal(size=q.shape) * np.array([1e-2, 1e-2, 1e-2, 1e-2, 1e-1])[:, None, None, None]
        lam = rng.normal(size=q.shape)
        ld = to_dev(lam)
        d64 = st64.vjp(qd, dt, ld).cpu().numpy() - lam
        d32 = st32.vjp(qd, dt, ld).cpu().numpy() - lam
        rel = float(np.linalg.norm(d32 - d64) / np.linalg.norm(d64))
        _, jv = oracle.jvp(p, q, v, [dt])
        lhs = float(np.sum(lam * (jv - v)))
        rhs = float(np.sum(d32 * v))
        scale = math.sqrt(float(np.sum(lam ** 2)) * float(np.sum((jv - v) ** 2)))
        announce(f"  trial {trial}: rel L2 of the operator part vs FP64 {rel:.2e}; "
                 f"dot product {lhs:.10e} vs {rhs:.10e} (rel to scale {abs(lhs - rhs) / scale:.2e})")
        assert rel <= 1e-5, rel
        assert abs(lhs - rhs) <= 1e-6 * scale, (lhs, rhs, scale)


def kinetic_energy(q):
    """E_k = (1/(rho0 |Omega|)) int rho |U|^2 / 2 (Sec. 3.1) on a uniform box, rho0 = 1."""
    return 0.5 * torch.sum((q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]) / q[0].numel()


def test_checkpointed_gradient_matches_oracle_jvp():
    """Gradient of E_k after 10 Taylor-Green steps at 32^3 (checkpoint every 4)
    along random directions, against the oracle's JVP with the same frozen dts."""
    n, steps = 32, 10
    announce(f"checkpointed gradient tgv{n}, {steps} steps")
    p = cases.tgv_params(n)
    q = cases.tgv_state(n)
    qd = to_dev(q)
    dts = ag.cfl_time_steps(p, qd, steps)
    st = ag.Stepper(p, qd)
    q0 = qd.clone().requires_grad_(True)
    J = kinetic_energy(ag.run_checkpointed(st, q0, dts, every=4))
    J.backward()
    g = q0.grad.cpu().numpy()
    rng = np.random.default_rng(5)
    for trial in range(2):
        v = rng.normal(size=q.shape) * 1e-2
        qf, jv = oracle.jvp(p, q, v, dts)
        m2 = qf[1] ** 2 + qf[2] ** 2 + qf[3] ** 2
        dJdq = np.zeros_like(qf)
        N = qf[0].size
        dJdq[0] = -0.5 * m2 / qf[0] ** 2 / N
        dJdq[1:4] = qf[1:4] / qf[0] / N
        ref = float(np.sum(dJdq * jv))
        got = float(np.sum(g * v))
        announce(f"  trial {trial}: adjoint {got:.15e}  oracle JVP {ref:.15e}")
        assert abs(got - ref) <= 1e-9 * abs(ref), (got, ref)


_TGV128 = {}


def _tgv128_problem():
    """Adjoint benchmark set-up: 128^3 Taylor-Green plus a seeded 1% solenoidal
    velocity perturbation, 100 CFL steps of the FP64 run frozen as the dts."""
    if "p" not in _TGV128:
        n, steps = 128, 100
        p = cases.tgv_params(n)
        q = cases.tgv_state(n)
        pert = cases.solenoidal_perturbation(n, seed=0, kmax=4.0, rms=0.01)
        gamma = p["gamma"]
        _TGV128.update(p=p, gamma=gamma, rho=to_dev(q[0]), U0=to_dev(q[1:4] / q[0] + pert),
                       pr=to_dev((gamma - 1) * (q[4] - 0.5 * np.sum(q[1:4] ** 2, axis=0) / q[0])))
        _TGV128["dts"] = ag.cfl_time_steps(p, _tgv128_state(_TGV128["U0"]), steps)
        dirs = []
        for seed in range(1, 9):
            d = to_dev(cases.solenoidal_perturbation(n, seed=seed, kmax=4.0, rms=1.0))
            dirs.append(d / torch.sqrt(torch.sum(d * d)))
        _TGV128["dirs"] = dirs
    return _TGV128


def _tgv128_state(U):
    """Conservative state from the velocity field U, rho and p of the set-up held."""
    t = _TGV128
    rho, gamma = t["rho"], t["gamma"]
    s = torch.empty((5,) + tuple(rho.shape), dtype=torch.float64, device=dev())
    s[0] = rho
    s[1:4] = rho * U
    s[4] = t["pr"] / (gamma - 1) + 0.5 * rho * torch.sum(U * U, dim=0)
    return s


def _tgv128_gradient(precision):
    """dE_k(step 100)/dU0 through the checkpointed adjoint (every 10 steps)."""
    key = ("grad", precision)
    if key not in _TGV128:
        t = _tgv128_problem()
        p = dict(t["p"])
        p["precision"] = precision
        st = ag.Stepper(p, _tgv128_state(t["U0"]))
        U = t["U0"].clone().requires_grad_(True)
        J = kinetic_energy(ag.run_checkpointed(st, _tgv128_state(U), t["dts"], every=10))
        J.backward()
        _TGV128[key] = (st, U.grad.detach(), J.item())
    return _TGV128[key]


def _tgv128_central_difference(st, d):
    """Richardson-extrapolated central difference of E_k(step 100) along d."""
    t = _TGV128

    def J_of(Uv):
        with torch.no_grad():
            x = _tgv128_state(Uv)
            for dt in t["dts"]:
                x = st.step(x, dt)
            return kinetic_energy(x).item()

    def cd(hh):
        return (J_of(t["U0"] + hh * d) - J_of(t["U0"] - hh * d)) / (2 * hh)

    h = 2.0
    return (4 * cd(h / 2) - cd(h)) / 3


def test_tgv128_gradient_matches_central_differences():
    """Config of the adjoint benchmark: gradient of E_k at step 100 of a 128^3
    Taylor-Green run (plus a seeded 1% solenoidal perturbation) with respect to
    the initial velocity field, rho and p held, dts frozen, checkpoint every 10;
    checked against central differences along 8 seeded solenoidal directions."""
    announce("tgv128 gradient vs central differences, 100 steps")
    t = _tgv128_problem()
    st, g, J = _tgv128_gradient(hgks.PREC_F64)
    announce(f"  J = {J:.12f}")
    worst = 0.0
    fds = []
    for i, d in enumerate(t["dirs"]):
        gd = float(torch.sum(g * d))
        fd = _tgv128_central_difference(st, d)
        fds.append(fd)
        rel = abs(gd - fd) / abs(fd)
        worst = max(worst, rel)
        announce(f"  direction {i + 1}: adjoint {gd:.10e}  central difference {fd:.10e}  rel {rel:.2e}")
    _TGV128["fd64"] = fds
    assert worst <= 1e-6, worst


def test_tgv128_fp32_form_gradient():
    """The same gradient through the FP32-flux form (forward and adjoint fluxes in
    FP32, state and cotangents in FP64), against the FP64 adjoint gradient, the
    FP64 scheme's central differences and the FP32 form's own central
    differences along the same 8 directions."""
    announce("tgv128 FP32-form gradient, 100 steps")
    t = _tgv128_problem()
    st64, g64, _ = _tgv128_gradient(hgks.PREC_F64)
    st32, g32, J32 = _tgv128_gradient(hgks.PREC_F32FLUX)
    rel_g = float(torch.linalg.vector_norm(g32 - g64) / torch.linalg.vector_norm(g64))
    announce(f"  J = {J32:.12f}; rel L2 of the gradient vs FP64 {rel_g:.2e}")
    fd64 = _TGV128.get("fd64")
    if fd64 is None:
        fd64 = [_tgv128_central_difference(st64, d) for d in t["dirs"]]
    w64 = w32 = 0.0
    for i, d in enumerate(t["dirs"]):
        gd = float(torch.sum(g32 * d))
        fd32 = _tgv128_central_difference(st32, d)
        r64, r32 = abs(gd - fd64[i]) / abs(fd64[i]), abs(gd - fd32) / abs(fd32)
        w64, w32 = max(w64, r64), max(w32, r32)
        announce(f"  direction {i + 1}: FP32 adjoint {gd:.10e}  FP64 central difference {fd64[i]:.10e} "
                 f"(rel {r64:.2e})  FP32-form central difference {fd32:.10e} (rel {r32:.2e})")
    assert rel_g <= 1e-4, rel_g
    assert w64 <= 1e-5, w64
    assert w32 <= 1e-4, w32
