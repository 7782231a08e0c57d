"""HGKS oracle: slow scalar FP64 CPU reference of the scheme (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library
(``paper_2005_08736_amd``) never imports it.

Arrays are numpy float64 in the layout ``[5][nz][ny][nx]`` (x fastest), holding
the conservative variables (rho, rho U, rho V, rho W, rho E) as cell averages.
Parameters are given as a plain dict with the keys of :data:`PARAM_FIELDS`.
"""
import ctypes
import os

import numpy as np

from . import build as _build

PARAM_FIELDS = [
    ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
    ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
    ("bc_y", ctypes.c_int32), ("stretch_b", ctypes.c_double),
    ("gamma", ctypes.c_double), ("prandtl", ctypes.c_double),
    ("mu_ref", ctypes.c_double), ("T_ref", ctypes.c_double), ("mu_exp", ctypes.c_double),
    ("mode", ctypes.c_int32), ("cfl", ctypes.c_double),
    ("c_art", ctypes.c_double), ("weno_eps", ctypes.c_double), ("weno_p", ctypes.c_int32),
    ("T_wall", ctypes.c_double), ("body_force_x", ctypes.c_double),
    ("bulk_momentum", ctypes.c_double),
]


class RefParams(ctypes.Structure):
    _fields_ = PARAM_FIELDS


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        # HGKS_ORACLE_SANITIZED=1 selects the ASan + UBSan build (the sanitizer
        # runtimes must then be preloaded into the process)
        path = _build.build(force=False, sanitize=os.environ.get("HGKS_ORACLE_SANITIZED") == "1")
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(RefParams)
        i32, dbl = ctypes.c_int, ctypes.c_double
        sig = {
            "hgks_ref_set_threads": (i32, [i32]),
            "hgks_ref_cfl_dt": (i32, [P, _D, _D]),
            "hgks_ref_step": (i32, [P, _D, i32, dbl, _D]),
            "hgks_ref_two_stage_linear": (i32, [P, _D, dbl, _D]),
            "hgks_ref_operator": (i32, [P, _D, dbl, _D, _D]),
            "hgks_ref_face_flux": (i32, [P, _D, i32, dbl, _D, _D]),
            "hgks_ref_wall_flux": (i32, [P, _D, dbl, _D, _D]),
            "hgks_ref_diagnostics": (i32, [P, _D, _D]),
            "hgks_ref_ndiag": (i32, []),
            "hgks_ref_dilatation": (i32, [P, _D, _D]),
            "hgks_ref_jvp": (i32, [P, _D, _D, i32, _D, _D, _D]),
            "hgks_ref_count_face_flux": (i32, [P, _D, i32, dbl, _D]),
            "hgks_ref_moments_1d": (i32, [dbl, dbl, _D, _D]),
            "hgks_ref_psimom": (i32, [dbl, dbl, dbl, dbl, dbl, i32, i32, i32, i32, _D, _D]),
            "hgks_ref_microslope": (i32, [_D, dbl, dbl, dbl, dbl, dbl, _D]),
            "hgks_ref_compat": (i32, [_D, _D, dbl, _D]),
            "hgks_ref_gp_flux_smooth": (i32, [_D, _D, dbl, dbl, dbl, _D, _D]),
            "hgks_ref_gp_flux_smooth_ext": (i32, [_D, _D, dbl, dbl, dbl, _D, _D]),
            "hgks_ref_gp_flux_full": (i32, [_D, _D, _D, _D, _D, _D, dbl, dbl, dbl, dbl, _D, _D]),
            "hgks_ref_gp_flux_full_parts": (i32, [_D, _D, _D, _D, _D, _D, dbl, dbl, dbl, dbl, dbl, _D, _D]),
            "hgks_ref_weights": (i32, [_D]),
            "hgks_ref_weno5": (i32, [_D, i32, dbl, i32, _D, _D]),
            "hgks_ref_tangential_line": (i32, [_D, i32, dbl, i32, i32, _D, _D]),
            "hgks_ref_eigenvectors": (i32, [_D, dbl, _D, _D]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_D)


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def make_params(d: dict) -> RefParams:
    p = RefParams()
    for name, _ in PARAM_FIELDS:
        # the constant-bulk-momentum switch is off unless given
        setattr(p, name, d.get(name, 0.0) if name == "bulk_momentum" else d[name])
    return p


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def set_threads(n: int) -> int:
    return lib().hgks_ref_set_threads(int(n))


def cfl_dt(params: dict, q: np.ndarray) -> float:
    q = _arr(q)
    out = np.zeros(1)
    _check(lib().hgks_ref_cfl_dt(ctypes.byref(make_params(params)), _p(q), _p(out)), "cfl_dt")
    return float(out[0])


def step(params: dict, q: np.ndarray, nsteps: int, dt: float = 0.0):
    """Advance a copy of q by nsteps two-stage steps; returns (q_new, dts)."""
    q = _arr(q).copy()
    dts = np.zeros(max(nsteps, 1))
    rc = lib().hgks_ref_step(ctypes.byref(make_params(params)), _p(q), int(nsteps), float(dt), _p(dts))
    _check(rc, "step")
    return q, dts[:nsteps]


def two_stage_linear(params: dict, A: np.ndarray, q: np.ndarray, dt: float):
    """One step of the two-stage time stepping with the operator replaced by the
    linear map L(Q) = A Q per cell (dL/dt = A L): pins the stage formulas."""
    q = np.ascontiguousarray(q, dtype=np.float64).copy()
    A = np.ascontiguousarray(A, dtype=np.float64)
    rc = lib().hgks_ref_two_stage_linear(ctypes.byref(make_params(params)), _p(A), float(dt), _p(q))
    if rc != 0:
        raise RuntimeError(f"hgks_ref_two_stage_linear failed with code {rc}")
    return q

def step_rc(params: dict, q: np.ndarray, nsteps: int, dt: float = 0.0) -> int:
    q = _arr(q).copy()
    dts = np.zeros(max(nsteps, 1))
    return lib().hgks_ref_step(ctypes.byref(make_params(params)), _p(q), int(nsteps), float(dt), _p(dts))


def operator(params: dict, q: np.ndarray, dt: float = 0.0):
    q = _arr(q)
    L = np.zeros_like(q)
    dL = np.zeros_like(q)
    _check(lib().hgks_ref_operator(ctypes.byref(make_params(params)), _p(q), float(dt), _p(L), _p(dL)), "operator")
    return L, dL


def face_flux(params: dict, q: np.ndarray, direction: int, dt: float = 0.0):
    q = _arr(q)
    F = np.zeros_like(q)
    dF = np.zeros_like(q)
    rc = lib().hgks_ref_face_flux(ctypes.byref(make_params(params)), _p(q), int(direction), float(dt), _p(F), _p(dF))
    _check(rc, "face_flux")
    return F, dF


def wall_flux(params: dict, q: np.ndarray, dt: float = 0.0):
    """Fluxes of the wall faces of a channel: (F, dF), each [2][5][nz][nx] with
    entry 0 the bottom wall (y = -1) and entry 1 the top wall (y = +1); global
    frame, area-weighted like face_flux."""
    q = _arr(q)
    nz, nx = q.shape[1], q.shape[3]
    F = np.zeros((2, 5, nz, nx))
    dF = np.zeros((2, 5, nz, nx))
    rc = lib().hgks_ref_wall_flux(ctypes.byref(make_params(params)), _p(q), float(dt), _p(F), _p(dF))
    _check(rc, "wall_flux")
    return F, dF


COUNT_KINDS = ["add", "sub", "mul", "div", "sqrt", "exp", "erfc", "pow"]


def count_face_flux(params: dict, q: np.ndarray, direction: int, dt: float = 0.0) -> dict:
    """Operation counts of the oracle's face fluxes of one direction, per face
    (the algorithm as the oracle writes it, run on a counting scalar)."""
    q = _arr(q)
    out = np.zeros(len(COUNT_KINDS))
    rc = lib().hgks_ref_count_face_flux(ctypes.byref(make_params(params)), _p(q), int(direction), float(dt),
                                        _p(out))
    _check(rc, "count_face_flux")
    nf = params["nx"] * params["ny"] * params["nz"]
    return {k: v / nf for k, v in zip(COUNT_KINDS, out)}


NDIAG = 34
DIAG_NAMES = [
    "mass", "mom_x", "mom_y", "mom_z", "energy", "E_k", "zeta", "eps1", "eps2", "eps3",
    "rho_rms", "u_rms", "Ma_t", "min_rho", "min_p", "K", "eps_s", "eps_d", "p_theta", "rho_mean",
    "dudx2", "dvdy2", "dwdz2", "dudx3", "dvdy3", "dwdz3", "dudx4", "dvdy4", "dwdz4",
    "S_u", "F_u", "c_mean", "volume", "max_speed",
]


def diagnostics(params: dict, q: np.ndarray) -> dict:
    q = _arr(q)
    out = np.zeros(NDIAG)
    _check(lib().hgks_ref_diagnostics(ctypes.byref(make_params(params)), _p(q), _p(out)), "diagnostics")
    return dict(zip(DIAG_NAMES, out.tolist()))


def dilatation(params: dict, q: np.ndarray) -> np.ndarray:
    """theta = div U of every cell, shape [nz][ny][nx] (uniform mesh only)."""
    q = _arr(q)
    th = np.zeros(q.shape[1:])
    _check(lib().hgks_ref_dilatation(ctypes.byref(make_params(params)), _p(q), _p(th)), "dilatation")
    return th


def dilatation_pdf(params: dict, q: np.ndarray, nbins: int, lo: float, hi: float):
    """Histogram of r = theta / theta_rms (Sec. 3.4's normalized dilation), with
    theta_rms the root mean square of theta over the cells and r = 0 where it is
    zero.  Returns (counts, theta_rms, r): counts has nbins + 2 slots, slot 0 for
    r < lo, 1 + floor((r - lo) * (nbins / (hi - lo))) (at most nbins) inside
    [lo, hi), nbins + 1 for r >= hi or r not finite.  Plain numpy, FP64."""
    th = dilatation(params, q).ravel()
    rms = float(np.sqrt(np.mean(th * th)))
    r = th / rms if rms > 0.0 else np.zeros_like(th)
    scale = float(nbins) / (hi - lo)
    slot = np.empty(r.size, dtype=np.int64)
    below = r < lo
    above = ~below & ((r >= hi) | ~np.isfinite(r))
    inside = ~below & ~above
    slot[below] = 0
    slot[above] = nbins + 1
    slot[inside] = 1 + np.minimum(np.floor((r[inside] - lo) * scale).astype(np.int64), nbins - 1)
    counts = np.bincount(slot, minlength=nbins + 2).astype(np.int64)
    return counts, rms, r.reshape(q.shape[1:])


PROFILE_NAMES = ["rho", "U", "V", "W", "p", "T", "uu", "vv", "ww", "uv", "rhoU"]


def plane_profiles(params: dict, q: np.ndarray) -> np.ndarray:
    """Reynolds averages over the x-z plane of each y row (the channel statistics of
    Sec. 3.3): <rho>, <U>, <V>, <W>, <p>, <T>, <u'u'>, <v'v'>, <w'w'>, <u'v'>,
    <rho U> per row, U = (rho U)/rho, p = (gamma - 1)(rho E - rho |U|^2/2),
    T = p/rho, fluctuations about the row means.  Plain numpy, FP64; [ny, 11]."""
    q = _arr(q)
    rho = q[0]
    U, V, W = q[1] / rho, q[2] / rho, q[3] / rho
    p = (params["gamma"] - 1.0) * (q[4] - 0.5 * rho * (U * U + V * V + W * W))
    T = p / rho

    def row_mean(a):
        return a.mean(axis=(0, 2))

    Um, Vm, Wm = row_mean(U), row_mean(V), row_mean(W)
    du = U - Um[None, :, None]
    dv = V - Vm[None, :, None]
    dw = W - Wm[None, :, None]
    cols = [row_mean(rho), Um, Vm, Wm, row_mean(p), row_mean(T), row_mean(du * du), row_mean(dv * dv),
            row_mean(dw * dw), row_mean(du * dv), row_mean(rho * U)]
    return np.stack(cols, axis=1)


def jvp(params: dict, q: np.ndarray, dq: np.ndarray, dts):
    q = _arr(q)
    dq = _arr(dq)
    dts = _arr(dts)
    qo = np.zeros_like(q)
    dqo = np.zeros_like(q)
    rc = lib().hgks_ref_jvp(ctypes.byref(make_params(params)), _p(q), _p(dq), int(dts.size), _p(dts), _p(qo), _p(dqo))
    _check(rc, "jvp")
    return qo, dqo


# ---- unit-level pins -------------------------------------------------------

def moments_1d(U, lam):
    full = np.zeros(7)
    plus = np.zeros(7)
    lib().hgks_ref_moments_1d(float(U), float(lam), _p(full), _p(plus))
    return full, plus


def psimom(U, V, W, lam, K, half, a, b, c, X):
    X = _arr(X, 5)
    out = np.zeros(5)
    _check(lib().hgks_ref_psimom(U, V, W, lam, K, int(half), int(a), int(b), int(c), _p(X), _p(out)), "psimom")
    return out


def microslope(b, U, V, W, lam, K):
    b = _arr(b, 5)
    a = np.zeros(5)
    lib().hgks_ref_microslope(_p(b), U, V, W, lam, K, _p(a))
    return a


def compat(Ql, Qr, gamma):
    Ql, Qr = _arr(Ql, 5), _arr(Qr, 5)
    Q0 = np.zeros(5)
    lib().hgks_ref_compat(_p(Ql), _p(Qr), float(gamma), _p(Q0))
    return Q0


def gp_flux_smooth(Q0, dQ, tau, gamma, prandtl):
    Q0, dQ = _arr(Q0, 5), _arr(dQ, 15)
    F0 = np.zeros(5)
    F1 = np.zeros(5)
    lib().hgks_ref_gp_flux_smooth(_p(Q0), _p(dQ), float(tau), float(gamma), float(prandtl), _p(F0), _p(F1))
    return F0, F1


def gp_flux_smooth_ext(Q0, dQ, tau, gamma, prandtl):
    """The smooth Gauss-point flux in x87 extended precision (error measurement only)."""
    Q0, dQ = _arr(Q0, 5), _arr(dQ, 15)
    F0 = np.zeros(5)
    F1 = np.zeros(5)
    lib().hgks_ref_gp_flux_smooth_ext(_p(Q0), _p(dQ), float(tau), float(gamma), float(prandtl), _p(F0), _p(F1))
    return F0, F1


def gp_flux_full(Ql, dQl, Qr, dQr, Q0, dQ0, tau, dt, gamma, prandtl):
    args = [_arr(Ql, 5), _arr(dQl, 15), _arr(Qr, 5), _arr(dQr, 15), _arr(Q0, 5), _arr(dQ0, 15)]
    F = np.zeros(5)
    dF = np.zeros(5)
    lib().hgks_ref_gp_flux_full(*[_p(a) for a in args], float(tau), float(dt), float(gamma), float(prandtl),
                                _p(F), _p(dF))
    return F, dF


def gp_flux_full_parts(Ql, dQl, Qr, dQr, Q0, dQ0, tau, delta, t, gamma, prandtl):
    args = [_arr(Ql, 5), _arr(dQl, 15), _arr(Qr, 5), _arr(dQr, 15), _arr(Q0, 5), _arr(dQ0, 15)]
    I = np.zeros(5)
    Ft = np.zeros(5)
    lib().hgks_ref_gp_flux_full_parts(*[_p(a) for a in args], float(tau), float(delta), float(t), float(gamma),
                                      float(prandtl), _p(I), _p(Ft))
    return I, Ft


def weights():
    out = np.zeros(25)
    lib().hgks_ref_weights(_p(out))
    return {
        "tan_val": out[0:10].reshape(2, 5),
        "tan_der": out[10:20].reshape(2, 5),
        "dn": out[20:25],
    }


def weno5(v, linear, eps=1e-6, p=2):
    v = _arr(v, 5)
    val = np.zeros(1)
    slope = np.zeros(1)
    lib().hgks_ref_weno5(_p(v), int(bool(linear)), float(eps), int(p), _p(val), _p(slope))
    return float(val[0]), float(slope[0])


def tangential_line(v, weno, gp, eps=1e-6, p=2):
    """One tangential line of five face averages to the Gauss point gp (0: -, 1: +)
    of the middle face: (value, derivative per unit width).  weno False: the
    quartic of mode S; True: WENO-Z edge values and the quadratic of mode Z."""
    v = _arr(v, 5)
    val = np.zeros(1)
    der = np.zeros(1)
    _check(lib().hgks_ref_tangential_line(_p(v), int(bool(weno)), float(eps), int(p), int(gp), _p(val), _p(der)),
           "tangential_line")
    return float(val[0]), float(der[0])


def eigenvectors(Q, gamma):
    """(R, L): right eigenvectors of the normal Euler-flux Jacobian at the
    local-frame state Q (columns for u - c, u, u, u, u + c) and L = R^-1."""
    Q = _arr(Q, 5)
    R = np.zeros((5, 5))
    L = np.zeros((5, 5))
    lib().hgks_ref_eigenvectors(_p(Q), float(gamma), _p(R), _p(L))
    return R, L


__all__ = [n for n in dir() if not n.startswith("_")] + ["_build"]
