"""Builds and loads tests/cpp/devmath.hip: the library's scalar device math
compiled for the host, for CPU checks of the forward and adjoint formulas."""
import ctypes
import fcntl
import glob
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpp", "devmath.hip")
LIB = os.path.join(HERE, "cpp", "libdevmath.so")
# every library header: the device math includes several of them, directly or not
HDRS = sorted(glob.glob(os.path.join(HERE, "..", "paper_2005_08736_amd", "csrc", "*.hpp")))
_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        # several test processes (pytest -n) may find the library stale at once:
        # one builds it under the lock, the others wait and load the result
        with open(LIB + ".lock", "w") as lock:
            fcntl.flock(lock, fcntl.LOCK_EX)
            newest = max(os.path.getmtime(p) for p in [SRC] + HDRS)
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
                tmp = f"{LIB}.{os.getpid()}.tmp"
                subprocess.run(["hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                                "-o", tmp, SRC], check=True)
                os.replace(tmp, LIB)
            _lib = ctypes.CDLL(LIB)
    return _lib


def _a(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    assert a.size == n
    return a


def _p(a):
    return a.ctypes.data_as(_D)


def smooth_flux(Q, D, gamma, prandtl, mu, rho_ref, p_ref):
    Q, D = _a(Q, 5), _a(D, 15)
    F, dF = np.zeros(5), np.zeros(5)
    lib().dm_smooth_flux(_p(Q), _p(D), ctypes.c_double(gamma), ctypes.c_double(prandtl), ctypes.c_double(mu),
                         ctypes.c_double(rho_ref), ctypes.c_double(p_ref), _p(F), _p(dF))
    return F, dF


def smooth_flux_vjp(Q, D, gamma, prandtl, mu, rho_ref, p_ref, Fb, dFb):
    Q, D, Fb, dFb = _a(Q, 5), _a(D, 15), _a(Fb, 5), _a(dFb, 5)
    Qb, Db = np.zeros(5), np.zeros(15)
    lib().dm_smooth_flux_vjp(_p(Q), _p(D), ctypes.c_double(gamma), ctypes.c_double(prandtl), ctypes.c_double(mu),
                             ctypes.c_double(rho_ref), ctypes.c_double(p_ref), _p(Fb), _p(dFb), _p(Qb), _p(Db))
    return Qb, Db


def compat(Ql, Qr, gamma, rho_ref, p_ref):
    Ql, Qr = _a(Ql, 5), _a(Qr, 5)
    Q0 = np.zeros(5)
    lib().dm_compat(_p(Ql), _p(Qr), ctypes.c_double(gamma), ctypes.c_double(rho_ref), ctypes.c_double(p_ref), _p(Q0))
    return Q0


def compat_vjp(Ql, Qr, gamma, rho_ref, p_ref, Q0b):
    Ql, Qr, Q0b = _a(Ql, 5), _a(Qr, 5), _a(Q0b, 5)
    Qlb, Qrb = np.zeros(5), np.zeros(5)
    lib().dm_compat_vjp(_p(Ql), _p(Qr), ctypes.c_double(gamma), ctypes.c_double(rho_ref), ctypes.c_double(p_ref),
                        _p(Q0b), _p(Qlb), _p(Qrb))
    return Qlb, Qrb


def weno_z_right(v, eps=1e-6, p=2):
    v = _a(v, 5)
    val, slope = np.zeros(1), np.zeros(1)
    lib().dm_weno_z_right(_p(v), ctypes.c_double(eps), ctypes.c_int(p), _p(val), _p(slope))
    return float(val[0]), float(slope[0])


def weno_z_edges(v, eps=1e-6, p=2):
    v = _a(v, 5)
    ea, eb = np.zeros(1), np.zeros(1)
    lib().dm_weno_z_edges(_p(v), ctypes.c_double(eps), ctypes.c_int(p), _p(ea), _p(eb))
    return float(ea[0]), float(eb[0])


def full_flux(Ql, Dl, Qr, Dr, Q0, D0, tau, dt, gamma, prandtl, rho_ref, p_ref):
    args = [_a(Ql, 5), _a(Dl, 15), _a(Qr, 5), _a(Dr, 15), _a(Q0, 5), _a(D0, 15)]
    F, dF = np.zeros(5), np.zeros(5)
    lib().dm_full_flux(*[_p(a) for a in args], ctypes.c_double(tau), ctypes.c_double(dt), ctypes.c_double(gamma),
                       ctypes.c_double(prandtl), ctypes.c_double(rho_ref), ctypes.c_double(p_ref), _p(F), _p(dF))
    return F, dF


def _zargs(dt, gamma, prandtl, mu, T_ref, mu_exp, c_art, rho_ref, p_ref):
    return [ctypes.c_double(v) for v in (dt, gamma, prandtl, mu, T_ref, mu_exp, c_art, rho_ref, p_ref)]


def zgp_flux(X, dt, gamma, prandtl, mu, T_ref, mu_exp, c_art, rho_ref, p_ref):
    X = _a(X, 60)
    F, dF = np.zeros(5), np.zeros(5)
    lib().dm_zgp_flux(_p(X), *_zargs(dt, gamma, prandtl, mu, T_ref, mu_exp, c_art, rho_ref, p_ref), _p(F), _p(dF))
    return F, dF


def zflux_jt(X, dt, gamma, prandtl, mu, T_ref, mu_exp, c_art, rho_ref, p_ref, Fb, dFb):
    X, Fb, dFb = _a(X, 60), _a(Fb, 5), _a(dFb, 5)
    Xb = np.zeros(60)
    lib().dm_zflux_jt(_p(X), *_zargs(dt, gamma, prandtl, mu, T_ref, mu_exp, c_art, rho_ref, p_ref), _p(Fb), _p(dFb),
                      _p(Xb))
    return Xb


def zflux_vjp(X, dt, gamma, prandtl, mu, T_ref, mu_exp, c_art, rho_ref, p_ref, Fb, dFb):
    X, Fb, dFb = _a(X, 60), _a(Fb, 5), _a(dFb, 5)
    Xb = np.zeros(60)
    lib().dm_zflux_vjp(_p(X), *_zargs(dt, gamma, prandtl, mu, T_ref, mu_exp, c_art, rho_ref, p_ref), _p(Fb),
                            _p(dFb), _p(Xb))
    return Xb


def wze_jac(v, eps, p):
    v = _a(v, 5)
    J = np.zeros((2, 5))
    lib().dm_wze_jac(_p(v), ctypes.c_double(eps), ctypes.c_int(p), _p(J))
    return J


def wze_vjp(v, eps, p, eab, ebb):
    v = _a(v, 5)
    vb = np.zeros(5)
    lib().dm_wze_vjp(_p(v), ctypes.c_double(eps), ctypes.c_int(p), ctypes.c_double(eab), ctypes.c_double(ebb), _p(vb))
    return vb


def wzr_vjp(v, eps, p, valb, slopeb):
    v = _a(v, 5)
    vb = np.zeros(5)
    lib().dm_wzr_vjp(_p(v), ctypes.c_double(eps), ctypes.c_int(p), ctypes.c_double(valb), ctypes.c_double(slopeb),
                     _p(vb))
    return vb


def wzr_jac(v, eps, p):
    v = _a(v, 5)
    Jv, Js = np.zeros(5), np.zeros(5)
    lib().dm_wzr_jac(_p(v), ctypes.c_double(eps), ctypes.c_int(p), _p(Jv), _p(Js))
    return Jv, Js
