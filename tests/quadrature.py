"""Independent numerical quadrature of Maxwellian moments, used to pin the
oracle's closed-form moment recursions.  Gauss-Hermite rules are exact for the
polynomial integrands that appear (degree <= 6 per variable, so 6 nodes are exact); half-space
integrals use a high-order Gauss-Legendre rule on a truncated interval."""
import math

import numpy as np

_HX, _HW = np.polynomial.hermite.hermgauss(6)


def _gauss_axis(U, lam, half=0, n_half=160):
    """Nodes and weights for E[f(u)] under the 1-D Maxwellian density
    sqrt(lam/pi) exp(-lam (u-U)^2), optionally restricted to u>0 / u<0."""
    if half == 0:
        return U + _HX / math.sqrt(lam), _HW / math.sqrt(math.pi)
    sig = 1.0 / math.sqrt(2 * lam)
    if half > 0:
        a, b = 0.0, max(U, 0.0) + 13 * sig
    else:
        a, b = min(U, 0.0) - 13 * sig, 0.0
    x, w = np.polynomial.legendre.leggauss(n_half)
    u = 0.5 * (b - a) * x + 0.5 * (b + a)
    ww = 0.5 * (b - a) * w * math.sqrt(lam / math.pi) * np.exp(-lam * (u - U) ** 2)
    return u, ww


def expect(fun, U, V, W, lam, half=0):
    """E[fun(u, v, w, xi2)] for the normalised Maxwellian with K = 2 internal
    degrees of freedom (xi a 2-vector with the same temperature)."""
    u, wu = _gauss_axis(U, lam, half)
    v, wv = _gauss_axis(V, lam)
    w, ww = _gauss_axis(W, lam)
    x1, w1 = _gauss_axis(0.0, lam)
    x2, w2 = _gauss_axis(0.0, lam)
    xi2 = (x1[:, None] ** 2 + x2[None, :] ** 2).ravel()
    wxi = (w1[:, None] * w2[None, :]).ravel()
    uu, vv, wwv, xx = np.meshgrid(u, v, w, xi2, indexing="ij")
    wt = wu[:, None, None, None] * wv[None, :, None, None] * ww[None, None, :, None] * wxi[None, None, None, :]
    return np.sum(wt * fun(uu, vv, wwv, xx))


def psi(u, v, w, xi2):
    return [np.ones_like(u), u, v, w, 0.5 * (u * u + v * v + w * w + xi2)]


def phi(X, u, v, w, xi2):
    return X[0] + X[1] * u + X[2] * v + X[3] * w + X[4] * 0.5 * (u * u + v * v + w * w + xi2)
