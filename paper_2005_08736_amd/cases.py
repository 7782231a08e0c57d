"""Seeded synthetic inputs: parameters and initial cell averages of the paper's cases.

This module holds the problem set-ups only (initial fields and physical
parameters, Sec. 3 of Cao, Pan & Xu, arXiv:2005.08736); it contains none of the
scheme's arithmetic.  Both the HIP path and the CPU oracle take their inputs from
here.  States are numpy float64 arrays ``[5][nz][ny][nx]`` of cell averages of
(rho, rho U, rho V, rho W, rho E).

Cell averages are taken with the 4-point Gauss-Legendre rule per axis.  Fields
that are sums of products of one-dimensional factors (Taylor-Green, density
wave, channel profile) are averaged term by term: the tensor Gauss rule of a
separable term is the product of the one-dimensional rules, so the result equals
the 64-point tensor rule without evaluating it point by point.
"""
from __future__ import annotations

import math

import numpy as np

_GL_X, _GL_W = np.polynomial.legendre.leggauss(4)
_GL_X = 0.5 * _GL_X  # offsets in units of the cell width, in (-1/2, 1/2)
_GL_W = 0.5 * _GL_W  # weights sum to 1


PARAM_DEFAULTS = dict(
    nx=32, ny=32, nz=32,
    lx=2 * math.pi, ly=2 * math.pi, lz=2 * math.pi,
    bc_y=0, stretch_b=0.0,
    gamma=1.4, prandtl=0.72,
    mu_ref=1.0 / 1600.0, T_ref=1.0, mu_exp=0.0,
    mode=0, cfl=0.4,
    c_art=1.0, weno_eps=1e-6, weno_p=2,
    T_wall=1.0, body_force_x=0.0, bulk_momentum=0.0,
)


def params(**kw) -> dict:
    """Parameter dict with every field set (unknown keys are rejected)."""
    p = dict(PARAM_DEFAULTS)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(k)
        p[k] = v
    return p


# ---------------------------------------------------------------------------
# separable cell averaging
# ---------------------------------------------------------------------------

def _gl_points(n: int, length: float, origin: float = 0.0) -> np.ndarray:
    """Gauss points of n uniform cells on [origin, origin+length]: shape (n, 4)."""
    h = length / n
    centres = origin + (np.arange(n) + 0.5) * h
    return centres[:, None] + _GL_X[None, :] * h


def _avg1(values: np.ndarray) -> np.ndarray:
    """Cell averages from values at the 4 Gauss points per cell: (n, 4) -> (n,)."""
    return values @ _GL_W


class Sep:
    """A sum of separable terms c * fx(x) fy(y) fz(z), with each factor sampled
    at the Gauss points of its axis (arrays of shape (n_axis, 4))."""

    def __init__(self, terms):
        self.terms = list(terms)

    @staticmethod
    def one(shape_xyz):
        nx, ny, nz = shape_xyz
        return Sep([(1.0, np.ones((nx, 4)), np.ones((ny, 4)), np.ones((nz, 4)))])

    def __add__(self, o):
        return Sep(self.terms + o.terms)

    def __mul__(self, o):
        if isinstance(o, (int, float)):
            return Sep([(c * o, a, b, d) for (c, a, b, d) in self.terms])
        return Sep([(c1 * c2, a1 * a2, b1 * b2, d1 * d2)
                    for (c1, a1, b1, d1) in self.terms for (c2, a2, b2, d2) in o.terms])

    __rmul__ = __mul__

    def average(self) -> np.ndarray:
        """Cell averages, array [nz][ny][nx]."""
        out = None
        for c, a, b, d in self.terms:
            t = c * _avg1(d)[:, None, None] * _avg1(b)[None, :, None] * _avg1(a)[None, None, :]
            out = t if out is None else out + t
        return out


def _fx(vals, ny, nz):
    return Sep([(1.0, vals, np.ones((ny, 4)), np.ones((nz, 4)))])


def _fy(vals, nx, nz):
    return Sep([(1.0, np.ones((nx, 4)), vals, np.ones((nz, 4)))])


def _fz(vals, nx, ny):
    return Sep([(1.0, np.ones((nx, 4)), np.ones((ny, 4)), vals)])


# ---------------------------------------------------------------------------
# Taylor-Green vortex (Sec. 3.1)
# ---------------------------------------------------------------------------

def tgv_params(n: int, **kw) -> dict:
    """3-D Taylor-Green vortex on the periodic box [0, 2 pi]^3, Re = 1600, Ma = 0.1.
    mu = rho0 V0 L / Re with rho0 = V0 = L = 1; Pr and gamma as given."""
    base = dict(nx=n, ny=n, nz=n, lx=2 * math.pi, ly=2 * math.pi, lz=2 * math.pi,
                gamma=1.4, prandtl=0.72, mu_ref=1.0 / 1600.0, T_ref=1.0, mu_exp=0.0, mode=0, cfl=0.4)
    base.update(kw)
    return params(**base)


def tgv_state(n: int, gamma: float = 1.4, mach: float = 0.1, V0: float = 1.0, rho0: float = 1.0,
              nxyz=None) -> np.ndarray:
    """Cell averages of the Taylor-Green initial field:
    U = V0 sin x cos y cos z, V = -V0 cos x sin y cos z, W = 0,
    p = p0 + rho0 V0^2/16 (cos 2x + cos 2y)(cos 2z + 2), p0 = rho0 V0^2/(gamma Ma^2),
    uniform temperature T0 = p0/rho0, rho = p / T0."""
    nx, ny, nz = nxyz if nxyz is not None else (n, n, n)
    L = 2 * math.pi
    x, y, z = _gl_points(nx, L), _gl_points(ny, L), _gl_points(nz, L)
    p0 = rho0 * V0 ** 2 / (gamma * mach ** 2)
    T0 = p0 / rho0
    sx, cx, c2x = _fx(np.sin(x), ny, nz), _fx(np.cos(x), ny, nz), _fx(np.cos(2 * x), ny, nz)
    sy, cy, c2y = _fy(np.sin(y), nx, nz), _fy(np.cos(y), nx, nz), _fy(np.cos(2 * y), nx, nz)
    cz, c2z = _fz(np.cos(z), nx, ny), _fz(np.cos(2 * z), nx, ny)
    one = Sep.one((nx, ny, nz))
    p = one * p0 + (c2x + c2y) * (c2z + one * 2.0) * (rho0 * V0 ** 2 / 16.0)
    rho = p * (1.0 / T0)
    U = sx * cy * cz * V0
    V = cx * sy * cz * (-V0)
    q = np.empty((5, nz, ny, nx))
    q[0] = rho.average()
    q[1] = (rho * U).average()
    q[2] = (rho * V).average()
    q[3] = 0.0
    q[4] = (p * (1.0 / (gamma - 1.0)) + rho * (U * U + V * V) * 0.5).average()
    return q


# ---------------------------------------------------------------------------
# uniform flow and the advected density wave
# ---------------------------------------------------------------------------

def uniform_state(nx, ny, nz, rho=1.0, vel=(0.3, -0.2, 0.1), p=1.0, gamma=1.4) -> np.ndarray:
    q = np.empty((5, nz, ny, nx))
    q[0] = rho
    for a in range(3):
        q[1 + a] = rho * vel[a]
    q[4] = p / (gamma - 1.0) + 0.5 * rho * sum(v * v for v in vel)
    return q


def density_wave_params(n: int, diagonal: bool = True, ny: int | None = None, nz: int | None = None, **kw) -> dict:
    """Periodic [0,2]^3, inviscid (mu = 0): rho = 1 + 0.2 sin(pi (x+y+z - 3t))
    (diagonal) or rho = 1 + 0.2 sin(pi (x - t)) (along x), U = (1,1,1) or (1,0,0), p = 1."""
    ny = ny if ny is not None else (n if diagonal else 6)
    nz = nz if nz is not None else (n if diagonal else 6)
    base = dict(nx=n, ny=ny, nz=nz, lx=2.0, ly=2.0 * ny / n if not diagonal else 2.0,
                lz=2.0 * nz / n if not diagonal else 2.0, mu_ref=0.0, prandtl=1.0, mode=0, cfl=0.4)
    base.update(kw)
    return params(**base)


def density_wave_state(prm: dict, t: float = 0.0, diagonal: bool = True, amp: float = 0.2,
                       gamma: float = 1.4) -> np.ndarray:
    nx, ny, nz = prm["nx"], prm["ny"], prm["nz"]
    x = _gl_points(nx, prm["lx"])
    y = _gl_points(ny, prm["ly"])
    z = _gl_points(nz, prm["lz"])
    one = Sep.one((nx, ny, nz))
    if diagonal:
        # sin(a+b+c) with a = pi(x-t), b = pi(y-t), c = pi(z-t)
        sa, ca = _fx(np.sin(math.pi * (x - t)), ny, nz), _fx(np.cos(math.pi * (x - t)), ny, nz)
        sb, cb = _fy(np.sin(math.pi * (y - t)), nx, nz), _fy(np.cos(math.pi * (y - t)), nx, nz)
        sc, cc = _fz(np.sin(math.pi * (z - t)), nx, ny), _fz(np.cos(math.pi * (z - t)), nx, ny)
        s = sa * cb * cc + ca * sb * cc + ca * cb * sc + sa * sb * sc * (-1.0)
        vel = (1.0, 1.0, 1.0)
    else:
        s = _fx(np.sin(math.pi * (x - t)), ny, nz)
        vel = (1.0, 0.0, 0.0)
    rho = one + s * amp
    q = np.empty((5, nz, ny, nx))
    r = rho.average()
    q[0] = r
    for a in range(3):
        q[1 + a] = vel[a] * r
    q[4] = 1.0 / (gamma - 1.0) + 0.5 * sum(v * v for v in vel) * r
    return q


# ---------------------------------------------------------------------------
# random solenoidal fields (isotropic turbulence, Sec. 3.4; adjoint perturbation)
# ---------------------------------------------------------------------------

def solenoidal_field(n: int, seed: int, spectrum, cell_average: bool = True) -> np.ndarray:
    """Real solenoidal velocity (3, n, n, n) on [0, 2 pi]^3 with energy spectrum
    E(|k|) for 0 < |k| <= n/2: u_hat(k) = sqrt(E(|k|) / (2 pi |k|^2)) e(k), e a unit
    complex vector orthogonal to k with uniform random phases (numpy PCG64).  The
    field is made Hermitian (real) by taking the real part of the inverse FFT of the
    one-sided construction.  With cell_average the Fourier modes are multiplied by
    prod_d sinc(k_d h / 2), which turns point values into cell averages."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    # two unit vectors orthogonal to k
    kvec = np.stack([kx, ky, kz])
    ref_axis = np.where(np.abs(kz)[None] < 0.9 * np.maximum(kk, 1e-30)[None],
                        np.array([0.0, 0.0, 1.0])[:, None, None, None],
                        np.array([1.0, 0.0, 0.0])[:, None, None, None])
    e1 = np.cross(kvec, ref_axis, axis=0)
    e1 /= np.maximum(np.linalg.norm(e1, axis=0), 1e-30)[None]
    e2 = np.cross(kvec, e1, axis=0)
    e2 /= np.maximum(np.linalg.norm(e2, axis=0), 1e-30)[None]
    th1 = rng.uniform(0.0, 2 * math.pi, size=kk.shape)
    th2 = rng.uniform(0.0, 2 * math.pi, size=kk.shape)
    phi = rng.uniform(0.0, 2 * math.pi, size=kk.shape)
    amp = np.zeros_like(kk)
    mask = (kk > 0) & (kk <= n / 2)
    amp[mask] = np.sqrt(spectrum(kk[mask]) / (2 * math.pi * kk[mask] ** 2))
    coef = (np.exp(1j * th1) * np.cos(phi))[None] * e1 + (np.exp(1j * th2) * np.sin(phi))[None] * e2
    uh = amp[None] * coef
    if cell_average:
        h = 2 * math.pi / n
        s = np.sinc(kx * h / (2 * math.pi)) * np.sinc(ky * h / (2 * math.pi)) * np.sinc(kz * h / (2 * math.pi))
        uh = uh * s[None]
    u = np.real(np.fft.ifftn(uh, axes=(1, 2, 3))) * n ** 3
    return u  # (3, z, y, x) after meshgrid 'ij' on (z, y, x)


ISO_A0 = 1.3e-4
ISO_K0 = 8.0


def isotropic_constants(re_lambda: float = 72.0, A0: float = ISO_A0, k0: float = ISO_K0, rho0: float = 1.0) -> dict:
    """Closed forms of Sec. 3.4: Re_lambda -> mu0; K0, Omega0, tau_to, eps0, eta0, tau0."""
    mu0 = (2 * math.pi) ** 0.25 / 4.0 * rho0 * math.sqrt(2 * A0) * k0 ** 1.5 / re_lambda
    K0 = 3 * A0 / 64.0 * math.sqrt(2 * math.pi) * k0 ** 5
    Om0 = 15 * A0 / 256.0 * math.sqrt(2 * math.pi) * k0 ** 7
    tau_to = math.sqrt(32.0 / A0) * (2 * math.pi) ** 0.25 * k0 ** -3.5
    eps0 = 2 * mu0 / rho0 * Om0
    nu0 = mu0 / rho0
    eta0 = (nu0 ** 3 / eps0) ** 0.25
    tau0 = (nu0 / eps0) ** 0.5
    u_rms = math.sqrt(2 * K0 / 3.0)
    return dict(mu0=mu0, K0=K0, Omega0=Om0, tau_to=tau_to, eps0=eps0, eta0=eta0, tau0=tau0, u_rms=u_rms)


def isotropic_params(n: int, ma_t: float, mode: int = 1, **kw) -> dict:
    c = isotropic_constants()
    gamma = kw.pop("gamma", 1.4)
    c0 = math.sqrt(3.0) * c["u_rms"] / ma_t
    T0 = c0 ** 2 / gamma
    base = dict(nx=n, ny=n, nz=n, lx=2 * math.pi, ly=2 * math.pi, lz=2 * math.pi, gamma=gamma,
                prandtl=0.72, mu_ref=c["mu0"], T_ref=T0, mu_exp=0.76, mode=mode, cfl=0.4)
    base.update(kw)
    return params(**base)


def isotropic_state(n: int, seed: int, ma_t: float, gamma: float = 1.4) -> np.ndarray:
    """Solenoidal velocity with E(k) = A0 k^4 exp(-2 k^2 / k0^2), rescaled to
    u_rms = sqrt(2 K0 / 3); rho = 1, uniform T0 = c0^2/gamma with c0 = sqrt(3) u_rms / Ma_t."""
    c = isotropic_constants()
    u = solenoidal_field(n, seed, lambda k: ISO_A0 * k ** 4 * np.exp(-2 * k ** 2 / ISO_K0 ** 2))
    urms = math.sqrt(np.mean(np.sum(u ** 2, axis=0)) / 3.0)
    u *= c["u_rms"] / urms
    c0 = math.sqrt(3.0) * c["u_rms"] / ma_t
    p0 = c0 ** 2 / gamma  # rho0 = 1
    q = np.empty((5, n, n, n))
    q[0] = 1.0
    q[1:4] = u
    q[4] = p0 / (gamma - 1.0) + 0.5 * np.sum(u ** 2, axis=0)
    return q


def solenoidal_perturbation(n: int, seed: int, kmax: float = 4.0, rms: float = 0.01) -> np.ndarray:
    """Flat-spectrum solenoidal field for |k| <= kmax, rescaled to the given rms
    per component; shape (3, n, n, n)."""
    u = solenoidal_field(n, seed, lambda k: np.where(k <= kmax, 1.0, 0.0))
    r = math.sqrt(np.mean(np.sum(u ** 2, axis=0)) / 3.0)
    return u * (rms / r)


# ---------------------------------------------------------------------------
# channel (Sec. 3.3)
# ---------------------------------------------------------------------------

def channel_params(nx=128, ny=128, nz=128, **kw) -> dict:
    """2 pi x 2 x pi channel, tanh-stretched in y (b_g = 2), isothermal no-slip
    walls, Ma = 0.1 on the unit bulk velocity (c0 = 10, T_w = c0^2/gamma),
    mu = u_tau / Re_tau with u_tau = 0.0541, Re_tau = 180, constant f_x = 2.93e-3."""
    gamma = kw.pop("gamma", 1.4)
    c0 = 10.0
    Tw = c0 ** 2 / gamma
    base = dict(nx=nx, ny=ny, nz=nz, lx=2 * math.pi, ly=2.0, lz=math.pi, bc_y=1, stretch_b=2.0,
                gamma=gamma, prandtl=0.72, mu_ref=0.0541 / 180.0, T_ref=Tw, mu_exp=0.0, mode=0, cfl=0.4,
                T_wall=Tw, body_force_x=2.93e-3)
    base.update(kw)
    return params(**base)


def channel_y(ny: int, b: float = 2.0):
    """Face and centre positions of the stretched wall-normal mesh:
    y = tanh(b (eta / (1.5 pi) - 1)) / tanh b, eta uniform on [0, 3 pi]."""
    deta = 3 * math.pi / ny
    eta_f = np.arange(ny + 1) * deta
    yf = np.tanh(b * (eta_f / (1.5 * math.pi) - 1.0)) / math.tanh(b)
    eta_c = (np.arange(ny) + 0.5) * deta
    yc = np.tanh(b * (eta_c / (1.5 * math.pi) - 1.0)) / math.tanh(b)
    return yf, yc


def channel_state(prm: dict, seed: int = 0, noise: float = 0.1) -> np.ndarray:
    """rho = 1, T = T_w, U = 1.5 (1 - y^2)(1 + noise r), r ~ U(-1, 1) per cell
    (seeded PCG64), V = W = 0; the profile is averaged over each stretched cell
    with the 4-point rule in eta."""
    nx, ny, nz = prm["nx"], prm["ny"], prm["nz"]
    gamma, Tw = prm["gamma"], prm["T_wall"]
    b = prm["stretch_b"]
    deta = 3 * math.pi / ny
    eta = (np.arange(ny)[:, None] + 0.5 + _GL_X[None, :]) * deta
    y = np.tanh(b * (eta / (1.5 * math.pi) - 1.0)) / math.tanh(b)
    dyde = b / (1.5 * math.pi) * (1 - np.tanh(b * (eta / (1.5 * math.pi) - 1.0)) ** 2) / math.tanh(b)
    prof = 1.5 * (1 - y ** 2)
    # average over the physical cell: int U dy / int dy with dy = y'(eta) d eta
    Ubar = (prof * dyde) @ _GL_W / (dyde @ _GL_W)
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    U = Ubar[None, :, None] * (1.0 + noise * r)
    rho = 1.0
    p = rho * Tw
    q = np.empty((5, nz, ny, nx))
    q[0] = rho
    q[1] = rho * U
    q[2] = 0.0
    q[3] = 0.0
    q[4] = p / (gamma - 1.0) + 0.5 * rho * U ** 2
    return q
