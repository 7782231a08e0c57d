"""Python binding of libhgks (the C ABI of include/hgks.h).

Argument marshalling only: every step of the scheme runs in the HIP kernels of
``libhgks.so``.  PyTorch provides the device memory (state, workspace, outputs)
and the stream.  Importing works without a GPU; creating a :class:`Solver` needs
the built library and a ROCm device, and raises otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhgks.so")

HGKS_OK = 0
HGKS_E_INVALID_ARG = -1
HGKS_E_DEVICE = -2
HGKS_E_NONPHYSICAL = -3
HGKS_E_UNSUPPORTED = -4
HGKS_E_WORKSPACE = -5
HGKS_NDIAG = 34
MODE_SMOOTH, MODE_WENOZ, MODE_WENOZ_CHAR = 0, 1, 2
PREC_F64, PREC_F32FLUX = 0, 1

DIAG_NAMES = [
    "mass", "mom_x", "mom_y", "mom_z", "energy", "E_k", "zeta", "eps1", "eps2", "eps3",
    "rho_rms", "u_rms", "Ma_t", "min_rho", "min_p", "K", "eps_s", "eps_d", "p_theta", "rho_mean",
    "dudx2", "dvdy2", "dwdz2", "dudx3", "dvdy3", "dwdz3", "dudx4", "dvdy4", "dwdz4",
    "S_u", "F_u", "c_mean", "volume", "max_speed",
]

EXPORTED = [
    "hgks_workspace_bytes", "hgks_init", "hgks_step", "hgks_operator", "hgks_face_flux",
    "hgks_diagnostics", "hgks_failed_step", "hgks_destroy", "hgks_strerror",
    "hgks_profile_enable", "hgks_profile_read", "hgks_step_vjp", "hgks_dilatation_pdf",
    "hgks_plane_profiles", "hgks_dilatation_slice", "hgks_wall_flux", "hgks_step_static",
]
STATIC_WORKSPACE_BYTES = 64 << 20
PDF_MAX_BINS = 4096
PROFILE_NAMES = ["rho", "U", "V", "W", "p", "T", "uu", "vv", "ww", "uv", "rhoU"]
KCLASS_NAMES = ["dt", "flux_stage1", "flux_stage2", "stage1", "stage2", "operator_vjp"]


class HgksParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
        ("bc_y", ctypes.c_int32), ("stretch_b", ctypes.c_double),
        ("gamma", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("mu_ref", ctypes.c_double), ("T_ref", ctypes.c_double), ("mu_exp", ctypes.c_double),
        ("mode", ctypes.c_int32), ("cfl", ctypes.c_double),
        ("c_art", ctypes.c_double), ("weno_eps", ctypes.c_double), ("weno_p", ctypes.c_int32),
        ("T_wall", ctypes.c_double), ("body_force_x", ctypes.c_double),
        ("precision", ctypes.c_int32), ("bulk_momentum", ctypes.c_double),
    ]


class HgksError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


_lib = None


def load():
    """Load libhgks.so (built in-tree by ``paper_2005_08736_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2005_08736_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(HgksParams)
    vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    D = ctypes.POINTER(ctypes.c_double)
    L.hgks_workspace_bytes.restype = sz
    L.hgks_workspace_bytes.argtypes = [P]
    L.hgks_init.restype = ctypes.c_int
    L.hgks_init.argtypes = [P, vp, vp, sz, vp, ctypes.POINTER(vp)]
    L.hgks_step.restype = ctypes.c_int
    L.hgks_step.argtypes = [vp, i32, dbl, D]
    L.hgks_operator.restype = ctypes.c_int
    L.hgks_operator.argtypes = [vp, vp, dbl, vp, vp]
    L.hgks_face_flux.restype = ctypes.c_int
    L.hgks_face_flux.argtypes = [vp, i32, vp, dbl, vp, vp]
    L.hgks_diagnostics.restype = ctypes.c_int
    L.hgks_diagnostics.argtypes = [vp, D]
    L.hgks_failed_step.restype = ctypes.c_int
    L.hgks_failed_step.argtypes = [vp]
    L.hgks_destroy.restype = None
    L.hgks_destroy.argtypes = [vp]
    L.hgks_profile_enable.restype = ctypes.c_int
    L.hgks_profile_enable.argtypes = [vp, ctypes.c_int]
    L.hgks_profile_read.restype = ctypes.c_int
    L.hgks_profile_read.argtypes = [vp, D, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    L.hgks_step_static.restype = ctypes.c_int
    L.hgks_step_static.argtypes = [P, vp, i32, dbl, D, vp]
    L.hgks_wall_flux.restype = ctypes.c_int
    L.hgks_wall_flux.argtypes = [vp, vp, vp, vp]
    L.hgks_step_vjp.restype = ctypes.c_int
    L.hgks_step_vjp.argtypes = [vp, vp, dbl, vp, vp]
    L.hgks_dilatation_pdf.restype = ctypes.c_int
    L.hgks_dilatation_pdf.argtypes = [vp, ctypes.c_int32, dbl, dbl, ctypes.POINTER(ctypes.c_int64), D]
    L.hgks_plane_profiles.restype = ctypes.c_int
    L.hgks_plane_profiles.argtypes = [vp, D]
    L.hgks_dilatation_slice.restype = ctypes.c_int
    L.hgks_dilatation_slice.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, D, D]
    L.hgks_strerror.restype = ctypes.c_char_p
    L.hgks_strerror.argtypes = [ctypes.c_int]
    _lib = L
    return L


def strerror(status: int) -> str:
    return load().hgks_strerror(int(status)).decode()


def make_params(d: dict) -> HgksParams:
    p = HgksParams()
    for name, _ in HgksParams._fields_:
        setattr(p, name, d.get(name, 0))
    return p


def workspace_bytes(params: dict) -> int:
    return int(load().hgks_workspace_bytes(ctypes.byref(make_params(params))))


def step_static(params: dict, q: torch.Tensor, nsteps: int = 1, dt: float = 0.0, return_dt: bool = False,
                stream: torch.cuda.Stream | None = None):
    """hgks_step_static: advance q (contiguous float64 device tensor [5, nz, ny,
    nx], in place) by nsteps steps using the library's static device workspace
    instead of an allocated one.  Returns the time steps when return_dt."""
    if not (q.is_cuda and q.dtype == torch.float64 and q.is_contiguous()):
        raise ValueError("q must be a contiguous float64 device tensor")
    if tuple(q.shape) != (5, params["nz"], params["ny"], params["nx"]):
        raise ValueError(f"q has shape {tuple(q.shape)}, expected (5, nz, ny, nx)")
    stream = stream if stream is not None else torch.cuda.current_stream(q.device)
    buf = (ctypes.c_double * max(int(nsteps), 1))()
    st = load().hgks_step_static(ctypes.byref(make_params(params)), ctypes.c_void_p(q.data_ptr()), int(nsteps),
                                 float(dt), buf if return_dt else None, ctypes.c_void_p(stream.cuda_stream))
    if st != HGKS_OK:
        raise HgksError(st, "hgks_step_static")
    return [buf[i] for i in range(int(nsteps))] if return_dt else None


def _check(status: int, what: str):
    if status != HGKS_OK:
        raise HgksError(status, what)


class Solver:
    """One HGKS state on one device: binds a caller-owned CUDA/HIP float64 tensor
    ``q`` of shape [5, nz, ny, nx] (updated in place) and a workspace tensor."""

    def __init__(self, params: dict, q: torch.Tensor, stream: torch.cuda.Stream | None = None):
        L = load()
        if not (q.is_cuda and q.dtype == torch.float64 and q.is_contiguous()):
            raise ValueError("q must be a contiguous float64 device tensor")
        if tuple(q.shape) != (5, params["nz"], params["ny"], params["nx"]):
            raise ValueError(f"q has shape {tuple(q.shape)}, expected (5, nz, ny, nx)")
        self.params = dict(params)
        self._p = make_params(params)
        nbytes = int(L.hgks_workspace_bytes(ctypes.byref(self._p)))
        if nbytes == 0:
            raise HgksError(HGKS_E_INVALID_ARG, "hgks_workspace_bytes")
        self.q = q
        self.stream = stream if stream is not None else torch.cuda.current_stream(q.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=q.device)
        h = ctypes.c_void_p()
        _check(L.hgks_init(ctypes.byref(self._p), ctypes.c_void_p(q.data_ptr()),
                           ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "hgks_init")
        self._h = h

    def step(self, nsteps: int = 1, dt: float = 0.0, return_dt: bool = False):
        """Advance nsteps steps (dt <= 0: CFL time step); optionally return the dts."""
        buf = (ctypes.c_double * max(int(nsteps), 1))()
        st = load().hgks_step(self._h, int(nsteps), float(dt), buf if return_dt else None)
        if st != HGKS_OK:
            raise HgksError(st, "hgks_step")
        return [buf[i] for i in range(int(nsteps))] if return_dt else None

    def step_status(self, nsteps: int = 1, dt: float = 0.0) -> int:
        return int(load().hgks_step(self._h, int(nsteps), float(dt), None))

    def failed_step(self) -> int:
        return int(load().hgks_failed_step(self._h))

    def operator(self, q_in: torch.Tensor | None = None, dt: float = 0.0):
        q_in = self.q if q_in is None else q_in
        L = torch.empty_like(self.q)
        dL = torch.empty_like(self.q)
        _check(load().hgks_operator(self._h, ctypes.c_void_p(q_in.data_ptr()), float(dt),
                                    ctypes.c_void_p(L.data_ptr()), ctypes.c_void_p(dL.data_ptr())), "hgks_operator")
        return L, dL

    def face_flux(self, direction: int, q_in: torch.Tensor | None = None, dt: float = 0.0):
        q_in = self.q if q_in is None else q_in
        F = torch.empty_like(self.q)
        dF = torch.empty_like(self.q)
        _check(load().hgks_face_flux(self._h, int(direction), ctypes.c_void_p(q_in.data_ptr()), float(dt),
                                     ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(dF.data_ptr())),
               "hgks_face_flux")
        return F, dF

    def wall_flux(self, q_in: torch.Tensor | None = None):
        """Face fluxes (F, dF) of the channel's wall faces (hgks_wall_flux): device
        tensors [2, 5, nz, nx], entry 0 the bottom wall, 1 the top wall."""
        q_in = self.q if q_in is None else q_in
        shape = (2, 5, self.params["nz"], self.params["nx"])
        F = torch.empty(shape, dtype=torch.float64, device=self.q.device)
        dF = torch.empty(shape, dtype=torch.float64, device=self.q.device)
        _check(load().hgks_wall_flux(self._h, ctypes.c_void_p(q_in.data_ptr()), ctypes.c_void_p(F.data_ptr()),
                                     ctypes.c_void_p(dF.data_ptr())), "hgks_wall_flux")
        return F, dF

    def step_vjp(self, q_n: torch.Tensor, dt: float, lam_np1: torch.Tensor) -> torch.Tensor:
        """(dQ^{n+1}/dQ^n)^T lam_np1 for one step of frozen dt starting at q_n."""
        lam_n = torch.empty_like(self.q)
        _check(load().hgks_step_vjp(self._h, ctypes.c_void_p(q_n.data_ptr()), float(dt),
                                    ctypes.c_void_p(lam_np1.data_ptr()), ctypes.c_void_p(lam_n.data_ptr())),
               "hgks_step_vjp")
        return lam_n

    def diagnostics(self) -> dict:
        out = (ctypes.c_double * HGKS_NDIAG)()
        _check(load().hgks_diagnostics(self._h, out), "hgks_diagnostics")
        return dict(zip(DIAG_NAMES, list(out)))

    def dilatation_pdf(self, nbins: int, lo: float, hi: float):
        """Histogram of theta / theta_rms (hgks_dilatation_pdf): returns (counts,
        theta_rms), counts an int64 array of nbins + 2 (below lo, the bins, at or
        above hi)."""
        if not 1 <= int(nbins) <= PDF_MAX_BINS:
            raise ValueError(f"nbins must lie in [1, {PDF_MAX_BINS}]")
        counts = np.zeros(int(nbins) + 2, dtype=np.int64)
        rms = ctypes.c_double(0.0)
        _check(load().hgks_dilatation_pdf(self._h, int(nbins), float(lo), float(hi),
                                          counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(rms)),
               "hgks_dilatation_pdf")
        return counts, rms.value

    def dilatation_slice(self, axis: int, index: int):
        """theta / theta_rms on the plane `index` of `axis` (hgks_dilatation_slice):
        returns (plane, theta_rms), plane shaped by the two remaining axes in state
        order ([nz, ny], [nz, nx] or [ny, nx])."""
        n = [self.params["nx"], self.params["ny"], self.params["nz"]]
        fa, sa = (1 if axis == 0 else 0), (1 if axis == 2 else 2)
        out = np.zeros((n[sa], n[fa]))
        rms = ctypes.c_double(0.0)
        _check(load().hgks_dilatation_slice(self._h, int(axis), int(index),
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(rms)),
               "hgks_dilatation_slice")
        return out, rms.value

    def plane_profiles(self) -> np.ndarray:
        """Per-y-row plane averages (hgks_plane_profiles): array [ny, 11], columns
        as PROFILE_NAMES."""
        ny = self.params["ny"]
        out = np.zeros((ny, len(PROFILE_NAMES)))
        _check(load().hgks_plane_profiles(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "hgks_plane_profiles")
        return out

    def profile(self, enable: bool = True):
        _check(load().hgks_profile_enable(self._h, int(bool(enable))), "hgks_profile_enable")

    def profile_read(self) -> dict:
        n = len(KCLASS_NAMES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(load().hgks_profile_read(self._h, ms, cnt, n), "hgks_profile_read")
        return {KCLASS_NAMES[k]: (ms[k], int(cnt[k])) for k in range(n)}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hgks_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
