"""GPU parity of hgks_dilatation_pdf (the histogram of the normalized dilatation
theta / theta_rms that Sec. 3.4 uses to mark shocklets and expansion regions)
against the oracle, through the C ABI.

theta_rms must agree to 1e-12.  The counts are integers decided by FP64 values
on both sides; theta is rounded differently on the two sides (the same stencil
in another order), so a cell whose r lies within 1e-8 bin widths of a bin edge
may fall on either side.  The counts must then agree exactly up to such cells,
and exactly when there are none.

Inputs: seeded random smooth fields with a compressive part (random potential
modes), on ragged periodic boxes, a wall-bounded uniform-mesh box and the
isotropic 256^3 workload (its seeded solenoidal field plus a potential part, Ma_t
= 1)."""
import ctypes
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


def potential_velocity(nx, ny, nz, lengths, seed, modes=4, amp=0.3):
    """grad phi for phi = sum of seeded cosine modes (|k_d| <= 3 per axis)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = [(np.arange(n) + 0.5) * L / n for n, L in zip((nx, ny, nz), lengths)]
    out = [np.zeros((nz, ny, nx)) for _ in range(3)]
    for _ in range(modes):
        kk = [2 * math.pi * int(rng.integers(1, 4)) / L for L in lengths]
        ph = rng.uniform(0, 2 * math.pi, size=3)
        a = amp * rng.uniform(0.5, 1.0) / math.sqrt(sum(k * k for k in kk))
        cx, sx = np.cos(kk[0] * xs[0] + ph[0]), np.sin(kk[0] * xs[0] + ph[0])
        cy, sy = np.cos(kk[1] * xs[1] + ph[1]), np.sin(kk[1] * xs[1] + ph[1])
        cz, sz = np.cos(kk[2] * xs[2] + ph[2]), np.sin(kk[2] * xs[2] + ph[2])
        out[0] += -a * kk[0] * (cz[:, None, None] * cy[None, :, None] * sx[None, None, :])
        out[1] += -a * kk[1] * (cz[:, None, None] * sy[None, :, None] * cx[None, None, :])
        out[2] += -a * kk[2] * (sz[:, None, None] * cy[None, :, None] * cx[None, None, :])
    return out


def random_state(nx, ny, nz, lengths, seed, gamma=1.4):
    """rho, p with seeded cell noise of 5%; U a potential part plus 5% cell noise."""
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    vel = potential_velocity(nx, ny, nz, lengths, seed)
    rho = 1.0 + 0.05 * rng.uniform(-1, 1, size=(nz, ny, nx))
    p = 2.0 * (1.0 + 0.05 * rng.uniform(-1, 1, size=(nz, ny, nx)))
    q = np.empty((5, nz, ny, nx))
    q[0] = rho
    for a in range(3):
        q[1 + a] = rho * (vel[a] + 0.05 * rng.uniform(-1, 1, size=(nz, ny, nx)))
    q[4] = p / (gamma - 1) + 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / rho
    return q


def compare(p, q, nbins, lo, hi, label):
    announce(f"{label}: {p['nx']}x{p['ny']}x{p['nz']}, {nbins} bins on [{lo}, {hi})")
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev())
    s = hgks.Solver(p, qd)
    try:
        c_gpu, rms_gpu = s.dilatation_pdf(nbins, lo, hi)
        again, rms_again = s.dilatation_pdf(nbins, lo, hi)
    finally:
        s.close()
    c_ref, rms_ref, r = oracle.dilatation_pdf(p, q, nbins, lo, hi)
    t = (r - lo) * (nbins / (hi - lo))
    near = int(np.count_nonzero(np.abs(t - np.round(t)) < 1e-8))
    diff = int(np.abs(c_gpu - c_ref).sum())
    announce(f"  theta_rms {rms_gpu:.15e} oracle {rms_ref:.15e}; count differences {diff}, cells near an edge "
             f"{near}; below {c_ref[0]}, above {c_ref[-1]}")
    assert np.array_equal(again, c_gpu) and rms_again == rms_gpu, "repeated calls differ"
    assert int(c_gpu.sum()) == q[0].size
    if rms_ref == 0.0:
        assert rms_gpu == 0.0
    else:
        assert abs(rms_gpu - rms_ref) <= 1e-12 * rms_ref
    assert diff <= 2 * near
    if near == 0:
        assert np.array_equal(c_gpu, c_ref)
    return c_gpu


@pytest.mark.parametrize("shape,nbins,lo,hi", [
    ((20, 14, 11), 64, -5.0, 5.0),
    ((33, 7, 9), 1, -3.0, 2.0),
    ((16, 16, 16), hgks.PDF_MAX_BINS, -4.0, 4.0),
])
def test_dilatation_pdf_periodic_ragged(shape, nbins, lo, hi):
    nx, ny, nz = shape
    L = (1.0 * nx / 16, 1.5 * ny / 16, 0.8 * nz / 16)
    p = cases.params(nx=nx, ny=ny, nz=nz, lx=L[0], ly=L[1], lz=L[2], mu_ref=1e-3)
    q = random_state(nx, ny, nz, L, seed=nx + 100 * ny + 10000 * nz)
    compare(p, q, nbins, lo, hi, "periodic random")


def test_dilatation_pdf_walls_uniform_mesh():
    nx, ny, nz = 24, 18, 16
    p = cases.channel_params(nx, ny, nz, stretch_b=0.0, ly=2.0)
    q = random_state(nx, ny, nz, (p["lx"], p["ly"], p["lz"]), seed=7)
    compare(p, q, 48, -4.0, 4.0, "walls in y, uniform mesh")


def test_dilatation_pdf_uniform_flow_is_degenerate():
    nx, ny, nz = 12, 10, 9
    p = cases.params(nx=nx, ny=ny, nz=nz, lx=1.0, ly=1.0, lz=1.0)
    q = cases.uniform_state(nx, ny, nz)
    c = compare(p, q, 4, -1.0, 1.0, "uniform flow")
    assert c.tolist() == [0, 0, 0, nx * ny * nz, 0, 0]


def test_dilatation_pdf_isotropic_256_full_size():
    n = 256
    p = cases.isotropic_params(n, 1.0)
    q = cases.isotropic_state(n, 1, 1.0)
    vel = potential_velocity(n, n, n, (p["lx"], p["ly"], p["lz"]), seed=11, amp=0.2)
    ke0 = 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]
    for a in range(3):
        q[1 + a] += q[0] * vel[a]
    q[4] += 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0] - ke0
    del vel, ke0
    c = compare(p, q, 160, -8.0, 8.0, "isotropic 256^3 + potential part")
    # bins of width 0.1 from -8: the first 50 lie below -3 (shocklets), those from
    # 100 on at or above 2 (strong expansion)
    announce(f"  cells with r < -3: {int(c[:51].sum())}, r >= 2: {int(c[101:].sum())}")


def test_dilatation_pdf_errors_through_the_c_abi():
    nx, ny, nz = 12, 10, 9
    p = cases.params(nx=nx, ny=ny, nz=nz, lx=1.0, ly=1.0, lz=1.0)
    qd = torch.from_numpy(cases.uniform_state(nx, ny, nz)).to(dev())
    s = hgks.Solver(p, qd)
    L = hgks.load()
    counts = np.zeros(hgks.PDF_MAX_BINS + 3, dtype=np.int64)
    cp = counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rms = ctypes.c_double()
    try:
        for nb, lo, hi in [(0, -1.0, 1.0), (hgks.PDF_MAX_BINS + 1, -1.0, 1.0), (4, 1.0, 1.0), (4, 2.0, 1.0),
                           (4, float("nan"), 1.0), (4, -1.0, float("inf")), (4, -1e308, 1e308)]:
            assert L.hgks_dilatation_pdf(s._h, nb, lo, hi, cp, ctypes.byref(rms)) == hgks.HGKS_E_INVALID_ARG
        assert L.hgks_dilatation_pdf(s._h, 4, -1.0, 1.0, None, ctypes.byref(rms)) == hgks.HGKS_E_INVALID_ARG
    finally:
        s.close()
    pc = cases.channel_params(16, 16, 16)
    qc = torch.from_numpy(cases.channel_state(pc)).to(dev())
    sc = hgks.Solver(pc, qc)
    try:
        with pytest.raises(hgks.HgksError) as e:
            sc.dilatation_pdf(8, -1.0, 1.0)
        assert e.value.status == hgks.HGKS_E_UNSUPPORTED
    finally:
        sc.close()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_dilatation_slices_match_oracle(axis):
    """theta / theta_rms on the first, a middle and the last plane of each axis
    (the slices of the contour figure of Sec. 3.4), element by element against
    the oracle's per-cell dilatation divided by its rms, on a ragged periodic
    box and a walled uniform-mesh box (whose y-planes 0 and ny-1 touch the
    walls)."""
    boxes = []
    nx, ny, nz = 20, 14, 11
    L = (1.0 * nx / 16, 1.5 * ny / 16, 0.8 * nz / 16)
    boxes.append((cases.params(nx=nx, ny=ny, nz=nz, lx=L[0], ly=L[1], lz=L[2]), random_state(nx, ny, nz, L, seed=31)))
    pw = cases.channel_params(24, 18, 16, stretch_b=0.0, ly=2.0)
    boxes.append((pw, random_state(24, 18, 16, (pw["lx"], pw["ly"], pw["lz"]), seed=32)))
    for p, q in boxes:
        n = [p["nx"], p["ny"], p["nz"]]
        th = oracle.dilatation(p, q)  # [nz][ny][nx]
        rms = float(np.sqrt(np.mean(th * th)))
        s = hgks.Solver(p, torch.from_numpy(np.ascontiguousarray(q)).to(dev()))
        try:
            for index in (0, n[axis] // 2, n[axis] - 1):
                got, rms_gpu = s.dilatation_slice(axis, index)
                ref = (th[:, :, index] if axis == 0 else th[:, index, :] if axis == 1 else th[index]) / rms
                err = np.abs(got - ref).max() / np.abs(ref).max()
                announce(f"slice axis {axis} index {index} of {n}: max error {err:.1e}")
                assert abs(rms_gpu - rms) <= 1e-12 * rms
                assert err <= 1e-12
        finally:
            s.close()


def test_dilatation_slice_argument_checks():
    p = cases.params(nx=8, ny=7, nz=6, lx=1.0, ly=1.0, lz=1.0)
    s = hgks.Solver(p, torch.from_numpy(cases.uniform_state(8, 7, 6)).to(dev()))
    L = hgks.load()
    out = np.zeros(8 * 8)
    op = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rms = ctypes.c_double()
    try:
        for axis, index in [(-1, 0), (3, 0), (0, 8), (1, 7), (2, 6), (2, -1)]:
            assert L.hgks_dilatation_slice(s._h, axis, index, op, ctypes.byref(rms)) == hgks.HGKS_E_INVALID_ARG
        plane, r = s.dilatation_slice(2, 5)
        assert plane.shape == (7, 8) and r == 0.0 and np.all(plane == 0.0)
    finally:
        s.close()
    pc = cases.channel_params(16, 16, 16)
    sc = hgks.Solver(pc, torch.from_numpy(cases.channel_state(pc)).to(dev()))
    try:
        with pytest.raises(hgks.HgksError) as e:
            sc.dilatation_slice(1, 0)
        assert e.value.status == hgks.HGKS_E_UNSUPPORTED
    finally:
        sc.close()
