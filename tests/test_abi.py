"""CPU checks of the C ABI: the HIP library loads and exports every function the
header declares; parameter validation that runs without a device."""
import os
import re

import pytest

from paper_2005_08736_amd import cases, hgks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(hgks_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = hgks.load()
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(hgks.EXPORTED) <= set(names)


def test_workspace_size_and_validation():
    p = cases.tgv_params(32)
    ws = hgks.workspace_bytes(p)
    assert ws >= 40 * 8 * 32 ** 3
    assert ws % 256 == 0
    # boxes of 2^31 cells and more are rejected: the launch grids count cells in 32 bits
    big = dict(p)
    big.update(nx=2048, ny=1024, nz=1023)
    assert hgks.workspace_bytes(big) >= 360 * 2048 * 1024 * 1023  # 45 doubles per cell besides the state
    for bad in (dict(nx=5), dict(gamma=1.0), dict(cfl=0.0), dict(prandtl=-1.0), dict(mode=7), dict(mu_ref=-1.0),
                dict(nx=2048, ny=2048, nz=512)):
        q = dict(p)
        q.update(bad)
        assert hgks.workspace_bytes(q) == 0, bad


def test_strerror_covers_codes():
    for code in (0, -1, -2, -3, -4, -5):
        assert hgks.strerror(code) != "unknown status"


def test_params_struct_matches_header_field_order():
    src = open(os.path.join(ROOT, "include", "hgks.h")).read()
    body = src[src.index("typedef struct {"):src.index("} hgks_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    decl = []
    for line in body.splitlines()[1:]:
        line = line.strip().rstrip(";")
        if not line:
            continue
        typ, rest = line.split(None, 1)
        decl += [(n.strip(), typ) for n in rest.split(",")]
    fields = [(n, "int32_t" if t.__name__ == "c_int" else "double") for n, t in hgks.HgksParams._fields_]
    assert [d[0] for d in decl] == [f[0] for f in fields]
    assert [d[1] for d in decl] == [f[1] for f in fields]


def test_init_rejects_missing_small_or_misaligned_workspace():
    """hgks_init checks the workspace before it touches the device: a NULL
    workspace, one byte too few and a pointer off the 256-byte alignment all
    return HGKS_E_WORKSPACE (the pointers are never dereferenced)."""
    import ctypes

    lib = hgks.load()
    p = cases.tgv_params(8)
    prm = hgks.make_params(p)
    need = hgks.workspace_bytes(p)
    fake_q = ctypes.c_void_p(1 << 20)
    h = ctypes.c_void_p()
    cases_ = [
        (None, need),
        (ctypes.c_void_p(1 << 21), need - 1),
        (ctypes.c_void_p((1 << 21) + 128), need),
        (ctypes.c_void_p((1 << 21) + 8), need + 256),
    ]
    for ws, nbytes in cases_:
        rc = lib.hgks_init(ctypes.byref(prm), fake_q, ws, nbytes, None, ctypes.byref(h))
        assert rc == hgks.HGKS_E_WORKSPACE, (ws, nbytes, rc)
        assert not h.value
    # invalid parameters are reported before the workspace
    bad = dict(p, nx=5)
    rc = lib.hgks_init(ctypes.byref(hgks.make_params(bad)), fake_q, None, 0, None, ctypes.byref(h))
    assert rc == hgks.HGKS_E_INVALID_ARG
    assert lib.hgks_init(ctypes.byref(prm), None, ctypes.c_void_p(1 << 21), need, None,
                         ctypes.byref(h)) == hgks.HGKS_E_INVALID_ARG


def test_static_step_checks_its_limit_before_the_device():
    """hgks_step_static validates the parameters and the size of its static
    workspace on the host: an oversized box returns HGKS_E_WORKSPACE and a
    negative step count HGKS_E_INVALID_ARG, without touching the device."""
    import ctypes

    lib = hgks.load()
    fake_q = ctypes.c_void_p(1 << 20)
    p = cases.tgv_params(64)
    assert hgks.workspace_bytes(p) > hgks.STATIC_WORKSPACE_BYTES
    assert lib.hgks_step_static(ctypes.byref(hgks.make_params(p)), fake_q, 1, 0.0, None,
                                None) == hgks.HGKS_E_WORKSPACE
    small = cases.tgv_params(16)
    assert hgks.workspace_bytes(small) <= hgks.STATIC_WORKSPACE_BYTES
    assert lib.hgks_step_static(ctypes.byref(hgks.make_params(small)), fake_q, -1, 0.0, None,
                                None) == hgks.HGKS_E_INVALID_ARG
    assert lib.hgks_step_static(ctypes.byref(hgks.make_params(small)), None, 1, 0.0, None,
                                None) == hgks.HGKS_E_INVALID_ARG
    assert lib.hgks_step_static(ctypes.byref(hgks.make_params(dict(small, nx=5))), fake_q, 1, 0.0, None,
                                None) == hgks.HGKS_E_INVALID_ARG
