"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/gpspca.h, and rejects invalid arguments on the host before
any HIP call (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_1312_6182_amd as G
from paper_1312_6182_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpspca.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(gpspca_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = _declared_functions()
    for n in ("gpspca_solve", "gpspca_step", "gpspca_workspace_bytes", "gpspca_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = G.load()
    for name in _declared_functions():
        assert hasattr(lib, name), f"{name} declared in gpspca.h but not exported"


def test_binding_covers_every_declared_symbol():
    assert set(_declared_functions()) == set(L.SIGNATURES)


def test_version_string():
    assert G.load().gpspca_version().decode().startswith("gpspca-gfx950")


def _mat(p=10, n=20, lda=None, dtype=L.F32, data=0x1000):
    M = L.Matrix()
    M.data = data
    M.p, M.n, M.lda = p, n, (p if lda is None else lda)
    M.dtype = dtype
    M.col_scale = None
    return M


def _solve(M, form=0, m=1, gamma=0.1, mu=None, tol=1e-4, max_iter=10, ws=0x2000, X=0x3000):
    lib = G.load()
    mu_arr = None if mu is None else (ctypes.c_double * len(mu))(*mu)
    return lib.gpspca_solve(ctypes.byref(M) if M is not None else None, form, m, gamma, mu_arr,
                            None, tol, max_iter, ws, 1 << 30, None, X, None, None, None, None)


@pytest.mark.parametrize("kwargs,code", [
    (dict(M=None), L.EINVAL),
    (dict(M="p0"), L.EINVAL),
    (dict(M="lda"), L.EINVAL),
    (dict(M="null"), L.EINVAL),
    (dict(form=7), L.EINVAL),
    (dict(form=L.SL1, m=2), L.EINVAL),
    (dict(form=L.BL1, m=0), L.EINVAL),
    (dict(form=L.BL1, m=11), L.EINVAL),       # m > p
    (dict(gamma=-1.0), L.EINVAL),
    (dict(gamma=float("nan")), L.EINVAL),
    (dict(form=L.BL0, m=2, mu=[1.0, 0.0]), L.EINVAL),
    (dict(form=L.BL0, m=2, mu=[1.0, float("inf")]), L.EINVAL),
    (dict(tol=-1.0), L.EINVAL),
    (dict(max_iter=0), L.EINVAL),
    (dict(X=0), L.EINVAL),
    (dict(ws=0), L.EINVAL),
    (dict(ws=0x2001), L.EINVAL),              # misaligned workspace
    (dict(M="dtype"), L.EDTYPE),
])
def test_host_validation(kwargs, code):
    special = kwargs.pop("M", "ok")
    if special is None:
        M = None
    elif special == "p0":
        M = _mat(p=0)
    elif special == "lda":
        M = _mat(p=10, lda=9)
    elif special == "null":
        M = _mat(data=0)
    elif special == "dtype":
        M = _mat(dtype=9)
    else:
        M = _mat()
    assert _solve(M, **kwargs) == code
    assert G.last_error() != ""


def test_step_validation():
    lib = G.load()
    M = _mat()
    rc = lib.gpspca_step(ctypes.byref(M), L.SL0, 1, 0.5, None, None, 0x2000, 1 << 20, None,
                         None, None, None, None)
    assert rc == L.EINVAL


def test_m_above_max_rejected():
    M = _mat(p=100, n=200)
    assert _solve(M, form=L.BL1, m=L.MAX_M + 1) == L.EINVAL
