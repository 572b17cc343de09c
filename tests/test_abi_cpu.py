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
    from paper_1312_6182_amd import serve as SV
    assert set(_declared_functions()) == set(L.SIGNATURES) | set(SV.SIGNATURES)


def test_reduced_precision_and_server_validation():
    """Argument checks of the quantizer, refinement and server entry points
    (all rejected on the host, before any HIP call)."""
    from paper_1312_6182_amd import serve as SV
    lib = SV._lib()
    buf = (ctypes.c_float * 64)()
    M = L.Matrix()
    M.data = ctypes.addressof(buf)
    M.p, M.n, M.lda, M.dtype = 4, 4, 4, L.F32
    out = (ctypes.c_uint8 * 64)()
    assert lib.gpspca_quantize(ctypes.byref(M), L.F32, ctypes.addressof(out), 4, None, None) == L.EDTYPE
    assert lib.gpspca_quantize(ctypes.byref(M), L.F8E4M3, ctypes.addressof(out), 4, None, None) == L.EINVAL
    assert lib.gpspca_quantize(ctypes.byref(M), L.BF16, ctypes.addressof(out), 3, None, None) == L.EINVAL
    # BF16 storage needs lda % 8 == 0; F8E4M3 needs a scale
    Mq = L.Matrix()
    Mq.data = ctypes.addressof(out) + (-ctypes.addressof(out)) % 16
    Mq.p, Mq.n, Mq.lda, Mq.dtype = 4, 4, 4, L.BF16
    assert lib.gpspca_workspace_bytes(ctypes.byref(Mq), L.SL1, 1, 10) == 0
    Mq.dtype, Mq.lda = L.F8E4M3, 16
    assert lib.gpspca_workspace_bytes(ctypes.byref(Mq), L.SL1, 1, 10) == 0
    assert "col_scale" in L.last_error()
    # F32 storage takes no scale
    M.col_scale = ctypes.addressof(buf)
    assert lib.gpspca_workspace_bytes(ctypes.byref(M), L.SL1, 1, 10) == 0
    M.col_scale = None
    # refinement needs a support and a start
    x = (ctypes.c_float * 4)()
    sup = (ctypes.c_uint32 * 4)()
    nit = ctypes.c_int(0)
    ws = (ctypes.c_uint8 * 1024)()
    wsp = ctypes.addressof(ws) + (-ctypes.addressof(ws)) % 256
    assert lib.gpspca_refine(ctypes.byref(M), L.SL1, 1, 0.1, None, None, ctypes.addressof(x), 0.0,
                             5, wsp, 512, None, ctypes.addressof(x), None, None, None,
                             ctypes.byref(nit)) == L.EINVAL
    assert lib.gpspca_refine(ctypes.byref(M), L.SL1, 1, 0.1, None, ctypes.addressof(sup), None,
                             0.0, 5, wsp, 512, None, ctypes.addressof(x), None, None, None,
                             ctypes.byref(nit)) == L.EINVAL
    # server: arena and slots are checked first
    h = ctypes.c_void_p()
    assert lib.gpspca_server_create(None, 1 << 30, 2, ctypes.byref(h)) == L.EINVAL
    assert lib.gpspca_server_create(wsp, 1 << 30, 0, ctypes.byref(h)) == L.EINVAL
    assert lib.gpspca_server_create(wsp, 1 << 20, 2, ctypes.byref(h)) == L.ENOMEM
    assert not h.value


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
