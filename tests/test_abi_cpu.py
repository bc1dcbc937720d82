"""C-ABI checks that need no GPU: the library loads, exports every function
include/syk.h declares, and rejects invalid arguments before touching HIP."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2002_05725_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(syk_\w+)\s*\(", txt):
            names.add(m.group(1))
    return names


def test_header_declares_functions():
    assert {"syk_build_terms", "syk_apply_H", "syk_krylov_expmv", "syk_otoc"} <= _declared()


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in sorted(_declared()):
        assert hasattr(L, name), f"{name} declared in include/ but not exported"


def test_binding_covers_header():
    assert set(_lib.declared_symbols()) == _declared()


def test_version():
    assert _lib.lib().syk_version() >= 100


def _build(N, n_real, J):
    h = ctypes.c_void_p()
    p = None if J is None else J.ctypes.data_as(ctypes.c_void_p)
    return _lib.lib().syk_build_terms(N, n_real, p, ctypes.byref(h)), h


@pytest.mark.parametrize("N", [3, 2, 62, 0])
def test_build_rejects_bad_N(N):
    st, h = _build(N, 1, np.zeros(10))
    assert st == _lib.SYK_EINVAL and not h.value
    assert b"N must be even" in _lib.lib().syk_last_error()


def test_build_rejects_bad_arguments():
    assert _build(8, 0, np.zeros(70))[0] == _lib.SYK_EINVAL
    assert _build(8, 1, None)[0] == _lib.SYK_EINVAL
    J = np.zeros(70)
    J[5] = np.nan
    assert _build(8, 1, J)[0] == _lib.SYK_EINVAL
    assert b"non-finite" in _lib.lib().syk_last_error()


def test_calls_reject_null_handle():
    L = _lib.lib()
    assert L.syk_apply_H(None, 0, 1, None, None, None, None) == _lib.SYK_EINVAL
    assert L.syk_terms_info(None, None, None, None, None, None) == _lib.SYK_EINVAL
    assert L.syk_destroy_terms(None) == _lib.SYK_OK
    o = _lib.KrylovOpts(20, 0.1, 0.1, 0.0)
    assert L.syk_otoc(None, 0, 0, 1, 1.0, None, 1, 1, None, None, ctypes.byref(o), None, None, None,
                      None) == _lib.SYK_EINVAL
    w = np.ones(1)
    out = np.zeros(4)
    assert L.syk_coupling_overlaps(None, 1, None, None, w.ctypes.data_as(ctypes.c_void_p),
                                   out.ctypes.data_as(ctypes.c_void_p), None) == _lib.SYK_EINVAL
    assert b"handle" in L.syk_last_error()
    c = _lib.ChebOpts(16, 0.1, 1, 4, 0.0, 2.0, 1)
    F = ctypes.c_double()
    assert L.syk_grad_couplings(None, 0, 1, 1.0, 0.2, ctypes.byref(c), None, ctypes.byref(F), None,
                                None) == _lib.SYK_EINVAL


def test_dot_rejects_bad_arguments():
    L = _lib.lib()
    out = np.zeros(2)
    assert L.syk_dot(0, 0, 1, None, None, out.ctypes.data_as(ctypes.c_void_p), None) == _lib.SYK_EINVAL
    assert L.syk_dot(7, 16, 1, None, None, out.ctypes.data_as(ctypes.c_void_p), None) == _lib.SYK_EINVAL
