"""syk_apply_H_noalloc, the apply_H entry point that allocates nothing (its
rotated-layout buffers live in a device scratch array built into the library),
against syk_apply_H through the C-ABI: the same kernels on the same inputs give
the same bits.  Two calls in a row on one device share the scratch, the second
with a smaller input; requests beyond the scratch and handles without tables
are rejected."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2002_05725_amd import _lib, api, inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(msg):
    print(f"[no-alloc] {msg}", file=sys.stderr, flush=True)


def _states(N, seeds, dtype):
    x = np.stack([inputs.typical_state(N, s) for s in seeds])
    return torch.from_numpy(x).to(DEV).to(dtype).contiguous()


def _raw(T, psi, out, real=None):
    nvec = psi.shape[0]
    r = None if real is None else np.ascontiguousarray(real, dtype=np.int32)
    rp = None if r is None else r.ctypes.data_as(ctypes.c_void_p)
    code = _lib.SYK_C128 if psi.dtype == torch.complex128 else _lib.SYK_C64
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return _lib.lib().syk_apply_H_noalloc(T.handle, code, nvec, rp, ctypes.c_void_p(psi.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), st)


def test_noalloc_equals_apply_two_calls_in_a_row():
    """N = 40 (two row layouts, complex128, two columns of two realisations),
    then N = 32 (one column, complex64): each against syk_apply_H on the same
    handle and inputs, bit for bit; the second call reuses the scratch the
    first filled with larger data."""
    cases = [(40, torch.complex128, [5, 6], [0, 1]), (32, torch.complex64, [7], None)]
    for N, dt, seeds, real in cases:
        _say(f"N={N} {dt} nvec={len(seeds)}")
        Js = np.stack([inputs.couplings(N, 90 + r) for r in range(2)])
        T = api.Terms(N, Js)
        psi = _states(N, seeds, dt)
        ref = api.apply_H(T, psi, real_of_col=real)          # also builds the handle's tables
        torch.cuda.synchronize()
        out = torch.full_like(psi, complex(float("nan"), float("nan")))
        assert _raw(T, psi, out, real) == _lib.SYK_OK, _lib.lib().syk_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        # the Python binding of the same entry point
        out2 = torch.zeros_like(psi)
        api.apply_H_noalloc(T, psi, out2, real_of_col=real)
        assert torch.equal(out2, ref)
        T.close()


def test_noalloc_two_columns_per_workgroup():
    """A complex64 block whose columns pair up by realisation runs two
    columns per workgroup (the automatic shape): the allocation-free call
    gives syk_apply_H's bits there too, at N = 36 (two row layouts)."""
    N = 36
    _say(f"N={N} complex64 nvec=4 paired")
    Js = np.stack([inputs.couplings(N, 95 + r) for r in range(2)])
    T = api.Terms(N, Js)
    psi = _states(N, [11, 12, 13, 14], torch.complex64)
    real = [1, 1, 0, 0]
    ref = api.apply_H(T, psi, real_of_col=real)
    torch.cuda.synchronize()
    out = torch.full_like(psi, complex(float("nan"), float("nan")))
    assert _raw(T, psi, out, real) == _lib.SYK_OK, _lib.lib().syk_last_error()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    T.close()


def test_noalloc_rejects_what_it_cannot_serve():
    # a handle that never ran syk_apply_H has no tables
    N = 36
    T = api.Terms(N, inputs.couplings(N, 0))
    psi = _states(N, [1], torch.complex128)
    out = torch.empty_like(psi)
    assert _raw(T, psi, out) == _lib.SYK_EINVAL
    assert b"tables" in _lib.lib().syk_last_error()
    # overlapping buffers
    assert _raw(T, psi, psi) == _lib.SYK_EINVAL
    T.close()
    # N = 46 complex128: 2 x 128 MiB of rotated buffers, above the 128 MiB scratch
    N = 46
    T = api.Terms(N, inputs.couplings(N, 0))
    psi = torch.zeros(1 << (N // 2), dtype=torch.complex128, device=DEV)
    psi[3] = 1.0
    api.apply_H(T, psi)
    out = torch.empty_like(psi)
    assert _raw(T, psi.view(1, -1), out.view(1, -1)) == _lib.SYK_EINVAL
    assert b"scratch" in _lib.lib().syk_last_error()
    T.close()
