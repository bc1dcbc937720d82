"""Python binding of the SYK library: the C calls of include/syk.h with torch
tensors for device memory and streams.  Argument marshalling only; every step
of the computation runs in the HIP library.

States are complex torch tensors on the GPU, shape [dim] (one vector) or
[nvec, dim] (a block of nvec states, each row one state, as the library expects).
Calls that take `sector` (0 or 1) work on fermion-parity-sector states of
dim // 2 entries instead (see syk.h: entry u is the full row u + 2^(M-1)
(parity(u) ^ sector)).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import ChebOpts, KrylovOpts, check, lib


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.complex128:
        return _lib.SYK_C128
    if t.dtype == torch.complex64:
        return _lib.SYK_C64
    raise TypeError(f"states must be complex128 or complex64, got {t.dtype}")


def _nvec(t: torch.Tensor) -> int:
    if t.dim() == 1:
        return 1
    if t.dim() == 2:
        return int(t.shape[0])
    raise ValueError("states must have shape [dim] or [nvec, dim]")


def _check_state(t: torch.Tensor, dim: int, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dim() not in (1, 2) or t.shape[-1] != dim:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [{dim}] or [nvec, {dim}]")


def _sdim(terms, sector):
    if sector is None:
        return terms.dim
    if sector not in (0, 1):
        raise ValueError("sector must be 0, 1 or None")
    return terms.dim // 2


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _real_arr(real_of_col, nvec):
    if real_of_col is None:
        return None, None
    a = np.ascontiguousarray(real_of_col, dtype=np.int32)
    if a.shape != (nvec,):
        raise ValueError("real_of_col must have one entry per column")
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _opts(m, dt, tau_step, tol):
    return KrylovOpts(int(m), float(dt), float(tau_step), float(tol))


class Terms:
    """Hamiltonian handle (syk_build_terms): N Majoranas, one or more coupling
    realisations J of shape [C(N,4)] or [n_real, C(N,4)] (FP64, lexicographic)."""

    def __init__(self, N: int, J):
        J = np.ascontiguousarray(J, dtype=np.float64)
        n_real = 1 if J.ndim == 1 else J.shape[0]
        h = ctypes.c_void_p()
        check(lib().syk_build_terms(int(N), int(n_real), J.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)),
              "syk_build_terms")
        self._h = h
        self.N = N
        self.n_real = n_real
        Nn, nr = ctypes.c_int(), ctypes.c_int()
        d, nt, nm = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(lib().syk_terms_info(h, ctypes.byref(Nn), ctypes.byref(nr), ctypes.byref(d), ctypes.byref(nt),
                                   ctypes.byref(nm)), "syk_terms_info")
        self.dim, self.n_terms, self.n_masks = d.value, nt.value, nm.value

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("Terms handle already closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().syk_destroy_terms(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_apply_tuning(terms: Terms, tile_bits: int = 0, xcd_remap: int = 1, cols_per_group: int = 0):
    """Launch shape of apply_H for this handle (0 = automatic); see syk_set_apply_tuning."""
    check(lib().syk_set_apply_tuning(terms.handle, int(tile_bits), int(xcd_remap), int(cols_per_group)),
          "syk_set_apply_tuning")


def set_workspace_limit(terms: Terms, nbytes: int):
    """Cap on the handle's device workspace in bytes (0 = none); see syk_set_workspace_limit."""
    check(lib().syk_set_workspace_limit(terms.handle, int(nbytes)), "syk_set_workspace_limit")


def timing_enable(on: bool = True):
    check(lib().syk_timing_enable(1 if on else 0), "syk_timing_enable")


def timing_reset():
    check(lib().syk_timing_reset(), "syk_timing_reset")


def timing_read():
    """(number of timed apply_H calls, summed milliseconds) since the last reset."""
    n, ms = ctypes.c_int64(), ctypes.c_double()
    check(lib().syk_timing_read(ctypes.byref(n), ctypes.byref(ms)), "syk_timing_read")
    return n.value, ms.value


def build_terms(N: int, J) -> Terms:
    return Terms(N, J)


def apply_H(terms: Terms, psi: torch.Tensor, out: torch.Tensor | None = None, real_of_col=None,
            sector: int | None = None) -> torch.Tensor:
    d = _sdim(terms, sector)
    _check_state(psi, d, "psi")
    nvec = _nvec(psi)
    if out is None:
        out = torch.empty_like(psi)
    _check_state(out, d, "out")
    ra, rp = _real_arr(real_of_col, nvec)
    args = (ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(out.data_ptr()), _stream())
    if sector is None:
        check(lib().syk_apply_H(terms.handle, _dtype_code(psi), nvec, rp, *args), "syk_apply_H")
    else:
        check(lib().syk_apply_H_sector(terms.handle, _dtype_code(psi), int(sector), nvec, rp, *args),
              "syk_apply_H_sector")
    return out


def apply_H_noalloc(terms: Terms, psi: torch.Tensor, out: torch.Tensor, real_of_col=None) -> torch.Tensor:
    """out = H psi with no device allocation (syk_apply_H_noalloc); out must be given."""
    _check_state(psi, terms.dim, "psi")
    _check_state(out, terms.dim, "out")
    nvec = _nvec(psi)
    ra, rp = _real_arr(real_of_col, nvec)
    check(lib().syk_apply_H_noalloc(terms.handle, _dtype_code(psi), nvec, rp, ctypes.c_void_p(psi.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), _stream()), "syk_apply_H_noalloc")
    return out


def apply_majorana(terms: Terms, a: int, psi: torch.Tensor, out: torch.Tensor | None = None,
                   sector: int | None = None) -> torch.Tensor:
    """chi_a psi; with `sector` psi is a state of that sector and the result one of the other."""
    _check_state(psi, _sdim(terms, sector), "psi")
    if out is None:
        out = torch.empty_like(psi)
    args = (_nvec(psi), ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(out.data_ptr()), _stream())
    if sector is None:
        check(lib().syk_apply_majorana(terms.handle, _dtype_code(psi), int(a), *args), "syk_apply_majorana")
    else:
        check(lib().syk_apply_majorana_sector(terms.handle, _dtype_code(psi), int(a), int(sector), *args),
              "syk_apply_majorana_sector")
    return out


def dot(a: torch.Tensor, b: torch.Tensor) -> np.ndarray:
    """Column-wise <a|b> (FP64 accumulation), complex numpy array [nvec]."""
    if a.shape != b.shape or a.dtype != b.dtype:
        raise ValueError("a and b must have equal shape and dtype")
    nvec = _nvec(a)
    out = np.empty(2 * nvec, dtype=np.float64)
    check(lib().syk_dot(_dtype_code(a), int(a.shape[-1]), nvec, ctypes.c_void_p(a.data_ptr()),
                        ctypes.c_void_p(b.data_ptr()), out.ctypes.data_as(ctypes.c_void_p), _stream()), "syk_dot")
    return out[0::2] + 1j * out[1::2]


def krylov_expmv(terms: Terms, psi: torch.Tensor, z: complex, total: float, m: int = 20, dt: float = 0.1,
                 tau_step: float = 0.1, tol: float = 0.0, real_of_col=None, sector: int | None = None) -> np.ndarray:
    """psi <- exp(total * z * H) psi in place; returns the per-column error estimate."""
    _check_state(psi, _sdim(terms, sector), "psi")
    nvec = _nvec(psi)
    ra, rp = _real_arr(real_of_col, nvec)
    err = np.zeros(nvec)
    o = _opts(m, dt, tau_step, tol)
    tail = (float(np.real(z)), float(np.imag(z)), float(total), ctypes.byref(o), ctypes.c_void_p(psi.data_ptr()),
            err.ctypes.data_as(ctypes.c_void_p), _stream())
    if sector is None:
        check(lib().syk_krylov_expmv(terms.handle, _dtype_code(psi), nvec, rp, *tail), "syk_krylov_expmv")
    else:
        check(lib().syk_krylov_expmv_sector(terms.handle, _dtype_code(psi), int(sector), nvec, rp, *tail),
              "syk_krylov_expmv_sector")
    return err


def _call(name: str, terms: Terms, psi: torch.Tensor, sector, *rest):
    """lib().name(handle, dtype, *rest), or name_sector with the sector after the dtype."""
    if sector is None:
        check(getattr(lib(), name)(terms.handle, _dtype_code(psi), *rest), name)
    else:
        check(getattr(lib(), name + "_sector")(terms.handle, _dtype_code(psi), int(sector), *rest), name + "_sector")


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def two_point(terms: Terms, i: int, beta: float, times, psi0: torch.Tensor, m: int = 20, dt: float = 0.1,
              tau_step: float = 0.1, real_of_col=None, sector: int | None = None):
    """G(t) (complex [nt, nvec]) and Z ([nvec]); see syk_two_point."""
    _check_state(psi0, _sdim(terms, sector), "psi0")
    nvec = _nvec(psi0)
    t = np.ascontiguousarray(times, dtype=np.float64)
    G = np.empty((t.size, nvec, 2))
    Z = np.empty(nvec)
    ra, rp = _real_arr(real_of_col, nvec)
    o = _opts(m, dt, tau_step, 0.0)
    _call("syk_two_point", terms, psi0, sector, int(i), float(beta), _ptr(t), t.size, nvec, rp,
          ctypes.c_void_p(psi0.data_ptr()), ctypes.byref(o), _ptr(G), _ptr(Z), _stream())
    return G[..., 0] + 1j * G[..., 1], Z


def otoc(terms: Terms, i: int, j: int, beta: float, times, psi0: torch.Tensor, m: int = 20, dt: float = 0.1,
         tau_step: float = 0.1, tol: float = 0.0, real_of_col=None, sector: int | None = None):
    """F(t) ([nt, nvec]), Im part ([nt, nvec]) and Z ([nvec]); see syk_otoc."""
    _check_state(psi0, _sdim(terms, sector), "psi0")
    nvec = _nvec(psi0)
    t = np.ascontiguousarray(times, dtype=np.float64)
    F = np.empty((t.size, nvec))
    Fi = np.empty((t.size, nvec))
    Z = np.empty(nvec)
    ra, rp = _real_arr(real_of_col, nvec)
    o = _opts(m, dt, tau_step, tol)
    _call("syk_otoc", terms, psi0, sector, int(i), int(j), float(beta), _ptr(t), t.size, nvec, rp,
          ctypes.c_void_p(psi0.data_ptr()), ctypes.byref(o), _ptr(F), _ptr(Fi), _ptr(Z), _stream())
    return F, Fi, Z


def otoc_unregularized(terms: Terms, i: int, j: int, beta: float, times, psi0: torch.Tensor, m: int = 20,
                       dt: float = 0.1, tau_step: float = 0.1, tol: float = 0.0, real_of_col=None,
                       sector: int | None = None):
    """Unregularized OTOC: Re F_u ([nt, nvec]), Im F_u ([nt, nvec]) and Z ([nvec]);
    see syk_otoc_unregularized."""
    _check_state(psi0, _sdim(terms, sector), "psi0")
    nvec = _nvec(psi0)
    t = np.ascontiguousarray(times, dtype=np.float64)
    F = np.empty((t.size, nvec))
    Fi = np.empty((t.size, nvec))
    Z = np.empty(nvec)
    ra, rp = _real_arr(real_of_col, nvec)
    o = _opts(m, dt, tau_step, tol)
    _call("syk_otoc_unregularized", terms, psi0, sector, int(i), int(j), float(beta), _ptr(t), t.size, nvec, rp,
          ctypes.c_void_p(psi0.data_ptr()), ctypes.byref(o), _ptr(F), _ptr(Fi), _ptr(Z), _stream())
    return F, Fi, Z


def imag_two_point(terms: Terms, i: int, beta: float, taus, psi0: torch.Tensor, m: int = 20, tau_step: float = 0.1,
                   real_of_col=None, sector: int | None = None):
    """G(tau) ([ntau, nvec], real) and Z ([nvec]); see syk_imag_two_point."""
    _check_state(psi0, _sdim(terms, sector), "psi0")
    nvec = _nvec(psi0)
    tau = np.ascontiguousarray(taus, dtype=np.float64)
    G = np.empty((tau.size, nvec))
    Z = np.empty(nvec)
    ra, rp = _real_arr(real_of_col, nvec)
    o = _opts(m, 0.1, tau_step, 0.0)
    _call("syk_imag_two_point", terms, psi0, sector, int(i), float(beta), _ptr(tau), tau.size, nvec, rp,
          ctypes.c_void_p(psi0.data_ptr()), ctypes.byref(o), _ptr(G), _ptr(Z), _stream())
    return G, Z


def spectrum_bounds(terms: Terms, psi0: torch.Tensor, m: int = 40):
    """(e_min, e_max): extreme Ritz values of m Lanczos steps from psi0."""
    _check_state(psi0, terms.dim, "psi0")
    lo, hi = ctypes.c_double(), ctypes.c_double()
    check(lib().syk_spectrum_bounds(terms.handle, _dtype_code(psi0), int(m), ctypes.c_void_p(psi0.data_ptr()),
                                    ctypes.byref(lo), ctypes.byref(hi), _stream()), "syk_spectrum_bounds")
    return lo.value, hi.value


def lowest_eigenvalues(terms: Terms, psi0: torch.Tensor, k: int = 20, m: int = 200):
    """(Ritz values, residual norms): the k lowest of m Lanczos steps from psi0
    (numpy arrays of length <= k); see syk_lowest_eigenvalues."""
    _check_state(psi0, terms.dim, "psi0")
    if psi0.dim() != 1:
        raise ValueError("eigenvalues take one state")
    ev = np.empty(k)
    res = np.empty(k)
    n = ctypes.c_int()
    check(lib().syk_lowest_eigenvalues(terms.handle, _dtype_code(psi0), int(m), int(k),
                                       ctypes.c_void_p(psi0.data_ptr()), ev.ctypes.data_as(ctypes.c_void_p),
                                       res.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n), _stream()),
          "syk_lowest_eigenvalues")
    return ev[:n.value].copy(), res[:n.value].copy()


def cheb_opts(degree: int = 32, dt: float = 0.1, tau_steps: int = 1, checkpoint_every: int = 10,
              e_center: float = 0.0, e_halfwidth: float = 1.0, keep_segment: bool = True) -> ChebOpts:
    """Options of the Chebyshev forward and its reverse sweep (syk_cheb_opts)."""
    return ChebOpts(int(degree), float(dt), int(tau_steps), int(checkpoint_every), float(e_center),
                    float(e_halfwidth), 1 if keep_segment else 0)


def cheb_otoc(terms: Terms, i: int, j: int, beta: float, t_star: float, psi0: torch.Tensor, opts: ChebOpts) -> float:
    """F(t_star) with Chebyshev propagators (syk_cheb_otoc); complex128 psi0 [dim]."""
    _check_state(psi0, terms.dim, "psi0")
    if psi0.dtype != torch.complex128 or psi0.dim() != 1:
        raise ValueError("the Chebyshev OTOC takes one complex128 state")
    F = ctypes.c_double()
    check(lib().syk_cheb_otoc(terms.handle, int(i), int(j), float(beta), float(t_star), ctypes.byref(opts),
                              ctypes.c_void_p(psi0.data_ptr()), ctypes.byref(F), _stream()), "syk_cheb_otoc")
    return F.value


def coupling_overlaps(terms: Terms, pairs):
    """sum_p w_p Re <g_p| dH/dJ_n |v_p> for every coupling n, as a numpy array of
    C(N,4) (syk_coupling_overlaps).  pairs: up to 64 (g, v, w) with g, v
    complex128 full-space states on the device."""
    pairs = list(pairs)
    if not 1 <= len(pairs) <= 64:
        raise ValueError("need 1 to 64 pairs")
    for g, v, _ in pairs:
        for x, name in ((g, "g"), (v, "v")):
            _check_state(x, terms.dim, name)
            if x.dtype != torch.complex128 or x.dim() != 1:
                raise ValueError(f"{name}: one complex128 state per pair")
    n = len(pairs)
    gp = (ctypes.c_void_p * n)(*[g.data_ptr() for g, _, _ in pairs])
    vp = (ctypes.c_void_p * n)(*[v.data_ptr() for _, v, _ in pairs])
    w = np.array([float(x) for _, _, x in pairs], dtype=np.float64)
    out = np.empty(terms.n_terms, dtype=np.float64)
    check(lib().syk_coupling_overlaps(terms.handle, n, ctypes.cast(gp, ctypes.c_void_p), ctypes.cast(vp, ctypes.c_void_p),
                                      _ptr(w), _ptr(out), _stream()), "syk_coupling_overlaps")
    return out


def grad_couplings(terms: Terms, i: int, j: int, beta: float, t_star: float, psi0: torch.Tensor, opts: ChebOpts):
    """(F, dF/dJ as a numpy array of C(N,4)) by the reverse sweep (syk_grad_couplings)."""
    _check_state(psi0, terms.dim, "psi0")
    if psi0.dtype != torch.complex128 or psi0.dim() != 1:
        raise ValueError("the gradient takes one complex128 state")
    F = ctypes.c_double()
    g = np.empty(terms.n_terms, dtype=np.float64)
    check(lib().syk_grad_couplings(terms.handle, int(i), int(j), float(beta), float(t_star), ctypes.byref(opts),
                                   ctypes.c_void_p(psi0.data_ptr()), ctypes.byref(F),
                                   g.ctypes.data_as(ctypes.c_void_p), _stream()), "syk_grad_couplings")
    return F.value, g
