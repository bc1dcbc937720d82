"""Two-point functions and regularized OTOCs from a typical state.

Test infrastructure only (see the package docstring).

Definitions followed:
* Main text, Eq. 2-3: G(tau), G_R(t) built from <chi_i(t) chi_i(0)>_beta,
  with <...>_beta = Tr[... e^{-beta H}] / Z.
* Main text, Eq. 4 (and the SI section "Unregularized OTOCs"): the
  regularized OTOC F(t) = <chi_i(t) rho^{1/4} chi_j rho^{1/4} chi_i(t)
  rho^{1/4} chi_j rho^{1/4}> with rho = e^{-beta H}, i != j.  The four
  rho^{1/4} factors already make up rho, so the bracket is read as
  Tr[...] / Tr[rho].
* SI, section "Disorder averaging", typicality formula: a trace against
  e^{-beta H} is replaced by an expectation in a Gaussian random state psi.
* Heisenberg picture chi(t) = e^{iHt} chi e^{-iHt}; U = e^{-iHt} moves states.

Estimator of F used here (the symmetric cut of the trace):
    A = rho^{1/8} W(t) rho^{1/4} V rho^{1/8},  W = chi_i, V = chi_j,
    F_est = Re <psi|A A|psi> / <psi|rho|psi>
          = Re <A^dag psi | A psi> / ||rho^{1/2} psi||^2,
with A psi = rho^{1/8} U^dag W U rho^{1/4} V rho^{1/8} psi and
A^dag psi = rho^{1/8} V rho^{1/4} U^dag W U rho^{1/8} psi.  Tr[A A] equals
Tr rho times Eq. 4's F, so summing the numerator over any orthonormal basis
gives the exact trace.
"""
from __future__ import annotations

import numpy as np

from .krylov import propagate


class Propagator:
    """e^{z s H} applied by Krylov steps: real-time legs with step dt, imaginary
    legs with step tau_step, m basis vectors per step."""

    def __init__(self, matvec, m: int, dt: float, tau_step: float):
        self.matvec, self.m, self.dt, self.tau_step = matvec, m, dt, tau_step

    def real(self, psi, t):          # e^{-iHt} psi  (t may be negative)
        if t == 0:
            return np.array(psi, dtype=np.complex128, copy=True)
        z = -1j if t > 0 else 1j
        return propagate(self.matvec, psi, z, abs(t), self.dt, self.m)

    def imag(self, psi, tau):        # e^{-tau H} psi
        if tau == 0:
            return np.array(psi, dtype=np.complex128, copy=True)
        return propagate(self.matvec, psi, -1.0, tau, self.tau_step, self.m)


class ExactPropagator:
    """Same interface, with exact exponentials from a dense eigendecomposition."""

    def __init__(self, dense_exp):
        self.E = dense_exp

    def real(self, psi, t):
        return self.E.apply(psi, -1j * t)

    def imag(self, psi, tau):
        return self.E.apply(psi, -tau)


def otoc_estimator(prop, maj, psi, i: int, j: int, beta: float, times):
    """F_est(t) for each t in `times` (module docstring), each time propagated
    from scratch.  `maj(a, v)` returns chi_a v.  Returns (F, F_imag, Z)."""
    a0 = prop.imag(psi, beta / 8)                      # rho^{1/8} psi
    b0 = prop.imag(maj(j, a0), beta / 4)               # rho^{1/4} V rho^{1/8} psi
    Z = float(np.linalg.norm(prop.imag(psi, beta / 2)) ** 2)   # <psi|rho|psi>
    F = np.empty(len(times))
    Fi = np.empty(len(times))
    for n, t in enumerate(times):
        x = prop.real(maj(i, prop.real(b0, t)), -t)   # U^dag W U b0
        A_psi = prop.imag(x, beta / 8)
        y = prop.real(maj(i, prop.real(a0, t)), -t)   # U^dag W U a0
        y = prop.imag(y, beta / 4)
        Adag_psi = prop.imag(maj(j, y), beta / 8)
        val = np.vdot(Adag_psi, A_psi) / Z
        F[n], Fi[n] = val.real, val.imag
    return F, Fi, Z


def otoc_trace(dense_exp, chis, i: int, j: int, beta: float, times):
    """Exact F(t) = Tr[W(t) r V r W(t) r V r] / Tr[rho], r = rho^{1/4} (Eq. 4)."""
    r = dense_exp.matrix(-beta / 4)
    Zt = float(np.trace(dense_exp.matrix(-beta)).real)
    out = np.empty(len(times))
    for n, t in enumerate(times):
        U = dense_exp.matrix(-1j * t)
        Wt = U.conj().T @ chis[i] @ U
        P = Wt @ r @ chis[j] @ r
        out[n] = float(np.trace(P @ P).real) / Zt
    return out


def two_point_beta0(prop, maj, psi, i: int, times):
    """G(t) = <psi| chi_i(t) chi_i |psi> at beta = 0 (Eq. 2-3 with the trace
    replaced by the typical state): with a = U psi and b = U chi_i psi,
    G = <a| chi_i |b>.  Complex; G_R = 2 Re G."""
    chi_psi = maj(i, psi)
    out = np.empty(len(times), dtype=np.complex128)
    for n, t in enumerate(times):
        a = prop.real(psi, t)
        b = prop.real(chi_psi, t)
        out[n] = np.vdot(a, maj(i, b))
    return out


def two_point_estimator(prop, maj, psi, i: int, beta: float, times):
    """G(t) = <chi_i(t) chi_i>_beta at any beta (Eq. 2-3) from a typical state
    (SI "Disorder averaging"), the thermal trace cut symmetrically:
        G_est(t) = <phi| chi_i(t) chi_i |phi> / <phi|phi>,  phi = rho^{1/2} psi,
    with chi_i(t) = U^dag chi_i U, so the numerator is <U phi | chi_i U chi_i phi>.
    Summed over an orthonormal basis the numerator is Tr[rho^{1/2} chi_i(t)
    chi_i rho^{1/2}] = Tr[chi_i(t) chi_i rho] and the denominator Tr rho.
    Each time is propagated from scratch.  Returns (G complex, Z = <phi|phi>);
    G_R = 2 Re G."""
    phi = prop.imag(psi, beta / 2)
    Z = float(np.vdot(phi, phi).real)
    chi_phi = maj(i, phi)
    out = np.empty(len(times), dtype=np.complex128)
    for n, t in enumerate(times):
        a = prop.real(phi, t)                 # U phi
        b = prop.real(chi_phi, t)             # U chi_i phi
        out[n] = np.vdot(a, maj(i, b)) / Z
    return out, Z


def two_point_trace(dense_exp, chis, i: int, beta: float, times):
    """Exact <chi_i(t) chi_i>_beta = Tr[chi_i(t) chi_i rho] / Tr rho."""
    rho = dense_exp.matrix(-beta)
    Zt = float(np.trace(rho).real)
    out = np.empty(len(times), dtype=np.complex128)
    for n, t in enumerate(times):
        U = dense_exp.matrix(-1j * t)
        out[n] = np.trace(U.conj().T @ chis[i] @ U @ chis[i] @ rho) / Zt
    return out


# ---------------------------------------------------------------------------
# Unregularized OTOC (SI section "Unregularized OTOCs"):
#     F_u(t) = <chi_i(t) chi_j chi_i(t) chi_j rho> = Tr[W V W V rho] / Tr rho,
# W = chi_i(t), V = chi_j.  Symmetric cut of the trace with phi = rho^{1/2} psi:
#     F_u_est = <phi| W V W V |phi> / <phi|phi> = <V W phi | W V phi> / <phi|phi>
# (W and V are Hermitian).  Complex in general; both parts are returned.
def otoc_u_estimator(prop, maj, psi, i: int, j: int, beta: float, times):
    """F_u estimate for each t (each time propagated from scratch).
    Returns (Re F_u, Im F_u, Z)."""
    phi = prop.imag(psi, beta / 2)
    Z = float(np.vdot(phi, phi).real)
    F = np.empty(len(times))
    Fi = np.empty(len(times))
    for n, t in enumerate(times):
        wv = prop.real(maj(i, prop.real(maj(j, phi), t)), -t)      # W V phi
        vw = maj(j, prop.real(maj(i, prop.real(phi, t)), -t))      # V W phi
        val = np.vdot(vw, wv) / Z
        F[n], Fi[n] = val.real, val.imag
    return F, Fi, Z


def otoc_u_trace(dense_exp, chis, i: int, j: int, beta: float, times):
    """Exact F_u(t) = Tr[W(t) V W(t) V rho] / Tr rho (complex)."""
    rho = dense_exp.matrix(-beta)
    Zt = float(np.trace(rho).real)
    out = np.empty(len(times), dtype=np.complex128)
    for n, t in enumerate(times):
        U = dense_exp.matrix(-1j * t)
        Wt = U.conj().T @ chis[i] @ U
        out[n] = np.trace(Wt @ chis[j] @ Wt @ chis[j] @ rho) / Zt
    return out


# ---------------------------------------------------------------------------
# Imaginary-time Green's function (main text Eq. 2):
#     G(tau) = <chi_i(tau) chi_i(0)>_beta,  chi(tau) = e^{tau H} chi e^{-tau H},
# 0 <= tau <= beta.  Tr[e^{-(beta - tau) H} chi e^{-tau H} chi] cut
# symmetrically around the typical state: with u = e^{-(beta - tau) H / 2} psi,
#     G_est(tau) = || e^{-tau H / 2} chi_i u ||^2 / || e^{-beta H / 2} psi ||^2.
def imag_two_point_estimator(prop, maj, psi, i: int, beta: float, taus):
    """G_est(tau) for each tau (each propagated from scratch).  Returns (G, Z)."""
    Z = float(np.linalg.norm(prop.imag(psi, beta / 2)) ** 2)
    out = np.empty(len(taus))
    for n, tau in enumerate(taus):
        u = prop.imag(psi, (beta - tau) / 2)
        w = prop.imag(maj(i, u), tau / 2)
        out[n] = float(np.vdot(w, w).real) / Z
    return out, Z


def imag_two_point_trace(dense_exp, chis, i: int, beta: float, taus):
    """Exact G(tau) = Tr[e^{tau H} chi_i e^{-tau H} chi_i rho] / Tr rho."""
    rho = dense_exp.matrix(-beta)
    Zt = float(np.trace(rho).real)
    out = np.empty(len(taus))
    for n, tau in enumerate(taus):
        Xt = dense_exp.matrix(tau) @ chis[i] @ dense_exp.matrix(-tau)
        out[n] = float(np.trace(Xt @ chis[i] @ rho).real) / Zt
    return out
