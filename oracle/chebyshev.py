"""Fixed-degree Chebyshev propagator and the exact derivative of the OTOC in
the couplings.  Test infrastructure only (see the package docstring).

The paper propagates with Krylov steps (SI "Krylov subspace methods"); the
gradient extension replaces every propagator by a fixed polynomial so that
the forward map is a fixed polynomial in the couplings and its derivative is
exact.  With H~ = (H - e_c) / e_h (spectrum inside [-1, 1]) and the
three-term recurrence T_0 v = v, T_1 v = H~ v, T_{n+1} v = 2 H~ T_n v - T_{n-1} v:

* e^{-i h H} = e^{-i h e_c} sum_n (2 - delta_n0) (-i)^n J_n(e_h h) T_n(H~)
  (Jacobi-Anger expansion),
* e^{-h H}   = e^{-h e_c}   sum_n (2 - delta_n0) (-1)^n I_n(e_h h) T_n(H~)
  (generating function of the modified Bessel functions),
both truncated at a fixed degree.  (e_c, e_h) are fixed inputs and do not
move with J.

The OTOC uses the same symmetric cut as ``correlators.otoc_estimator``: real
legs are round(t/dt) Chebyshev steps of length dt; each imaginary leg
(rho^{1/8}, rho^{1/4}, and rho^{1/2} for Z) is `tau_steps` steps.

``derivative`` propagates, next to every vector, its derivative along one
coupling J_k (forward mode: d(H v) = Q_k v + H dv, where Q_k is the quartet
operator multiplying J_k).
"""
from __future__ import annotations

import numpy as np
import scipy.special


def coefficients(kind: str, h: float, e_c: float, e_h: float, degree: int) -> np.ndarray:
    n = np.arange(degree + 1)
    w = np.where(n == 0, 1.0, 2.0)
    if kind == "real":
        return w * (-1j) ** n * scipy.special.jv(n, e_h * h) * np.exp(-1j * e_c * h)
    if kind == "imag":
        return (w * (-1.0) ** n * scipy.special.iv(n, e_h * h) * np.exp(-e_c * h)).astype(np.complex128)
    raise ValueError(kind)


class ChebPropagator:
    """Applies the truncated expansions above to a vector and, optionally, to
    its tangent along one coupling."""

    def __init__(self, matvec, e_c: float, e_h: float, degree: int, dmatvec=None):
        self.matvec, self.e_c, self.e_h, self.degree = matvec, e_c, e_h, degree
        self.dmatvec = dmatvec          # v -> Q_k v, or None

    def _Ht(self, v):
        return (self.matvec(v) - self.e_c * v) / self.e_h

    def step(self, v, dv, kind: str, h: float):
        c = coefficients(kind, h, self.e_c, self.e_h, self.degree)
        t0, t1 = v, self._Ht(v)
        acc = c[0] * t0 + c[1] * t1
        if dv is None:
            for n in range(2, self.degree + 1):
                t0, t1 = t1, 2.0 * self._Ht(t1) - t0
                acc = acc + c[n] * t1
            return acc, None
        d0 = dv
        d1 = self._Ht(dv) + self.dmatvec(v) / self.e_h
        dacc = c[0] * d0 + c[1] * d1
        for n in range(2, self.degree + 1):
            t_new = 2.0 * self._Ht(t1) - t0
            d_new = 2.0 * (self._Ht(d1) + self.dmatvec(t1) / self.e_h) - d0
            t0, t1, d0, d1 = t1, t_new, d1, d_new
            acc = acc + c[n] * t1
            dacc = dacc + c[n] * d1
        return acc, dacc

    def real(self, v, dv, t: float, dt: float):
        n = int(round(abs(t) / dt))
        if abs(n * dt - abs(t)) > 1e-9 * max(1.0, abs(t)):
            raise ValueError("t must be a multiple of dt")
        sgn = 1.0 if t >= 0 else -1.0
        for _ in range(n):
            v, dv = self.step(v, dv, "real", sgn * dt)
        return v, dv

    def imag(self, v, dv, tau: float, tau_steps: int):
        if tau == 0:
            return v, dv
        for _ in range(tau_steps):
            v, dv = self.step(v, dv, "imag", tau / tau_steps)
        return v, dv


def otoc(prop: ChebPropagator, maj, psi, i: int, j: int, beta: float, t: float, dt: float,
         tau_steps: int = 1):
    """F(t) of the Chebyshev forward; with prop.dmatvec set also dF/dJ_k.

    Returns (F, dF or None)."""
    tangent = prop.dmatvec is not None
    zero = np.zeros_like(psi, dtype=np.complex128) if tangent else None
    dmaj = (lambda a, dv: None if dv is None else maj(a, dv))

    u, du = prop.imag(psi, zero, beta / 2, tau_steps)                 # rho^{1/2} psi
    a0, da0 = prop.imag(psi, zero, beta / 8, tau_steps)               # rho^{1/8} psi
    b0, db0 = prop.imag(maj(j, a0), dmaj(j, da0), beta / 4, tau_steps)

    x, dx = prop.real(b0, db0, t, dt)
    x, dx = prop.real(maj(i, x), dmaj(i, dx), -t, dt)
    A, dA = prop.imag(x, dx, beta / 8, tau_steps)                     # A psi

    y, dy = prop.real(a0, da0, t, dt)
    y, dy = prop.real(maj(i, y), dmaj(i, dy), -t, dt)
    y, dy = prop.imag(y, dy, beta / 4, tau_steps)
    B, dB = prop.imag(maj(j, y), dmaj(j, dy), beta / 8, tau_steps)   # A^dag psi

    Z = float(np.vdot(u, u).real)
    F = float(np.vdot(B, A).real) / Z
    if not tangent:
        return F, None
    dZ = 2.0 * float(np.vdot(u, du).real)
    dnum = float((np.vdot(dB, A) + np.vdot(B, dA)).real)
    return F, (dnum - F * dZ) / Z


def gradient_tangent(matvec_of_J, quartet_matvec, J, maj, psi, i, j, beta, t, dt, e_c, e_h,
                     degree, couplings, tau_steps: int = 1):
    """dF/dJ_k for k in `couplings` by forward-mode tangents (one run per k).

    matvec_of_J(J) -> (v -> H(J) v); quartet_matvec(k) -> (v -> Q_k v)."""
    mv = matvec_of_J(J)
    out = np.empty(len(couplings))
    F = None
    for n, k in enumerate(couplings):
        prop = ChebPropagator(mv, e_c, e_h, degree, dmatvec=quartet_matvec(k))
        F, out[n] = otoc(prop, maj, psi, i, j, beta, t, dt, tau_steps)
    return F, out


def gradient_fd(matvec_of_J, J, maj, psi, i, j, beta, t, dt, e_c, e_h, degree, couplings,
                h: float = 1e-6, tau_steps: int = 1):
    """Central finite differences (F(J + h e_k) - F(J - h e_k)) / 2h."""
    out = np.empty(len(couplings))
    for n, k in enumerate(couplings):
        vals = []
        for s in (+1.0, -1.0):
            Jp = np.array(J, dtype=np.float64, copy=True)
            Jp[k] += s * h
            prop = ChebPropagator(matvec_of_J(Jp), e_c, e_h, degree)
            vals.append(otoc(prop, maj, psi, i, j, beta, t, dt, tau_steps)[0])
        out[n] = (vals[0] - vals[1]) / (2.0 * h)
    return out
