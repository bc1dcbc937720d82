"""Finite-size rescaling estimate of the Lyapunov exponent (host
post-processing of OTOC curves; no GPU work).

Main text, "Lyapunov exponent of the SYK model", and the SI section on the
finite-size extrapolation: near the semiclassical limit OTOCs obey the
rescaling symmetry N -> r N, t -> t + log(r) / lambda.  For each size N the
normalized curve F~(t) = F(t)/F(0) is interpolated to the time t*(N) where it
crosses the level 1 - F0; 1/lambda_fit(N) is the finite difference of t*
against log N between successive sizes; lambda_fit(N) is fitted by a
polynomial in 1/N whose constant term lambda_0 estimates lambda.

Readings (the text is not uniform): the crossing level is 1 - F0 as in the
main text and the figure caption (the SI body writes F0); lambda_fit from the
sizes N_{k-1} < N_k is attached to N_k, as in the SI formula; the curve is
interpolated linearly between samples unless `cubic=True`.
"""
from __future__ import annotations

import numpy as np


def crossing_time(times, F, F0: float, cubic: bool = False) -> float:
    """First t with F(t)/F(0) = 1 - F0 (interpolated); times ascending, times[0] = 0."""
    t = np.asarray(times, dtype=float)
    f = np.asarray(F, dtype=float) / float(F[0])
    level = 1.0 - F0
    below = np.nonzero(f <= level)[0]
    if below.size == 0 or below[0] == 0:
        raise ValueError("the curve does not cross the level after t = 0")
    k = int(below[0])
    if not cubic:
        t0, t1, f0, f1 = t[k - 1], t[k], f[k - 1], f[k]
        return float(t0 + (level - f0) * (t1 - t0) / (f1 - f0))
    # cubic through up to four samples around the crossing, then bisection
    lo, hi = max(0, k - 2), min(len(t), k + 2)
    c = np.polyfit(t[lo:hi], f[lo:hi], min(3, hi - lo - 1))
    a, b = t[k - 1], t[k]
    for _ in range(100):
        m = 0.5 * (a + b)
        if (np.polyval(c, m) - level) * (np.polyval(c, a) - level) <= 0:
            b = m
        else:
            a = m
    return float(0.5 * (a + b))


def lambda_fit(sizes, tstar):
    """(N_k, lambda_fit(N_k)) from successive sizes: 1/lambda = dt*/d log N."""
    N = np.asarray(sizes, dtype=float)
    ts = np.asarray(tstar, dtype=float)
    order = np.argsort(N)
    N, ts = N[order], ts[order]
    dlog = np.diff(np.log(N))
    dt = np.diff(ts)
    return N[1:], dlog / dt


def extrapolate(N, lam, degree: int = 1):
    """Least-squares fit lambda_fit(N) = sum_k c_k / N^k, k <= degree.
    Returns (lambda_0, its standard error, all coefficients)."""
    N = np.asarray(N, dtype=float)
    lam = np.asarray(lam, dtype=float)
    A = np.vander(1.0 / N, degree + 1, increasing=True)
    coef, *_ = np.linalg.lstsq(A, lam, rcond=None)
    dof = len(lam) - (degree + 1)
    if dof > 0:
        r = lam - A @ coef
        s2 = float(r @ r) / dof
        cov = s2 * np.linalg.inv(A.T @ A)
        err = float(np.sqrt(cov[0, 0]))
    else:
        err = float("nan")
    return float(coef[0]), err, coef


def lyapunov(curves, F0: float = 0.25, degree: int = 1, keep=None, cubic: bool = False):
    """lambda_0 from {N: (times, F)} curves at one temperature.  `keep`
    (optional) selects the sizes used in the 1/N fit, e.g. those whose lowest
    20 eigenstates lie within 1/beta of the ground state (spectrum.beta_max)."""
    sizes = sorted(curves)
    ts = [crossing_time(*curves[n], F0, cubic=cubic) for n in sizes]
    Nk, lam = lambda_fit(sizes, ts)
    if keep is not None:
        sel = np.array([keep(int(n)) for n in Nk], dtype=bool)
        Nk, lam = Nk[sel], lam[sel]
    lam0, err, coef = extrapolate(Nk, lam, degree)
    return {"lambda_0": lam0, "stderr": err, "coef": coef.tolist(), "N": Nk.tolist(),
            "lambda_fit": lam.tolist(), "tstar": dict(zip(sizes, ts))}
