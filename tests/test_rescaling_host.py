"""The finite-size rescaling estimate of lambda on synthetic curves that obey
the rescaling symmetry (N -> rN, t -> t + log(r)/lambda) exactly."""
import numpy as np
import pytest

from paper_2002_05725_amd import rescaling


def _curve(N, lam, c=0.05):
    # F~(t) = min(1, 2 - c e^{lam t} / N): F~(0) = 1, and F~ depends on t only
    # through t - log(N) / lam, so it obeys the rescaling symmetry exactly;
    # crossing 1 - F0 at t* = log((1 + F0) N / c) / lam.
    t = np.linspace(0.0, 12.0, 2401)
    return t, -0.25 * np.minimum(1.0, 2.0 - c * np.exp(lam * t) / N)


def test_crossing_time_matches_closed_form():
    lam, N, F0, a = 0.9, 40, 0.25, 0.02
    t = np.linspace(0.0, 12.0, 2401)
    F = -0.25 * (1.0 - a * np.exp(lam * t) / N)      # F~ = (1 - a e^{lam t}/N) / (1 - a/N)
    exact = np.log(F0 * N / a + (1.0 - F0)) / lam
    assert abs(rescaling.crossing_time(t, F, F0) - exact) < 1e-4
    assert abs(rescaling.crossing_time(t, F, F0, cubic=True) - exact) < 1e-8


def test_lambda_recovered_exactly_under_the_symmetry():
    lam = 1.3
    curves = {N: _curve(N, lam) for N in (24, 28, 32, 36, 40, 44)}
    out = rescaling.lyapunov(curves, F0=0.16, degree=1, cubic=True)
    assert np.allclose(out["lambda_fit"], lam, rtol=1e-7)
    assert abs(out["lambda_0"] - lam) < 1e-6


def test_one_over_n_extrapolation_recovers_lambda_0():
    lam0, lam1 = 2.0, -15.0
    N = np.array([24.0, 28.0, 32.0, 36.0, 40.0, 44.0, 48.0, 52.0])
    l0, err, coef = rescaling.extrapolate(N, lam0 + lam1 / N, degree=1)
    assert abs(l0 - lam0) < 1e-12 and abs(coef[1] - lam1) < 1e-10 and err < 1e-10
    l0, err, coef = rescaling.extrapolate(N, lam0 + lam1 / N + 40.0 / N**2, degree=2)
    assert abs(l0 - lam0) < 1e-10


def test_keep_filters_sizes_and_bad_curve_raises():
    curves = {N: _curve(N, 1.0) for N in (24, 28, 32, 36)}
    out = rescaling.lyapunov(curves, keep=lambda n: n >= 32)
    assert out["N"] == [32.0, 36.0]
    t = np.linspace(0, 1, 11)
    with pytest.raises(ValueError):
        rescaling.crossing_time(t, -0.25 * np.ones_like(t), 0.25)
