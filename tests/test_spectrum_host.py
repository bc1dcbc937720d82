"""Host post-processing of Lanczos levels (level multiplicity, states within
1/beta of the ground state) against the dense spectrum."""
import numpy as np
import pytest

from oracle import jw
from paper_2002_05725_amd import inputs, spectrum


@pytest.mark.parametrize("N", [8, 10, 12, 14])
def test_multiplicity_and_state_count_match_dense_spectrum(N):
    ev = np.linalg.eigvalsh(jw.dense_H(N, inputs.couplings(N, 6)))
    levels = spectrum.distinct_levels(ev, np.zeros_like(ev), tol=1e-9)
    assert levels.size * spectrum.level_multiplicity(N) == ev.size
    for width in (0.0, 0.05, 0.2, 0.7):
        assert spectrum.states_within(levels, N, width) == np.count_nonzero(ev - ev[0] <= width + 1e-12)


def test_beta_max_is_the_window_of_the_count():
    N = 14
    ev = np.linalg.eigvalsh(jw.dense_H(N, inputs.couplings(N, 6)))
    levels = spectrum.distinct_levels(ev, np.zeros_like(ev), tol=1e-9)
    b = spectrum.beta_max(levels, N, count=20)
    assert np.count_nonzero(ev - ev[0] <= 1.0 / b + 1e-12) >= 20
    assert np.count_nonzero(ev - ev[0] < 1.0 / b - 1e-9) < 20
    with pytest.raises(ValueError):
        spectrum.beta_max(levels[:3], N, count=20)


def test_distinct_levels_drops_unconverged_and_merges_copies():
    theta = np.array([-1.0, -1.0 + 1e-12, -0.9, -0.5])
    res = np.array([1e-12, 1e-11, 1e-3, 0.0])
    assert np.allclose(spectrum.distinct_levels(theta, res, tol=1e-8), [-1.0, -0.5])
