"""The seeded input generators: sector states are the typical states on the
sector rows (checked against the checker's own row map)."""
import numpy as np
import pytest

from oracle import jw
from paper_2002_05725_amd import inputs


@pytest.mark.parametrize("N", [6, 12, 20])
@pytest.mark.parametrize("s", [0, 1])
def test_typical_sector_state_is_the_restricted_typical_state(N, s):
    full = inputs.typical_state(N, 3)[jw.sector_rows(N, s)]
    assert np.allclose(inputs.typical_sector_state(N, s, 3), full / np.linalg.norm(full), rtol=0, atol=1e-15)


def test_couplings_distribution():
    J = inputs.couplings(40, 0)
    assert J.size == 91390
    assert abs(J.std() - np.sqrt(6 / 40**3)) < 0.01 * np.sqrt(6 / 40**3)
