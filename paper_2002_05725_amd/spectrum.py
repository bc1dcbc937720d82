"""Host post-processing of low-lying Ritz values (no GPU work).

The paper keeps a system size for the finite-size extrapolation at inverse
temperature beta only if its lowest 20 eigenstates lie within Delta E = 1/beta
of the ground state (main text, discussion of the validity range; SI,
finite-size extrapolation).  Lanczos returns levels; the state count needs the
multiplicity of each level, fixed in the full 2^(N/2) space by N mod 8 (every
level twofold for N mod 8 in {2, 4, 6}, simple for N mod 8 = 0).
"""
from __future__ import annotations

import numpy as np


def level_multiplicity(N: int) -> int:
    """Degeneracy of every level of the q=4 SYK Hamiltonian in the full space."""
    return 2 if N % 8 in (2, 4, 6) else 1


def distinct_levels(theta, resid, tol: float = 1e-8):
    """Converged Ritz values (residual <= tol), ascending, with copies of the
    same level (closer than tol) merged."""
    theta = np.asarray(theta, dtype=float)
    resid = np.asarray(resid, dtype=float)
    good = np.sort(theta[resid <= tol])
    if good.size == 0:
        return good
    keep = np.concatenate(([True], np.diff(good) > tol))
    return good[keep]


def states_within(levels, N: int, width: float) -> int:
    """Number of eigenstates within `width` of the lowest level."""
    levels = np.asarray(levels, dtype=float)
    return int(level_multiplicity(N) * np.count_nonzero(levels - levels[0] <= width))


def beta_max(levels, N: int, count: int = 20) -> float:
    """Largest beta at which at least `count` eigenstates lie within 1/beta of
    the ground state: 1 / (E_k - E_0), E_k the level that completes the count.
    Raises if the levels given do not reach `count` states."""
    levels = np.asarray(levels, dtype=float)
    per = level_multiplicity(N)
    need = -(-count // per)          # levels needed
    if levels.size < need:
        raise ValueError(f"need {need} converged levels for {count} states, have {levels.size}")
    width = levels[need - 1] - levels[0]
    return float("inf") if width <= 0 else 1.0 / width
