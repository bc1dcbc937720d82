"""Seeded synthetic inputs for the SYK workloads.

This module only draws random numbers; it holds none of the method's
arithmetic.  Both the HIP path and the CPU checker receive the arrays it
returns, so neither side regenerates them.

* Couplings: the SYK Hamiltonian (main text, Eq. 1) draws real J_ijkl from a
  Gaussian with zero mean and variance 6 J^2 / N^3.  The quartets i<j<k<l
  are enumerated lexicographically over 0-based Majorana indices, i.e. in
  ``itertools.combinations(range(N), 4)`` order.
* Typical states: the SI section "Disorder averaging" draws every complex
  amplitude of a Haar-random state from a Gaussian.  Recipe used here: the
  state is filled in chunks of ``_CHUNK`` amplitudes; each chunk takes
  2*chunk consecutive standard normals g from one ``numpy.random.Generator``
  and sets psi = g[0::2] + 1j*g[1::2]; the whole vector is then divided by its
  FP64 2-norm.
"""
from __future__ import annotations

import math

import numpy as np

_CHUNK = 1 << 22


def n_quartets(N: int) -> int:
    """Number of couplings C(N, 4)."""
    return math.comb(N, 4)


def dim(N: int) -> int:
    """Hilbert-space dimension 2^(N/2) of N Majoranas on N/2 qubits."""
    if N % 2:
        raise ValueError("N must be even")
    return 1 << (N // 2)


def couplings(N: int, seed: int, J: float = 1.0) -> np.ndarray:
    """C(N,4) real couplings with variance 6 J^2 / N^3, FP64, lexicographic order."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n_quartets(N)) * math.sqrt(6.0 * J * J / N ** 3)


def typical_state(N: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Normalized Gaussian random state of dimension 2^(N/2) (see module doc)."""
    D = dim(N)
    rng = np.random.default_rng(seed)
    psi = np.empty(D, dtype=np.complex128)
    for lo in range(0, D, _CHUNK):
        n = min(_CHUNK, D - lo)
        g = rng.standard_normal(2 * n)
        psi.real[lo:lo + n] = g[0::2]
        psi.imag[lo:lo + n] = g[1::2]
        del g
    psi /= np.linalg.norm(psi)
    if dtype != np.complex128:
        psi = psi.astype(dtype)
    return psi


def quartet_sample(N: int, seed: int, count: int) -> np.ndarray:
    """Indices of `count` distinct couplings, chosen uniformly without replacement."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_quartets(N), count, replace=False))


def row_sample(N: int, seed: int, count: int) -> np.ndarray:
    """`count` distinct basis rows, sorted, for row-sampled checks at large N."""
    D = dim(N)
    rng = np.random.default_rng(seed)
    if count >= D:
        return np.arange(D, dtype=np.int64)
    return np.sort(rng.choice(D, count, replace=False)).astype(np.int64)


# Seeds for the batched disorder-averaging workload: realisation r of size N
# uses couplings seed 1000*N + r and typical-state seeds 10^6 + 1000*N + 2r + s.
def batch_coupling_seed(N: int, r: int) -> int:
    return 1000 * N + r


def batch_state_seed(N: int, r: int, s: int) -> int:
    return 10 ** 6 + 1000 * N + 2 * r + s


def typical_sector_state(N: int, s: int, seed: int) -> np.ndarray:
    """Typical state of the fermion-parity sector s: the entries of
    typical_state(N, seed) on the rows of popcount parity s, in the sector
    order (entry u is the full row u + 2^(M-1) (parity(u) ^ s)), renormalized."""
    M = N // 2
    u = np.arange(1 << (M - 1), dtype=np.int64)
    par = np.zeros_like(u)
    v = u.copy()
    while v.any():
        par ^= v & 1
        v >>= 1
    rows = u + ((par ^ (s & 1)) << (M - 1))
    del u, par, v
    psi = typical_state(N, seed)[rows]
    return psi / np.linalg.norm(psi)

