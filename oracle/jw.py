"""Majoranas under the Jordan-Wigner map and the dense SYK Hamiltonian.

Test infrastructure only (see the package docstring).

* SI, section "Jordan-Wigner transformation": N Majoranas on N/2 qubits,
  chi_i = (prod_{q<k} Z_q) X_k for even i and (prod_{q<k} Z_q) Y_k for odd i,
  with k = floor(i/2) and 0 <= i < N.
* Main text, Eq. 1 and the sentence after it: {chi_i, chi_j} = delta_ij.  The
  bare Pauli strings square to 1, so each is divided by sqrt(2) here.
* Qubit k is bit k of the basis index (least significant first);
  Y = [[0, -i], [i, 0]].
"""
from __future__ import annotations

import itertools
import math
from functools import reduce

import numpy as np

_I2 = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def quartets(N: int):
    """All i<j<k<l over 0..N-1, lexicographic (the coupling order)."""
    return list(itertools.combinations(range(N), 4))


def dense_majoranas(N: int):
    """chi_0 .. chi_{N-1} as dense 2^(N/2) x 2^(N/2) matrices, built with np.kron.

    np.kron puts its first factor on the most significant bit, so the factor
    list runs from qubit M-1 down to qubit 0.
    """
    M = N // 2
    out = []
    for i in range(N):
        k = i // 2
        factors = []
        for q in range(M - 1, -1, -1):
            if q < k:
                factors.append(_Z)
            elif q == k:
                factors.append(_X if i % 2 == 0 else _Y)
            else:
                factors.append(_I2)
        out.append(reduce(np.kron, factors) / math.sqrt(2.0))
    return out


def dense_H(N: int, J: np.ndarray, chis=None) -> np.ndarray:
    """H = sum_{i<j<k<l} J_ijkl chi_i chi_j chi_k chi_l as a dense matrix (Eq. 1)."""
    if chis is None:
        chis = dense_majoranas(N)
    D = chis[0].shape[0]
    H = np.zeros((D, D), dtype=np.complex128)
    for n, (i, j, k, l) in enumerate(quartets(N)):
        H += J[n] * (chis[i] @ chis[j] @ chis[k] @ chis[l])
    return H


def dense_quartet(N: int, n: int, chis=None) -> np.ndarray:
    """The operator chi_i chi_j chi_k chi_l multiplying coupling n."""
    if chis is None:
        chis = dense_majoranas(N)
    i, j, k, l = quartets(N)[n]
    return chis[i] @ chis[j] @ chis[k] @ chis[l]


def majorana_apply(N: int, a: int, psi: np.ndarray) -> np.ndarray:
    """chi_a psi without building a matrix: chi_a maps |s> to
    amp(s) |s xor 2^k>, amp = 2^{-1/2} (-1)^{popcount(s mod 2^k)}, times
    i (-1)^{s_k} when a is odd (Y_k = i X_k Z_k)."""
    D = psi.shape[0]
    k = a // 2
    s = np.arange(D, dtype=np.uint64)
    below = s & np.uint64((1 << k) - 1)
    neg = np.bitwise_count(below).astype(np.int64) & 1
    amp = np.where(neg == 1, -1.0, 1.0).astype(np.complex128) / math.sqrt(2.0)
    if a % 2 == 1:
        bit = ((s >> np.uint64(k)) & np.uint64(1)).astype(np.int64)
        amp = amp * 1j * np.where(bit == 1, -1.0, 1.0)
    out = np.empty_like(psi, dtype=np.complex128)
    out[(s ^ np.uint64(1 << k)).astype(np.int64)] = amp * psi
    return out


def parity_operator(N: int) -> np.ndarray:
    """Diagonal of prod_k Z_k: the fermion parity of the SI (conserved by H)."""
    D = 1 << (N // 2)
    s = np.arange(D, dtype=np.uint64)
    return np.where(np.bitwise_count(s) % 2 == 0, 1.0, -1.0)


def sector_rows(N: int, s: int) -> np.ndarray:
    """Full-space rows of the fermion-parity sector s (popcount(r) = s mod 2),
    in the order of the sector index u: r = u + 2^(M-1) (parity(u) ^ s), M = N/2.
    (H conserves the parity of the qubit string; each Majorana flips it.)"""
    M = N // 2
    u = np.arange(1 << (M - 1), dtype=np.int64)
    par = np.zeros_like(u)
    v = u.copy()
    while v.any():
        par ^= v & 1
        v >>= 1
    return u + ((par ^ s) << (M - 1))


def quartet_apply(N: int, q, psi: np.ndarray) -> np.ndarray:
    """chi_i chi_j chi_k chi_l psi for the quartet q = (i, j, k, l), i < j < k < l:
    the operator multiplying J_ijkl in Eq. 1, applied as four Majoranas (the
    rightmost acts first), without a matrix."""
    i, j, k, l = q
    out = psi
    for a in (l, k, j, i):
        out = majorana_apply(N, a, out)
    return out


def coupling_overlaps(N: int, qs, pairs) -> np.ndarray:
    """For each quartet q in qs: sum_p w_p Re <g_p| chi_i chi_j chi_k chi_l |v_p>,
    the derivative of sum_p w_p Re <g_p|H|v_p> with respect to J_ijkl (Eq. 1 is
    linear in the couplings).  pairs: (g, v, w) triples."""
    out = np.zeros(len(qs))
    for n, q in enumerate(qs):
        for g, v, w in pairs:
            out[n] += w * np.vdot(g, quartet_apply(N, q, v)).real
    return out
