"""Krylov (Lanczos) propagation, written plainly.  Test infrastructure only.

SI, section "Krylov subspace methods": e^{-iHt}|psi> is approximated by a
degree-m polynomial in H obtained from the projection of H onto the
subspace spanned by psi, H psi, ..., i.e. by exponentiating the small
projected matrix, and long evolutions are cut into short time steps.

Reading used here: m is the number of basis vectors, so one step applies H
m times and the projection T is m x m (tridiagonal for Hermitian H).  The
basis is kept orthonormal by classical Gram-Schmidt against all previous
vectors, done twice.  e^{zT} e_1 comes from the eigendecomposition of T.
The same routine with a real exponent z = -tau gives e^{-tau H}.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg
from threadpoolctl import threadpool_limits


def _one_blas_thread(fn):
    """Runs fn with numpy's BLAS on one thread: the loops below interleave small
    products with the C checker's OpenMP matvec, and idle BLAS threads spinning
    between products would compete with it for the cores."""
    def wrapped(*args, **kwargs):
        with threadpool_limits(1, user_api="blas"):
            return fn(*args, **kwargs)
    wrapped.__name__, wrapped.__doc__ = fn.__name__, fn.__doc__
    return wrapped


@_one_blas_thread
def krylov_step(matvec, psi: np.ndarray, z: complex, m: int, breakdown_tol: float = 1e-13):
    """Return (e^{z H} psi, error estimate) from an m-dimensional Krylov space.

    The error estimate is beta_m |e_m^T e^{zT} e_1| ||psi||.  When the space
    becomes invariant (beta_j ~ 0) the projection is exact and the loop stops.
    """
    nrm = float(np.linalg.norm(psi))
    if nrm == 0.0:
        return np.zeros_like(psi, dtype=np.complex128), 0.0
    V = np.zeros((m, psi.size), dtype=np.complex128)
    V[0] = psi / nrm
    alpha, beta = [], []
    beta_last = 0.0
    k = m
    for j in range(m):
        w = matvec(V[j]).astype(np.complex128)
        Vj = V[: j + 1]
        c1 = Vj.conj() @ w
        w = w - Vj.T @ c1
        c2 = Vj.conj() @ w
        w = w - Vj.T @ c2
        alpha.append(float((c1[j] + c2[j]).real))
        b = float(np.linalg.norm(w))
        scale = max(abs(a) for a in alpha) + (beta[-1] if beta else 0.0)
        if j == m - 1:
            beta_last = b
            break
        if b <= breakdown_tol * max(scale, 1e-300):
            k = j + 1
            beta_last = 0.0
            break
        beta.append(b)
        V[j + 1] = w / b
    a = np.array(alpha[:k])
    b = np.array(beta[: k - 1])
    if k == 1:
        evals, evecs = a.copy(), np.ones((1, 1))
    else:
        evals, evecs = scipy.linalg.eigh_tridiagonal(a, b)
    coef = evecs @ (np.exp(z * evals) * evecs[0, :])
    y = nrm * (V[:k].T @ coef)
    err = nrm * beta_last * abs(coef[-1])
    return y, err


@_one_blas_thread
def propagate(matvec, psi: np.ndarray, z: complex, total: float, dt: float, m: int):
    """e^{z * total * H} psi in ceil(total/dt) equal Krylov steps."""
    if total == 0.0:
        return np.array(psi, dtype=np.complex128, copy=True)
    nsteps = max(1, int(math.ceil(total / dt - 1e-9)))
    h = total / nsteps
    y = np.array(psi, dtype=np.complex128, copy=True)
    for _ in range(nsteps):
        y, _ = krylov_step(matvec, y, z * h, m)
    return y


class DenseExp:
    """Exact e^{zH} from a dense eigendecomposition (exact diagonalisation)."""

    def __init__(self, H: np.ndarray):
        self.evals, self.evecs = np.linalg.eigh(H)

    def apply(self, psi: np.ndarray, z: complex) -> np.ndarray:
        c = self.evecs.conj().T @ psi
        return self.evecs @ (np.exp(z * self.evals) * c)

    def matrix(self, z: complex) -> np.ndarray:
        return (self.evecs * np.exp(z * self.evals)) @ self.evecs.conj().T


@_one_blas_thread
def lanczos_ritz(matvec, psi: np.ndarray, m: int, breakdown_tol: float = 1e-13):
    """Ritz values of H from an m-step Lanczos run started at psi (the same
    projection as krylov_step: orthonormal basis by classical Gram-Schmidt
    done twice, T tridiagonal).  Returns (theta ascending, residual norms
    beta_k |s_{k,i}|), where s_i is the i-th eigenvector of T and beta_k the
    coefficient that would start the next basis vector (0 when the space is
    invariant: then theta are exact eigenvalues of H, one per distinct
    eigenvalue that psi touches)."""
    nrm = float(np.linalg.norm(psi))
    V = np.zeros((m, psi.size), dtype=np.complex128)
    V[0] = psi / nrm
    alpha, beta = [], []
    beta_last = 0.0
    k = m
    for j in range(m):
        w = matvec(V[j]).astype(np.complex128)
        Vj = V[: j + 1]
        c1 = Vj.conj() @ w
        w = w - Vj.T @ c1
        c2 = Vj.conj() @ w
        w = w - Vj.T @ c2
        alpha.append(float((c1[j] + c2[j]).real))
        b = float(np.linalg.norm(w))
        scale = max(abs(a) for a in alpha) + (beta[-1] if beta else 0.0)
        if j == m - 1:
            beta_last = b
            break
        if b <= breakdown_tol * max(scale, 1e-300):
            k = j + 1
            break
        beta.append(b)
        V[j + 1] = w / b
    a = np.array(alpha[:k])
    if k == 1:
        return a.copy(), np.zeros(1)
    theta, S = scipy.linalg.eigh_tridiagonal(a, np.array(beta[: k - 1]))
    return theta, beta_last * np.abs(S[-1, :])
