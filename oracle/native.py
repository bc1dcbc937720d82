"""ctypes wrapper and build step for the checker's plain C code (plain_apply.c).

Test infrastructure only: see the package docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "plain_apply.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile plain_apply.c with gcc/OpenMP into oracle/liboracle.so."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        c_i64p = ctypes.POINTER(ctypes.c_int64)
        c_dp = ctypes.c_void_p
        L.oracle_apply_rows.argtypes = [ctypes.c_int, c_dp, c_dp, c_dp, ctypes.c_int64, c_dp]
        L.oracle_apply_range.argtypes = [ctypes.c_int, c_dp, c_dp, ctypes.c_int64, ctypes.c_int64, c_dp]
        L.oracle_majorana.argtypes = [ctypes.c_int, ctypes.c_int, c_dp, c_dp]
        L.oracle_sparse_nflips.argtypes = [ctypes.c_int]
        L.oracle_sparse_nflips.restype = ctypes.c_int64
        L.oracle_sparse_H.argtypes = [ctypes.c_int, c_dp, c_dp, c_dp, c_dp]
        L.oracle_sparse_matvec.argtypes = [ctypes.c_int64, c_dp, c_dp, c_dp, c_dp, c_dp]
        L.oracle_num_threads.restype = ctypes.c_int
        for f in (L.oracle_apply_rows, L.oracle_apply_range, L.oracle_majorana,
                  L.oracle_sparse_H, L.oracle_sparse_matvec):
            f.restype = ctypes.c_int
        del c_i64p
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def apply_rows(N: int, J: np.ndarray, psi: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """(H psi)[rows], each row summed term by term over all C(N,4) quartets."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.size, dtype=np.complex128)
    _check(lib().oracle_apply_rows(N, _p(J), _p(psi), _p(rows), rows.size, _p(out)), "apply_rows")
    return out


def apply_range(N: int, J: np.ndarray, psi: np.ndarray, begin: int, end: int) -> np.ndarray:
    J = np.ascontiguousarray(J, dtype=np.float64)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty(end - begin, dtype=np.complex128)
    _check(lib().oracle_apply_range(N, _p(J), _p(psi), begin, end, _p(out)), "apply_range")
    return out


def apply_full(N: int, J: np.ndarray, psi: np.ndarray) -> np.ndarray:
    return apply_range(N, J, psi, 0, psi.size)


def majorana(N: int, a: int, psi: np.ndarray) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty_like(psi)
    _check(lib().oracle_majorana(N, a, _p(psi), _p(out)), "majorana")
    return out


class SparseH:
    """H as an explicit sparse matrix (one entry per row per distinct qubit flip)."""

    def __init__(self, N: int, J: np.ndarray):
        self.N = N
        self.D = 1 << (N // 2)
        nu = int(lib().oracle_sparse_nflips(N))
        if nu <= 0:
            raise ValueError("bad N")
        J = np.ascontiguousarray(J, dtype=np.float64)
        self.row_ptr = np.empty(self.D + 1, dtype=np.int64)
        self.cols = np.empty(self.D * nu, dtype=np.int64)
        self.vals = np.empty(self.D * nu, dtype=np.complex128)
        _check(lib().oracle_sparse_H(N, _p(J), _p(self.row_ptr), _p(self.cols), _p(self.vals)),
               "sparse_H")
        self.n_flips = nu

    def __call__(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.empty_like(x)
        _check(lib().oracle_sparse_matvec(self.D, _p(self.row_ptr), _p(self.cols), _p(self.vals),
                                          _p(x), _p(y)), "sparse_matvec")
        return y
