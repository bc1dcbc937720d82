"""Host check of the library's tridiagonal eigensolver (the Ritz values and
vectors of every Lanczos step), without a GPU: tests/host/tridiag_eig_check.cpp
runs it on seeded tridiagonal matrices (random, split by a zero coupling,
constant diagonal, graded, 1 x 1 and 2 x 2, and up to 200 x 200 as in the
lowest-eigenvalue search), and the results are compared with numpy's
symmetric eigensolver on the same dense matrix."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _cases():
    rng = np.random.default_rng(11)
    out = []
    for n in (1, 2, 3, 5, 12, 16, 30, 64, 200):
        d = rng.standard_normal(n)
        e = np.abs(rng.standard_normal(n - 1))
        out.append((d, e))
        if n >= 4:
            e2 = e.copy()
            e2[n // 2] = 0.0                       # splits into two blocks
            out.append((d, e2))
            out.append((np.ones(n), e))            # constant diagonal
            out.append((d * 10.0 ** np.linspace(-6, 6, n), e))   # graded diagonal
            out.append((d, e * 1e-9))              # nearly diagonal
    return out


def test_tridiagonal_eigensolver_matches_dense(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "tridiag_eig_check")
    r = subprocess.run([gxx, "-O2", "-std=c++17", os.path.join(ROOT, "tests", "host", "tridiag_eig_check.cpp"),
                        "-o", exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    cases = _cases()
    inp = []
    for d, e in cases:
        inp.append(str(d.size))
        inp += [repr(float(x)) for x in d] + [repr(float(x)) for x in e]
    r = subprocess.run([exe], input="\n".join(inp) + "\n", capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    vals = np.array([float(x) for x in r.stdout.split()])
    pos = 0
    for d, e in cases:
        n = d.size
        w = vals[pos:pos + n]
        v = vals[pos + n:pos + n + n * n].reshape(n, n)
        pos += n + n * n
        A = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        scale = max(1.0, np.abs(A).max())
        ref = np.linalg.eigvalsh(A)
        assert np.abs(np.sort(w) - ref).max() <= 1e-13 * scale * max(1.0, np.sqrt(n)), n
        assert np.abs(A @ v - v * w).max() <= 1e-13 * scale, n          # A v_l = w_l v_l
        assert np.abs(v.T @ v - np.eye(n)).max() <= 1e-13 * max(1.0, np.sqrt(n)), n
    assert pos == vals.size
