"""Fermion-parity sectors on the GPU against the checker on the embedded
full-space states (a sector state u stands for the full row
u + 2^(M-1) (parity(u) ^ s); jw.sector_rows)."""
import sys

import numpy as np
import pytest
import torch

from oracle import correlators, jw, krylov, native
from paper_2002_05725_amd import api, inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-sector] {msg}", file=sys.stderr, flush=True)


def _gpu(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda").to(dtype)


def _sector_state(N, s, seed):
    """A normalized Gaussian state of sector s (the typical state restricted
    to the sector rows, renormalized)."""
    psi = inputs.typical_state(N, seed)[jw.sector_rows(N, s)]
    return psi / np.linalg.norm(psi)


def _embed(N, s, u):
    full = np.zeros(1 << (N // 2), dtype=np.complex128)
    full[jw.sector_rows(N, s)] = u
    return full


@pytest.mark.parametrize("N", [8, 10, 12, 14])
@pytest.mark.parametrize("s", [0, 1])
def test_sector_apply_equals_dense_block(N, s):
    J = inputs.couplings(N, 0)
    rows = jw.sector_rows(N, s)
    Hs = jw.dense_H(N, J)[np.ix_(rows, rows)]
    u = _sector_state(N, s, 3)
    T = api.Terms(N, J)
    out = api.apply_H(T, _gpu(u), sector=s).cpu().numpy()
    ref = Hs @ u
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("N", [20, 24, 28])
def test_sector_apply_vs_checker(N):
    """Both sectors, complex128 and complex64, against the checker's
    term-by-term apply on the embedded state (its sector rows)."""
    J = inputs.couplings(N, 0)
    T = api.Terms(N, J)
    for s in (0, 1):
        _say(f"apply sector {s} N={N}")
        u = _sector_state(N, s, 5)
        ref = native.apply_full(N, J, _embed(N, s, u))[jw.sector_rows(N, s)]
        out = api.apply_H(T, _gpu(u), sector=s).cpu().numpy()
        assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
        o64 = api.apply_H(T, _gpu(u, torch.complex64), sector=s).cpu().numpy()
        assert np.abs(o64 - ref).max() <= 2e-6 * np.abs(ref).max()


@pytest.mark.parametrize("N", [40, 52])
def test_sector_apply_rows_large(N):
    """Sampled rows of the sector apply against the checker's rows of the
    full-space apply on the embedded state."""
    J = inputs.couplings(N, 0)
    T = api.Terms(N, J)
    s = 1
    _say(f"sector apply N={N}")
    rows = jw.sector_rows(N, s)
    u = _sector_state(N, s, 9)
    out = api.apply_H(T, _gpu(u), sector=s).cpu().numpy()
    full = _embed(N, s, u)
    del u
    rng = np.random.default_rng(N)
    pick = np.concatenate((np.arange(8), rng.choice(rows.size, 56, replace=False), [rows.size - 1]))
    ref = native.apply_rows(N, J, full, rows[pick])
    assert np.abs(out[pick] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("N", [10, 12])
def test_sector_majoranas(N):
    """chi_a maps sector s to 1 - s: every a, both sectors, against the dense map."""
    rows = [jw.sector_rows(N, 0), jw.sector_rows(N, 1)]
    chis = jw.dense_majoranas(N)
    T = api.Terms(N, inputs.couplings(N, 0))
    for s in (0, 1):
        u = _sector_state(N, s, 4)
        for a in range(N):
            out = api.apply_majorana(T, a, _gpu(u), sector=s).cpu().numpy()
            ref = chis[a][np.ix_(rows[1 - s], rows[s])] @ u
            assert np.abs(out - ref).max() <= 1e-14


@pytest.mark.parametrize("N,beta", [(12, 0.0), (12, 6.0), (16, 3.0)])
def test_sector_correlators_vs_exact(N, beta):
    """OTOC (regularized and not), G(t) and G(tau) of a sector state equal the
    checker's full-space estimators on the embedded state."""
    J = inputs.couplings(N, 0)
    T = api.Terms(N, J)
    E = krylov.DenseExp(jw.dense_H(N, J))
    ex = correlators.ExactPropagator(E)
    maj = lambda a, v: jw.majorana_apply(N, a, v)
    times, taus = [0.0, 0.5, 1.5, 3.0], [0.0, 0.4 * beta, beta]
    for s in (0, 1):
        u = _sector_state(N, s, 1)
        psi = _embed(N, s, u)
        F, Fi, Z = api.otoc(T, 0, 1, beta, times, _gpu(u), m=20, dt=0.25, tau_step=0.25, sector=s)
        Fr, Fir, Zr = correlators.otoc_estimator(ex, maj, psi, 0, 1, beta, times)
        assert np.abs(F[:, 0] - Fr).max() <= 1e-10 * np.abs(Fr).max()
        assert np.abs(Fi[:, 0] - Fir).max() <= 1e-10 * np.abs(Fr).max()
        assert abs(Z[0] - Zr) <= 1e-10 * Zr
        Fu, Fui, _ = api.otoc_unregularized(T, 2, 3, beta, times, _gpu(u), m=20, dt=0.25, tau_step=0.25, sector=s)
        Fur, Fuir, _ = correlators.otoc_u_estimator(ex, maj, psi, 2, 3, beta, times)
        sc = np.abs(Fur + 1j * Fuir).max()
        assert np.abs(Fu[:, 0] - Fur).max() <= 1e-10 * sc and np.abs(Fui[:, 0] - Fuir).max() <= 1e-10 * sc
        G, Zg = api.two_point(T, 1, beta, times, _gpu(u), m=20, dt=0.25, tau_step=0.25, sector=s)
        Gref, Zgr = correlators.two_point_estimator(ex, maj, psi, 1, beta, times)
        assert np.abs(G[:, 0] - Gref).max() <= 1e-10 * np.abs(Gref).max()
        assert abs(Zg[0] - Zgr) <= 1e-10 * Zgr
        if beta > 0:
            Gt, _ = api.imag_two_point(T, 5, beta, taus, _gpu(u), m=20, tau_step=0.25, sector=s)
            Gtr, _ = correlators.imag_two_point_estimator(ex, maj, psi, 5, beta, taus)
            assert np.abs(Gt[:, 0] - Gtr).max() <= 1e-10 * np.abs(Gtr).max()


def test_sector_krylov_and_blocks():
    """e^{-iHt} of sector states (a block of two realisations) against the
    exact exponential of the embedded states, and block calls against single
    columns."""
    N = 16
    Js = np.stack([inputs.couplings(N, 30 + r) for r in range(2)])
    T = api.Terms(N, Js)
    s = 0
    us = np.stack([_sector_state(N, s, 40 + c) for c in range(4)])
    real = [0, 1, 0, 1]
    x = _gpu(us)
    api.krylov_expmv(T, x, -1j, 1.3, m=20, dt=0.2, real_of_col=real, sector=s)
    got = x.cpu().numpy()
    rows = jw.sector_rows(N, s)
    for c in range(4):
        E = krylov.DenseExp(jw.dense_H(N, Js[real[c]]))
        ref = E.apply(_embed(N, s, us[c]), -1.3j)[rows]
        assert np.abs(got[c] - ref).max() <= 1e-11
    F, _, _ = api.otoc(T, 0, 3, 2.0, [0.0, 0.8], _gpu(us), m=16, dt=0.2, tau_step=0.25, real_of_col=real, sector=s)
    for c in range(4):
        Tc = api.Terms(N, Js[real[c]])
        F1, _, _ = api.otoc(Tc, 0, 3, 2.0, [0.0, 0.8], _gpu(us[c]), m=16, dt=0.2, tau_step=0.25, sector=s)
        assert np.abs(F[:, c] - F1[:, 0]).max() <= 1e-12
