"""Two columns of one realisation per workgroup (syk_set_apply_tuning with
cols_per_group = 2): every column of a block against the checker's
term-by-term product, and against the one-column launch of the same tile
shape bit for bit (both forms add a row's terms in the same order).  Blocks
whose columns do not pair up by realisation, odd blocks and the column slices
of blocks wider than one launch run one column per workgroup."""
import numpy as np
import pytest
import torch

from oracle import native
from paper_2002_05725_amd import api, autotune, inputs
from paper_2002_05725_amd._lib import SykError

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = {torch.complex128: 1e-12, torch.complex64: 2e-6}


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _block(N, R, nvec, seed0):
    Js = np.stack([inputs.couplings(N, seed0 + r) for r in range(R)])
    psis = np.stack([inputs.typical_state(N, seed0 + 100 + c) for c in range(nvec)])
    return Js, psis


def _apply(T, psis, real, dt, tb, xr, nc):
    api.set_apply_tuning(T, tb, xr, nc)
    return api.apply_H(T, torch.from_numpy(psis).to(DEV).to(dt), real_of_col=real).cpu().numpy()


@pytest.mark.parametrize("N", [20, 24])
def test_two_columns_match_checker(N):
    """Four columns, two realisations, every two-column shape, both dtypes:
    each column against the full term-by-term product of its realisation."""
    Js, psis = _block(N, 2, 4, 600)
    real = np.array([0, 0, 1, 1], dtype=np.int32)
    refs = [native.apply_full(N, Js[real[c]], psis[c]) for c in range(4)]
    T = api.Terms(N, Js)
    shapes = [s for s in autotune.candidates(N, 4) if s[2] == 2]
    assert shapes, "no two-column shape at this size"
    for tb, xr, nc in shapes:
        for dt, tol in TOL.items():
            print(f"[pairs] N={N} tile_bits={tb} xcd_remap={xr} {dt}", flush=True)
            y2 = _apply(T, psis, real, dt, tb, xr, 2)
            for c in range(4):
                assert _rel(y2[c].astype(np.complex128), refs[c]) <= tol, (tb, xr, dt, c)
            y1 = _apply(T, psis, real, dt, tb, xr, 1)
            assert np.array_equal(y2, y1), (tb, xr, dt)
    T.close()


def test_two_columns_two_layouts_n36():
    """N=36 runs in two row layouts (the rotated one through its own pair of
    transposes): the two-column block equals the one-column block and each
    column alone, bit for bit, and sampled rows match the checker."""
    N = 36
    Js, psis = _block(N, 2, 4, 700)
    real = np.array([1, 1, 0, 0], dtype=np.int32)
    rows = np.unique(np.concatenate([inputs.row_sample(N, 29, 1024), [0, 1023, 1024, psis.shape[1] - 1]]))
    T = api.Terms(N, Js)
    for tb in (10, 11):
        for dt, tol in TOL.items():
            print(f"[pairs] N=36 tile_bits={tb} {dt}", flush=True)
            y2 = _apply(T, psis, real, dt, tb, 1, 2)
            y1 = _apply(T, psis, real, dt, tb, 1, 1)
            assert np.array_equal(y2, y1), (tb, dt)
            api.set_apply_tuning(T, tb, 1, 1)
            for c in range(4):
                one = api.apply_H(T, torch.from_numpy(psis[c]).to(DEV).to(dt), real_of_col=[real[c]])
                assert np.array_equal(one.cpu().numpy(), y2[c]), (tb, dt, c)
            for c in (0, 3):
                ref = native.apply_rows(N, Js[real[c]], psis[c], rows)
                got = y2[c][rows].astype(np.complex128)
                assert _rel(got, ref) <= tol, (tb, dt, c)
    T.close()


@pytest.mark.parametrize("nvec,real_of", [(66, "pairs"), (67, "pairs"), (6, "unpaired")])
def test_two_columns_slices_and_fallback(nvec, real_of):
    """Blocks wider than one launch (64 columns: slices of 64 and 2 or 3
    columns) and blocks whose neighbours belong to different realisations:
    the two-column setting gives the one-column result bit for bit, and every
    column matches the checker."""
    N, R = 20, 3
    Js, psis = _block(N, R, nvec, 800)
    if real_of == "pairs":
        real = (np.arange(nvec) // 2 % R).astype(np.int32)
    else:
        real = (np.arange(nvec) % R).astype(np.int32)
    T = api.Terms(N, Js)
    for dt, tol in TOL.items():
        print(f"[pairs] N=20 nvec={nvec} {real_of} {dt}", flush=True)
        y2 = _apply(T, psis, real, dt, 10, 1, 2)
        y1 = _apply(T, psis, real, dt, 10, 1, 1)
        assert np.array_equal(y2, y1), (nvec, real_of, dt)
        for c in (0, 1, nvec - 2, nvec - 1):
            ref = native.apply_full(N, Js[real[c]], psis[c])
            assert _rel(y2[c].astype(np.complex128), ref) <= tol, (nvec, real_of, dt, c)
    T.close()


def test_two_columns_tuning_validation():
    """cols_per_group = 2 needs tiles of 2^10 or 2^11 rows: smaller explicit
    tiles are rejected (and the setting kept); automatic tiles fall back."""
    N = 24
    Js, psis = _block(N, 1, 2, 900)
    T = api.Terms(N, Js)
    api.set_apply_tuning(T, 11, 1, 2)
    with pytest.raises(SykError):
        api.set_apply_tuning(T, 9, 1, 2)
    with pytest.raises(SykError):
        api.set_apply_tuning(T, 11, 1, 3)
    api.set_apply_tuning(T, 0, 1, 2)   # automatic tiles: small blocks fall back to one column
    y = api.apply_H(T, torch.from_numpy(psis).to(DEV)).cpu().numpy()
    for c in range(2):
        assert _rel(y[c], native.apply_full(N, Js[0], psis[c])) <= 1e-12
    T.close()
