"""apply_H in every launch shape the autotuner may pick, against the checker,
and the autotuner itself: it installs the fastest shape, caches it, and a
cached entry is installed without timing."""
import numpy as np
import pytest
import torch

from oracle import native
from paper_2002_05725_amd import api, autotune, inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("N", [24, 36])
def test_every_candidate_shape_matches_checker(N):
    """Each (tile_bits, xcd order) candidate, complex128 and complex64; N=36
    runs the masks in two row layouts (row-sampled reference)."""
    J = inputs.couplings(N, 0)
    psi = inputs.typical_state(N, 1)
    T = api.Terms(N, J)
    if N <= 28:
        rows = np.arange(psi.size)
        ref = native.apply_full(N, J, psi)
    else:
        rows = np.unique(np.concatenate([inputs.row_sample(N, 23, 2048), [0, 255, 256, 2047, 2048, psi.size - 1]]))
        ref = native.apply_rows(N, J, psi, rows)
    idx = torch.from_numpy(rows).to(DEV)
    for tb, xr, _ in autotune.candidates(N):
        api.set_apply_tuning(T, tb, xr, 1)
        for dt, tol in ((torch.complex128, 1e-12), (torch.complex64, 2e-6)):
            print(f"N={N} tile_bits={tb} xcd_remap={xr} {dt}", flush=True)
            y = api.apply_H(T, torch.from_numpy(psi).to(DEV).to(dt))
            got = y[idx].cpu().numpy().astype(np.complex128)
            assert _rel(got, ref) <= tol, (tb, xr, dt)
    T.close()


def test_tune_installs_fastest_and_caches(tmp_path):
    N = 32
    T = api.Terms(N, inputs.couplings(N, 0))
    cache = str(tmp_path / "tune.json")
    best = autotune.tune_apply(T, torch.complex64, nvec=4, reps=2, cache=cache)
    assert len(best["timed"]) == len(autotune.candidates(N, 4))
    assert best["ms"] == min(r["ms"] for r in best["timed"]) and best["ms"] > 0
    # the installed shape gives the same product as the default one
    x = torch.from_numpy(np.stack([inputs.typical_state(N, s) for s in range(4)])).to(DEV).to(torch.complex64)
    y_tuned = api.apply_H(T, x).cpu().numpy()
    api.set_apply_tuning(T, 0, 1)
    y_def = api.apply_H(T, x).cpu().numpy()
    assert _rel(y_tuned, y_def) <= 2e-6
    # a second call installs the cached entry without timing
    again = autotune.tune_apply(T, torch.complex64, nvec=4, reps=2, cache=cache)
    assert again == autotune.read_cache(cache)[autotune.cache_key(autotune._arch(), N, torch.complex64, 4)]
    assert ((again["tile_bits"], again["xcd_remap"], again["cols_per_group"]) ==
            (best["tile_bits"], best["xcd_remap"], best["cols_per_group"]))
    T.close()
