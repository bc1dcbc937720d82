"""Largest single-GPU size: N=60 (dim 2^30, 487,635 couplings, 16 GiB per
complex128 state).  One apply_H in each precision, checked on sampled rows
against the checker's term-by-term sum, and one Lanczos step with m = 2."""
import sys
import time

import numpy as np
import pytest
import torch

from oracle import native
from paper_2002_05725_amd import api, inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(msg):
    print(f"[n60 {time.strftime('%H:%M:%S')}] {msg}", flush=True)
    sys.stdout.flush()


def test_n60_apply_and_lanczos():
    N = 60
    _say("couplings and terms")
    J = inputs.couplings(N, 0)
    T = api.Terms(N, J)
    assert T.dim == 1 << 30 and T.n_terms == 487635 and T.n_masks == 27841
    _say("typical state (16 GiB host)")
    psi = inputs.typical_state(N, 1)
    rows = np.unique(np.concatenate([inputs.row_sample(N, 17, 192), [0, 2047, 2048, (1 << 30) - 1]]))
    _say("checker rows")
    ref = native.apply_rows(N, J, psi, rows)
    idx = torch.from_numpy(rows).to(DEV)

    _say("complex128 apply")
    x = torch.from_numpy(psi).to(DEV)
    y = api.apply_H(T, x)
    torch.cuda.synchronize()
    got = y[idx].cpu().numpy()
    err128 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _say(f"complex128 rows rel err {err128:.2e}")
    assert err128 <= 1e-12
    del y

    _say("Lanczos step, m = 2")
    err = api.krylov_expmv(T, x, -1j, 0.01, m=2, dt=0.01)
    nrm = float(torch.linalg.vector_norm(x))
    _say(f"norm {nrm:.15f}, error estimate {err[0]:.2e}")
    # the projection is unitary; the a-posteriori estimate is first order in dt * beta_1
    assert abs(nrm - 1.0) <= 1e-10 and np.isfinite(err[0]) and err[0] <= 0.05
    del x
    torch.cuda.empty_cache()

    _say("complex64 apply")
    x64 = torch.from_numpy(psi).to(DEV).to(torch.complex64)
    del psi
    y64 = api.apply_H(T, x64)
    torch.cuda.synchronize()
    got64 = y64[idx].cpu().numpy()
    err64 = np.linalg.norm(got64 - ref) / np.linalg.norm(ref)
    _say(f"complex64 rows rel err {err64:.2e}")
    assert err64 <= 2e-6
    del x64, y64
    T.close()
    torch.cuda.empty_cache()
