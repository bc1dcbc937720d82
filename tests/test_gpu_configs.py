"""The workload schedules at their stated sizes and the boundary's failure
modes, through the C-ABI, against the CPU checker.

* Finite-beta G(t) (main text Eq. 2-3, typical state as in the SI section
  "Disorder averaging") in the full space against the checker's estimator.
* The N = 32 OTOC (beta J = 10, Lanczos m = 30, dt = 0.05) out to t = 15
  against checker values stored in tests/golden/otoc_beta10_n32.txt, and its
  full 31-point grid t in [0, 15] at N = 20 against the checker directly.
* The Lyapunov rescaling tool (main text "Lyapunov exponent of the SYK model";
  SI finite-size extrapolation) on OTOC curves the GPU produced, against the
  same tool on the checker's curves.
* Failure modes: overlapping buffers, a NaN in the state, a tolerance below
  the step error, a workspace cap, and gradient degrees above the per-call
  pair limit.

Tolerances: 1e-10 relative for complex128 results (max_t |dF| / max_t |F|).
"""
import ctypes
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sps
import torch

from oracle import chebyshev, correlators, jw, krylov, native
from paper_2002_05725_amd import _lib, api, inputs, rescaling

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(msg):
    print(f"[gpu-configs] {msg}", file=sys.stderr, flush=True)


def _gpu(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV).to(dtype)


def _dense_exp(N, J):
    """Exact exponentials from the checker's own sparse H (plain_apply.c), made dense."""
    sp = native.SparseH(N, J)
    H = sps.csr_matrix((sp.vals, sp.cols, sp.row_ptr), shape=(sp.D, sp.D)).toarray()
    return krylov.DenseExp(H)


# ------------------------------------------------------- finite-beta G(t)
@pytest.mark.parametrize("N,beta", [(12, 3.0), (12, 10.0), (16, 3.0), (16, 10.0)])
def test_two_point_finite_beta_vs_checker(N, beta):
    """syk_two_point at beta > 0 in the full space: G(t) and Z against the
    checker's estimator with exact exponentials on the same state."""
    _say(f"two_point N={N} beta={beta}")
    J = inputs.couplings(N, 0)
    psi = inputs.typical_state(N, 1)
    times = [0.0, 0.4, 1.5, 3.0, 6.0]
    T = api.Terms(N, J)
    G, Z = api.two_point(T, 0, beta, times, _gpu(psi), m=20, dt=0.25, tau_step=0.25)
    maj = lambda a, v: native.majorana(N, a, v)
    Gr, Zr = correlators.two_point_estimator(correlators.ExactPropagator(_dense_exp(N, J)), maj, psi, 0, beta,
                                             times)
    assert np.abs(G[:, 0] - Gr).max() <= 1e-10 * np.abs(Gr).max()
    assert abs(Z[0] - Zr) <= 1e-10 * Zr
    assert abs(G[0, 0] - 0.5) <= 1e-13
    T.close()


# ------------------------------------------------- the N = 32 OTOC to t = 15
def test_otoc_beta10_n32_long_times():
    """N=32, beta J = 10, m = 30, dt = 0.05 on the GPU out to t = 15 against
    the checker's values (tests/golden/make_otoc_beta10_n32.py: its Lanczos on its
    sparse H with dt = 0.5, each time propagated from scratch)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "otoc_beta10_n32.txt"))
    times, Fr, Fir, Zr = rows[:, 0], rows[:, 1], rows[:, 2], rows[:, 3]
    N = 32
    _say("otoc N=32 to t=15")
    T = api.Terms(N, inputs.couplings(N, 0))
    F, Fi, Z = api.otoc(T, 0, 1, 10.0, times, _gpu(inputs.typical_state(N, 1)), m=30, dt=0.05, tau_step=0.625)
    scale = np.abs(Fr).max()
    assert np.abs(F[:, 0] - Fr).max() <= 1e-10 * scale
    assert np.abs(Fi[:, 0] - Fir).max() <= 1e-10 * scale
    assert abs(Z[0] - Zr[0]) <= 1e-10 * Zr[0]
    T.close()


def test_otoc_beta10_full_grid_n20():
    """The N = 32 schedule's full output grid (t = 0, 0.5, ..., 15; beta J = 10;
    m = 30) at N = 20, where the checker can propagate every point from
    scratch: GPU (dt = 0.25) against the checker's Lanczos (dt = 0.5) on its
    sparse H."""
    N = 20
    J = inputs.couplings(N, 0)
    psi = inputs.typical_state(N, 1)
    times = np.round(np.arange(31) * 0.5, 10)
    T = api.Terms(N, J)
    _say("otoc N=20 31-point grid: GPU")
    F, Fi, Z = api.otoc(T, 0, 1, 10.0, times, _gpu(psi), m=30, dt=0.25, tau_step=0.625)
    _say("otoc N=20 31-point grid: checker")
    prop = correlators.Propagator(native.SparseH(N, J), 30, 0.5, 0.625)
    maj = lambda a, v: native.majorana(N, a, v)
    Fr, Fir, Zr = correlators.otoc_estimator(prop, maj, psi, 0, 1, 10.0, times)
    scale = np.abs(Fr).max()
    assert np.abs(F[:, 0] - Fr).max() <= 1e-10 * scale
    assert np.abs(Fi[:, 0] - Fir).max() <= 1e-10 * scale
    assert abs(Z[0] - Zr) <= 1e-10 * Zr
    T.close()


# ----------------------------------------- rescaling on GPU-produced curves
def test_rescaling_on_gpu_curves_matches_checker_curves():
    """OTOC curves (beta = 2, t = 0 .. 6) for N = 12, 16, 20 from syk_otoc,
    then crossing times, lambda_fit(N) and the 1/N extrapolation; the same
    analysis on the checker's curves (exact exponentials on the same states)
    must give the same numbers to 1e-8."""
    times = np.round(np.arange(25) * 0.25, 10)
    gpu_curves, ref_curves = {}, {}
    for N in (12, 16, 20):
        _say(f"rescaling curves N={N}")
        J = inputs.couplings(N, 0)
        psi = inputs.typical_state(N, 1)
        T = api.Terms(N, J)
        F, _, _ = api.otoc(T, 0, 1, 2.0, times, _gpu(psi), m=20, dt=0.25, tau_step=0.25)
        T.close()
        gpu_curves[N] = (times, F[:, 0])
        maj = lambda a, v, N=N: native.majorana(N, a, v)
        Fr, _, _ = correlators.otoc_estimator(correlators.ExactPropagator(_dense_exp(N, J)), maj, psi, 0, 1, 2.0,
                                              times)
        ref_curves[N] = (times, Fr)
        assert np.abs(F[:, 0] - Fr).max() <= 1e-10 * np.abs(Fr).max()
    for F0, cubic in ((0.25, False), (0.5, True)):
        a = rescaling.lyapunov(gpu_curves, F0=F0, degree=1, cubic=cubic)
        b = rescaling.lyapunov(ref_curves, F0=F0, degree=1, cubic=cubic)
        for N in (12, 16, 20):
            assert abs(a["tstar"][N] - b["tstar"][N]) <= 1e-8
        assert np.abs(np.array(a["lambda_fit"]) - np.array(b["lambda_fit"])).max() <= 1e-8
        assert abs(a["lambda_0"] - b["lambda_0"]) <= 1e-8 * max(1.0, abs(b["lambda_0"]))


# ------------------------------------------------------------ failure modes
def _raw_handle(T):
    return T.handle


def test_overlapping_buffers_rejected():
    N = 12
    T = api.Terms(N, inputs.couplings(N, 0))
    x = _gpu(np.stack([inputs.typical_state(N, 1)] * 2))
    L = _lib.lib()
    p = x.data_ptr()
    assert L.syk_apply_H(_raw_handle(T), _lib.SYK_C128, 1, None, ctypes.c_void_p(p), ctypes.c_void_p(p + 16),
                         None) == _lib.SYK_EINVAL
    assert b"overlap" in L.syk_last_error()
    assert L.syk_apply_majorana(_raw_handle(T), _lib.SYK_C128, 3, 1, ctypes.c_void_p(p), ctypes.c_void_p(p),
                                None) == _lib.SYK_EINVAL
    # the handle still works
    y = api.apply_H(T, x[0].contiguous()).cpu().numpy()
    ref = native.apply_full(N, inputs.couplings(N, 0), inputs.typical_state(N, 1))
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
    T.close()


@pytest.mark.parametrize("N", [12, 36])
def test_empty_requests_and_degenerate_values(N):
    """Empty requests are rejected (no columns, no time points, descending
    times, i == j); a propagation by zero leaves the state bit for bit; and at
    beta = 0, t = 0 the estimators take their closed forms on any normalized
    state: chi_i chi_j chi_i chi_j = -chi_i^2 chi_j^2 = -1/4 (i != j) gives
    F = -1/4, chi_i^2 = 1/2 gives G = 1/2, and Z = 1."""
    T = api.Terms(N, inputs.couplings(N, 0))
    psi = inputs.typical_state(N, 1)
    x = _gpu(psi)
    y = torch.empty_like(x)
    L = _lib.lib()
    assert L.syk_apply_H(_raw_handle(T), _lib.SYK_C128, 0, None, ctypes.c_void_p(x.data_ptr()),
                         ctypes.c_void_p(y.data_ptr()), None) == _lib.SYK_EINVAL
    for bad in ([], [1.0, 0.5]):
        with pytest.raises(_lib.SykError):
            api.otoc(T, 0, 1, 0.0, bad, x)
    with pytest.raises(_lib.SykError):
        api.otoc(T, 2, 2, 0.0, [0.0], x)
    z = x.clone()
    api.krylov_expmv(T, z, -1j, 0.0)
    assert torch.equal(z, x)
    for dt, tol in ((torch.complex128, 1e-13), (torch.complex64, 1e-6)):
        xs = _gpu(psi, dt)
        F, Fi, Z = api.otoc(T, 0, 1, 0.0, [0.0], xs)
        assert abs(F[0, 0] + 0.25) <= tol and abs(Fi[0, 0]) <= tol and abs(Z[0] - 1.0) <= 10 * tol
        G, Zg = api.two_point(T, 3, 0.0, [0.0], xs)
        assert abs(G[0, 0] - 0.5) <= tol and abs(Zg[0] - 1.0) <= 10 * tol
    T.close()


def test_nan_state_is_a_breakdown():
    N = 12
    T = api.Terms(N, inputs.couplings(N, 0))
    psi = inputs.typical_state(N, 1)
    psi[17] = np.nan
    x = _gpu(psi)
    with pytest.raises(_lib.SykError) as e:
        api.krylov_expmv(T, x, -1j, 0.5, m=10, dt=0.25)
    assert e.value.status == _lib.SYK_EBREAKDOWN
    with pytest.raises(_lib.SykError) as e:
        api.otoc(T, 0, 1, 1.0, [0.0, 0.5], x, m=10, dt=0.25, tau_step=0.25)
    assert e.value.status == _lib.SYK_EBREAKDOWN
    T.close()


def test_tolerance_below_step_error_is_not_converged():
    """A long step with few basis vectors has a large a-posteriori error: with
    tol below it the call returns SYK_ENOTCONVERGED (the result still written);
    with tol above it, SYK_OK and the same result."""
    N = 12
    J = inputs.couplings(N, 0)
    T = api.Terms(N, J)
    psi = inputs.typical_state(N, 1)
    x = _gpu(psi)
    err = api.krylov_expmv(T, x, -1j, 2.0, m=4, dt=2.0)
    assert err[0] > 1e-6
    y = x.cpu().numpy()
    x2 = _gpu(psi)
    with pytest.raises(_lib.SykError) as e:
        api.krylov_expmv(T, x2, -1j, 2.0, m=4, dt=2.0, tol=err[0] / 10)
    assert e.value.status == _lib.SYK_ENOTCONVERGED
    assert np.array_equal(x2.cpu().numpy(), y)
    x3 = _gpu(psi)
    api.krylov_expmv(T, x3, -1j, 2.0, m=4, dt=2.0, tol=err[0] * 10)
    assert np.array_equal(x3.cpu().numpy(), y)
    with pytest.raises(_lib.SykError) as e:
        api.otoc(T, 0, 1, 1.0, [0.0, 2.0], _gpu(psi), m=4, dt=2.0, tau_step=1.0, tol=1e-12)
    assert e.value.status == _lib.SYK_ENOTCONVERGED
    T.close()


def test_workspace_cap_gives_enomem_and_handle_survives():
    N = 16
    J = inputs.couplings(N, 0)
    T = api.Terms(N, J)
    psi = _gpu(inputs.typical_state(N, 1))
    api.set_workspace_limit(T, 4096)
    with pytest.raises(_lib.SykError) as e:
        api.otoc(T, 0, 1, 2.0, [0.0, 1.0], psi, m=16, dt=0.25, tau_step=0.25)
    assert e.value.status == _lib.SYK_ENOMEM
    assert b"cap" in _lib.lib().syk_last_error()
    api.set_workspace_limit(T, 0)
    F, _, _ = api.otoc(T, 0, 1, 2.0, [0.0, 1.0], psi, m=16, dt=0.25, tau_step=0.25)
    T2 = api.Terms(N, J)
    F2, _, _ = api.otoc(T2, 0, 1, 2.0, [0.0, 1.0], psi, m=16, dt=0.25, tau_step=0.25)
    assert np.array_equal(F, F2)
    T.close()
    T2.close()


def test_gradient_degree_above_pair_limit():
    """Degree 65 and 80: the reverse sweep hands more (g, v) pairs to the
    per-coupling reductions than one call takes, so they run in batches; every
    coupling against the checker's forward-mode tangents."""
    N = 8
    J = inputs.couplings(N, 0)
    H = jw.dense_H(N, J)
    ev = np.linalg.eigvalsh(H)
    e_h = 1.1 * max(abs(ev[0]), abs(ev[-1]))
    psi = inputs.typical_state(N, 1)
    T = api.Terms(N, J)
    chis = jw.dense_majoranas(N)
    maj = lambda a, v: jw.majorana_apply(N, a, v)
    mvJ = lambda Jx: (lambda v, Hx=jw.dense_H(N, Jx, chis): Hx @ v)
    qmv = lambda k: (lambda v, Q=jw.dense_quartet(N, k, chis): Q @ v)
    for degree in (65, 80):
        o = api.cheb_opts(degree=degree, dt=0.1, tau_steps=1, checkpoint_every=4, e_halfwidth=e_h)
        F, g = api.grad_couplings(T, 0, 1, 2.0, 0.3, _gpu(psi), o)
        Fo, go = chebyshev.gradient_tangent(mvJ, qmv, J, maj, psi, 0, 1, 2.0, 0.3, 0.1, 0.0, e_h, degree,
                                            list(range(len(J))), tau_steps=1)
        assert abs(F - Fo) <= 1e-12
        assert np.abs(g - go).max() <= 1e-10 * max(1.0, np.abs(go).max())
    T.close()
