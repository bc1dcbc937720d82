"""Writes otoc_beta10_n32.txt: the CPU checker's regularized OTOC at N=32.

Workload (regularized OTOC, main text Eq. 4, from one typical state as in the
SI section "Disorder averaging"): N = 32 Majoranas (dim 65,536, 35,960
couplings), couplings seed 0, typical state seed 1, beta J = 10, i = 0, j = 1
(the paper's chi_1, chi_2), t in {0, 5, 10, 15}.

The checker propagates every time from scratch with Lanczos steps of m = 30
basis vectors (SI "Krylov subspace methods") on its sparse H (plain_apply.c):
real-time step 0.5, imaginary-time step 0.625.  Both step sizes keep the
Krylov error far below 1e-12 here, so a propagation with any finer step (the
HIP path uses dt = 0.05) must agree to about that.  Only oracle/ is called.

Run from the repository root:  python tests/golden/make_otoc_beta10_n32.py
(a few minutes on 8 cores).
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import correlators, native  # noqa: E402
from paper_2002_05725_amd import inputs  # noqa: E402

N, BETA, M, DT, TAU = 32, 10.0, 30, 0.5, 0.625
TIMES = [0.0, 5.0, 10.0, 15.0]


def main():
    J = inputs.couplings(N, 0)
    psi = inputs.typical_state(N, 1)
    t0 = time.time()
    sp = native.SparseH(N, J)
    prop = correlators.Propagator(sp, M, DT, TAU)
    maj = lambda a, v: native.majorana(N, a, v)
    rows = []
    for t in TIMES:
        F, Fi, Z = correlators.otoc_estimator(prop, maj, psi, 0, 1, BETA, [t])
        rows.append((t, F[0], Fi[0], Z))
        print(f"t={t}: F={F[0]!r} ({time.time() - t0:.0f} s)", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "otoc_beta10_n32.txt")
    with open(out, "w") as f:
        f.write("# t F F_im Z  (make_otoc_beta10_n32.py: checker Lanczos m=30, dt=0.5, tau_step=0.625, "
                "N=32, beta=10, couplings seed 0, state seed 1, i=0, j=1)\n")
        for r in rows:
            f.write(" ".join(repr(float(x)) for x in r) + "\n")


if __name__ == "__main__":
    main()
