"""Writes block_n36_otoc.txt: the CPU checker's regularized OTOC for one column
of the N=36 disorder-averaging block.

Workload (regularized OTOC, main text Eq. 4, from one typical state as in the
SI section "Disorder averaging"): N = 36 Majoranas (dim 262,144, 58,905
couplings), the block's realisation r = 18 (couplings seed
inputs.batch_coupling_seed(36, 18)) and its second typical state (seed
inputs.batch_state_seed(36, 18, 1)), i.e. column 37 of the 64-column block;
beta J = 5, i = 0, j = 1, t in {0, 6}.

The checker propagates each time from scratch with Lanczos steps of m = 16
basis vectors (SI "Krylov subspace methods") on its explicit sparse H
(plain_apply.c; about 20 GB at this size): real-time step 0.5, imaginary-time
step 0.625, the block test's own parameters, so the two sides differ only in
rounding.  Only oracle/ is called.

Run from the repository root:  python tests/golden/make_block_n36.py
(about half an hour on 8 cores, 24 GB of memory).
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import correlators, native  # noqa: E402
from paper_2002_05725_amd import inputs  # noqa: E402

N, R, S, BETA, M, DT, TAU = 36, 18, 1, 5.0, 16, 0.5, 0.625
TIMES = [0.0, 6.0]


def main():
    J = inputs.couplings(N, inputs.batch_coupling_seed(N, R))
    psi = inputs.typical_state(N, inputs.batch_state_seed(N, R, S))
    t0 = time.time()
    sp = native.SparseH(N, J)
    print(f"sparse H built ({time.time() - t0:.0f} s)", flush=True)
    prop = correlators.Propagator(sp, M, DT, TAU)
    maj = lambda a, v: native.majorana(N, a, v)
    rows = []
    for t in TIMES:
        F, Fi, Z = correlators.otoc_estimator(prop, maj, psi, 0, 1, BETA, [t])
        rows.append((t, F[0], Fi[0], Z))
        print(f"t={t}: F={F[0]!r} ({time.time() - t0:.0f} s)", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "block_n36_otoc.txt")
    with open(out, "w") as f:
        f.write("# t F F_im Z  (make_block_n36.py: checker Lanczos m=16, dt=0.5, tau_step=0.625, N=36, beta=5, "
                "realisation 18 (couplings seed batch_coupling_seed(36, 18)), state seed batch_state_seed(36, 18, 1), "
                "i=0, j=1)\n")
        for r in rows:
            f.write(" ".join(repr(float(x)) for x in r) + "\n")


if __name__ == "__main__":
    main()
