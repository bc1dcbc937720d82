"""CPU checker for the SYK hot path.  TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of what the HIP library
computes, used to prove parity.  It shares no code with the library: no
kernels, headers, tables or helpers.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.

Contents (each module cites the passage of arXiv:2002.05725 it follows):
* ``jw``           -- Jordan-Wigner Majoranas and the dense Hamiltonian (Eq. 1, SI "Jordan-Wigner transformation").
* ``native``       -- plain_apply.c: term-by-term H|psi>, chi_a|psi>, sparse H.
* ``krylov``       -- Lanczos propagation (SI "Krylov subspace methods") and exact exponentials.
* ``correlators``  -- G(t) and the regularized OTOC from a typical state (Eq. 2-4, SI "Disorder averaging").
* ``chebyshev``    -- fixed-degree Chebyshev propagator and its exact derivative in the couplings.

Floating point is FP64 / complex128 throughout.
"""
