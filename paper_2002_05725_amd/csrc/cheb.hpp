// Fixed-degree Chebyshev propagation of the regularized OTOC and its exact
// derivative in every coupling (reverse sweep with checkpoints).
#pragma once

#include <complex>
#include <vector>

#include "grad.hpp"
#include "krylov.hpp"

namespace syk {

struct ChebSettings {
    int degree;            // K: polynomial degree of every step
    double dt;             // real-time step
    int tau_steps;         // steps per imaginary-time leg
    int checkpoint_every;  // stored state every this many operations of a chain
    double e_c, e_h;       // spectrum centre and half-width (fixed: do not move with J)
    int keep_segment;      // keep a segment's Chebyshev vectors for the reverse sweep when memory allows
};

// One operation of a chain: a Chebyshev step with coefficients c, or chi_maj.
struct ChebOp {
    int maj;                                  // -1 for a Chebyshev step
    std::vector<std::complex<double>> c;      // c_0..c_K
};

std::vector<std::complex<double>> cheb_coeffs_real(double h, const ChebSettings& s);  // e^{-i h H}
std::vector<std::complex<double>> cheb_coeffs_imag(double tau, const ChebSettings& s); // e^{-tau H}

// The three chains of the estimator F = Re <B|A> / ||u||^2 (see cheb.cpp).
struct OtocChains {
    std::vector<ChebOp> A, B, U;
};
OtocChains otoc_chains(int i, int j, double beta, double t, const ChebSettings& s);

// F of the Chebyshev forward; with grad != NULL also dF/dJ_n for every coupling
// (host array of C(N,4)).  complex128, one column, realisation 0.
void cheb_otoc(BlockCtx& c, int i, int j, double beta, double t, const ChebSettings& s, const void* psi0,
               double* F, double* grad);

}  // namespace syk
