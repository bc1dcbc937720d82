// Typical-state correlators built on the Krylov propagator.
#pragma once

#include "krylov.hpp"

namespace syk {

// G[k][c] (re, im) = <psi|rho^{1/2} chi_i(t_k) chi_i rho^{1/2}|psi> / Z_c
void two_point(BlockCtx& c, int i, double beta, const double* t, int nt, const void* psi0,
               const syk_krylov_opts& o, double* G, double* Z);

// F[k][c] = Re <A^dag psi|A psi> / <psi|rho|psi>, A = rho^{1/8} chi_i(t) rho^{1/4} chi_j rho^{1/8}
void otoc(BlockCtx& c, int i, int j, double beta, const double* t, int nt, const void* psi0,
          const syk_krylov_opts& o, double* F, double* F_im, double* Z);

// F[k][c] + i F_im[k][c] = <V W phi|W V phi> / <phi|phi>, W = chi_i(t_k), V = chi_j, phi = rho^{1/2} psi
void otoc_unregularized(BlockCtx& c, int i, int j, double beta, const double* t, int nt, const void* psi0,
                        const syk_krylov_opts& o, double* F, double* F_im, double* Z);

// G[k][c] = ||e^{-tau_k H/2} chi_i e^{-(beta - tau_k) H/2} psi||^2 / <psi|rho|psi>
void imag_two_point(BlockCtx& c, int i, double beta, const double* tau, int ntau, const void* psi0,
                    const syk_krylov_opts& o, double* G, double* Z);

}  // namespace syk
