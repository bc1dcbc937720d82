// Krylov (Lanczos) propagation on top of apply_H.
#pragma once

#include <complex>
#include <vector>

#include "apply_h.hpp"
#include "vec.hpp"

namespace syk {

// Everything a propagation needs for one block of columns.  With sector >= 0
// the states live in a fermion-parity sector (2^(M-1) rows): apply_H uses the
// tables of the active sector (at()), and chi maps a sector to the other.
struct BlockCtx {
    syk_terms_s& h;
    syk_dtype dtype;
    int nvec;
    const int32_t* real_of_col;   // host or NULL
    hipStream_t stream;
    int sector0;                  // sector of the input states, -1 for the full space
    const HamiltonianDev* Hact;   // tables apply_H uses
    ApplyPlan plan;
    VecOps ops;

    BlockCtx(syk_terms_s& h_, syk_dtype dt, int nvec_, const int32_t* real, hipStream_t s, int sector = -1);
    int64_t dim() const { return (int64_t)1 << Hact->M; }
    void apply_H(const void* in, void* out);
    // apply_H acts in sector s from now on (nothing in the full space)
    void at(int s);
    // out = chi_a in for states of sector s_in (-1: the full space); out is in sector 1 - s_in
    void majorana(int a, int s_in, const void* in, void* out);
    // the sector opposite to s (-1 stays -1)
    static int other(int s) { return s < 0 ? -1 : 1 - s; }
};

struct KrylovStats {
    std::vector<double> err;   // largest step error estimate per column
    int steps = 0;
};

// Lanczos basis of one step: V (m vectors of the block, workspace), the
// tridiagonal T per column (alpha: diagonal, beta: off-diagonal, [m][nvec]),
// the Krylov dimension per column (< m after an invariant subspace) and ||psi||.
struct LanczosBasis {
    int m = 0;
    char* V = nullptr;
    std::vector<double> alpha, beta, nrm;
    std::vector<int> kdim;
};
LanczosBasis lanczos_build(BlockCtx& c, const void* psi, int m);
void ritz_values(const LanczosBasis& L, int col, int nvec, std::vector<double>& ev, std::vector<double>& S);

// Smallest and largest Ritz values of m Lanczos steps from psi (one column).
void lanczos_extremes(BlockCtx& c, const void* psi, int m, double* emin, double* emax);

// The k lowest Ritz values of m Lanczos steps from psi (one column), ascending,
// and their residual norms beta_m |s_m,i| (res_out may be NULL).  Returns how
// many were written (fewer than k when the Krylov space became invariant).
int lowest_eigenvalues(BlockCtx& c, const void* psi, int m, int k, double* ev_out, double* res_out);

// psi <- exp(z H) psi per column with one Lanczos step of m vectors.
void krylov_step(BlockCtx& c, void* psi, std::complex<double> z, int m, KrylovStats& st);

// psi <- exp(total * z H) psi in ceil(total / step) equal steps (total >= 0).
void krylov_propagate(BlockCtx& c, void* psi, std::complex<double> z, double total, double step, int m,
                      KrylovStats& st);

}  // namespace syk
