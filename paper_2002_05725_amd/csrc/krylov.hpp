// Krylov (Lanczos) propagation on top of apply_H.
#pragma once

#include <complex>
#include <vector>

#include "apply_h.hpp"
#include "vec.hpp"

namespace syk {

// Everything a propagation needs for one block of columns.
struct BlockCtx {
    syk_terms_s& h;
    syk_dtype dtype;
    int nvec;
    const int32_t* real_of_col;   // host or NULL
    hipStream_t stream;
    ApplyPlan plan;
    VecOps ops;

    BlockCtx(syk_terms_s& h_, syk_dtype dt, int nvec_, const int32_t* real, hipStream_t s);
    int64_t dim() const { return (int64_t)1 << h.H.M; }
    void apply_H(const void* in, void* out);
};

struct KrylovStats {
    std::vector<double> err;   // largest step error estimate per column
    int steps = 0;
};

// Eigen-decomposition of a real symmetric n x n matrix (row-major a, destroyed):
// eigenvalues in w, eigenvectors as columns of v (row-major n x n).
void symmetric_eig(int n, std::vector<double>& a, std::vector<double>& w, std::vector<double>& v);

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
