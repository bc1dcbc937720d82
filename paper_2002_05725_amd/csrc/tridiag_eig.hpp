// Eigen-decomposition of a real symmetric tridiagonal matrix (host, FP64).
#pragma once

#include <cfloat>
#include <cmath>
#include <stdexcept>
#include <vector>

namespace syk {

// Diagonal d[0..n), off-diagonal e[0..n-1).  On return w[l] are the
// eigenvalues (unsorted) and column l of v (row-major n x n) is the unit
// eigenvector of w[l].  Implicit symmetric QR steps with the Wilkinson shift
// of the trailing 2 x 2 block, chasing the bulge with Givens rotations that
// are accumulated into v (Golub and Van Loan, Matrix Computations, sec. 8.3);
// an off-diagonal entry at or below DBL_EPSILON (|d_i| + |d_i+1|) splits the
// matrix.  O(n^2) per step for the eigenvectors, about 1.5 steps per
// eigenvalue.  Throws std::runtime_error if 30 n steps do not converge.
inline void tridiag_eig(int n, std::vector<double> d, std::vector<double> e, std::vector<double>& w,
                        std::vector<double>& v)
{
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    e.resize(n > 0 ? n : 1, 0.0);
    auto small = [&](int i) {   // e[i] couples rows i and i + 1
        return std::fabs(e[i]) <= DBL_EPSILON * (std::fabs(d[i]) + std::fabs(d[i + 1])) ||
               std::fabs(e[i]) < DBL_MIN;
    };
    int hi = n - 1, steps = 0;
    while (hi > 0) {
        if (small(hi - 1)) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && !small(lo - 1)) --lo;
        if (++steps > 30 * n) throw std::runtime_error("tridiagonal eigensolver did not converge");
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer d[hi]
        const double dl = 0.5 * (d[hi - 1] - d[hi]);
        const double eh = e[hi - 1];
        const double mu = d[hi] - eh * eh / (dl + std::copysign(std::hypot(dl, eh), dl));
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            // rotation J in the (k, k+1) plane with J (x, z)^T = (r, 0)^T; T <- J T J^T
            const double r = std::hypot(x, z);
            const double c = r > 0.0 ? x / r : 1.0, s = r > 0.0 ? z / r : 0.0;
            if (k > lo) e[k - 1] = r;
            const double a = d[k], b = e[k], f = d[k + 1];
            d[k] = c * c * a + 2.0 * c * s * b + s * s * f;
            d[k + 1] = s * s * a - 2.0 * c * s * b + c * c * f;
            e[k] = c * s * (f - a) + (c * c - s * s) * b;
            if (k + 1 < hi) {   // the bulge at (k, k+2) is the next rotation's target
                x = e[k];
                z = s * e[k + 1];
                e[k + 1] *= c;
            }
            for (int i = 0; i < n; ++i) {   // v <- v J^T
                double* row = &v[(size_t)i * n];
                const double p = row[k], q = row[k + 1];
                row[k] = c * p + s * q;
                row[k + 1] = c * q - s * p;
            }
        }
    }
    w = d;
}

}  // namespace syk
