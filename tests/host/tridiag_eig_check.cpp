// Runs the library's tridiagonal eigensolver on matrices read from stdin:
// per case "n", then n diagonal and n-1 off-diagonal values; prints n
// eigenvalues, then the n x n eigenvector matrix (row-major, column l for
// eigenvalue l).
#include <cstdio>
#include <vector>

#include "../../paper_2002_05725_amd/csrc/tridiag_eig.hpp"

int main()
{
    int n;
    while (std::scanf("%d", &n) == 1) {
        std::vector<double> d(n), e(n > 1 ? n - 1 : 0), w, v;
        for (auto& x : d) std::scanf("%lf", &x);
        for (auto& x : e) std::scanf("%lf", &x);
        syk::tridiag_eig(n, d, e, w, v);
        for (double x : w) std::printf("%.17g\n", x);
        for (double x : v) std::printf("%.17g\n", x);
    }
    return 0;
}
