// Vector kernels on [dim][nvec] blocks: Majorana action, FP64 reductions,
// Gram-Schmidt updates and basis combinations.
#pragma once

#include <complex>
#include <vector>

#include "handle.hpp"

namespace syk {

using zd = std::complex<double>;

// Device arrays of one Lanczos build (see VecOps::lanczos_coef): alpha and
// beta [m][nvec], per column kdim, scale, the start norm nrm and the factor f
// of the next basis vector, and an error flag.
struct LanczosScalars {
    double* alpha;
    double* beta;
    int* kdim;
    double* scale;
    const double* nrm;
    double* f;
    int* flag;
};

class VecOps {
public:
    VecOps(syk_terms_s& h, syk_dtype dt, int64_t dim, int nvec, hipStream_t s);

    size_t vec_bytes() const { return (size_t)dim_ * nvec_ * elem_bytes(dt_); }
    int64_t dim() const { return dim_; }
    int nvec() const { return nvec_; }
    syk_dtype dtype() const { return dt_; }
    hipStream_t stream() const { return s_; }

    // out = chi_a in (SI Jordan-Wigner map, with the 2^{-1/2}).
    void majorana(int a, const void* in, void* out);
    // chi_a between parity sectors: rows u of a sector-s_in state stand for the
    // full rows u + 2^top (parity(u) ^ s_in); out is in sector 1 - s_in
    void majorana_sector(int a, int top, int s_in, const void* in, void* out);
    // Largest basis the fused update_dot serves.
    static constexpr int kFusedMax = 16;

    // host [K][nvec]: <V_k | w> per column, V_k = V + k * vec_bytes.
    std::vector<zd> multidot(const void* V, int K, const void* w);
    // The same left on the device as [K][nvec] (re, im) FP64 pairs in the
    // workspace buffer `slot` (valid until the next use of that slot).
    const double* multidot_dev(const void* V, int K, const void* w, const char* slot);
    // host copy of a [K][nvec] device array of (re, im) pairs.
    std::vector<zd> fetch(const double* dev, int K);
    // w -= sum_k c1[k][c] V_k (c1 on the device, [K][nvec] pairs) in one pass
    // that also forms <V_k | w_new>, returned on the device in `slot`;
    // K <= kFusedMax.
    const double* update_dot(void* w, const void* V, int K, const double* c1, const char* slot);
    // host [nvec]: ||a||^2 per column.
    std::vector<double> norm2(const void* a);
    // w -= sum_k coef[k][c] V_k; returns ||w||^2 per column if want_norm.
    std::vector<double> update(void* w, const void* V, int K, const std::vector<zd>& coef, bool want_norm);
    // the same with the coefficients already on the device ([K][nvec] pairs).
    std::vector<double> update_dev(void* w, const void* V, int K, const double* dcoef, bool want_norm);
    // ... leaving ||w||^2 per column on the device (nullptr without want_norm).
    const double* update_dev_norm(void* w, const void* V, int K, const double* dcoef, bool want_norm);
    // Lanczos iteration j's scalars on the device from the two projections
    // c1, c2 ([K][nvec] pairs) and ||w||^2: alpha_j, beta_j, the invariant-
    // subspace test and the factor f of the next basis vector, per column.
    void lanczos_coef(const double* c1, const double* c2, const double* wnorm2, int j, int m, LanczosScalars& z);
    // out[:, c] = f[c] * in[:, c] with f on the device
    void scale_dev(void* out, const void* in, const double* df);
    // synchronous copies of small arrays
    void to_device(void* dev, const void* host, size_t bytes);
    void to_host(void* host, const void* dev, size_t bytes);
    // out[:, c] = f[c] * in[:, c]   (out may equal in)
    void scale(void* out, const void* in, const std::vector<double>& f);
    // y = sum_k coef[k][c] V_k (FP64 accumulation)
    void combine(void* y, const void* V, int K, const std::vector<zd>& coef);
    void copy(void* dst, const void* src);

private:
    syk_terms_s& h_;
    syk_dtype dt_;
    int64_t dim_;
    int nvec_;
    hipStream_t s_;
    void* upload(const std::vector<zd>& c);
    void* upload(const std::vector<double>& c);
    template <typename T>
    std::vector<T> download(const void* dev, size_t n);
};

}  // namespace syk
