// Vector kernels on [dim][nvec] blocks: Majorana action, FP64 reductions,
// Gram-Schmidt updates and basis combinations.
#pragma once

#include <complex>
#include <vector>

#include "handle.hpp"

namespace syk {

using zd = std::complex<double>;

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
    // host [K][nvec]: <V_k | w> per column, V_k = V + k * vec_bytes.
    std::vector<zd> multidot(const void* V, int K, const void* w);
    // host [nvec]: ||a||^2 per column.
    std::vector<double> norm2(const void* a);
    // w -= sum_k coef[k][c] V_k; returns ||w||^2 per column if want_norm.
    std::vector<double> update(void* w, const void* V, int K, const std::vector<zd>& coef, bool want_norm);
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
