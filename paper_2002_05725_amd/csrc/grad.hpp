// Chebyshev recurrence kernel and coupling-derivative bins.
#pragma once

#include <complex>
#include <vector>

#include "apply_h.hpp"

namespace syk {

constexpr int kGradBinCap = 2048;   // derivative bins of one chunk held in LDS

// Masks sharing x >> tile_bits, cut so that their bins fit in LDS.
struct alignas(16) GChunk {
    uint32_t x_high, first, count, bin_begin, bin_count, pad[3];
};

std::vector<GChunk> make_grad_chunks(const std::vector<MaskRec>& masks, const std::vector<uint64_t>& bin_off,
                                     uint64_t n_bins, int tile_bits);

// out = b (w - gamma y) + s z + c x ; acc += ca out.  Null pointers drop their term.
void cheb_rec(syk_dtype dtype, int64_t n, void* out, const void* w, const void* y, const void* z, const void* x,
              void* acc, double b, double gamma, double s, std::complex<double> c, std::complex<double> ca,
              hipStream_t st);

// bins_dev (device, n_bins complex) += sum_p w_p * bins of (g_p, v_p); complex128 states.
void grad_bins(syk_terms_s& h, const std::vector<const void*>& g, const std::vector<const void*>& v,
               const std::vector<double>& w, double* bins_dev, hipStream_t st);

}  // namespace syk
