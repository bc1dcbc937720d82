// Chebyshev recurrence kernel and coupling-derivative bins.
#pragma once

#include <complex>
#include <vector>

#include "apply_h.hpp"

namespace syk {

constexpr int kGradBinCap = 1024;   // derivative bins of one chunk held in LDS
constexpr int kGradAccMasks = 3;    // PAIR / DIAG masks of one chunk, summed over the pairs per row
constexpr int kGradPairsPerStage = 2;   // (g, v) pairs whose source tiles are staged together
constexpr int kGradMaxPairs = 64;        // (g, v) pairs of one grad_bins call
constexpr int kGradTileBits = 9;         // rows of a tile of the bins kernel (fewer for states of fewer rows)
constexpr int kGradTileRows = 1 << kGradTileBits;
constexpr int kGradSrcTiles = 2;         // source tiles (distinct x >> tile_bits) a near chunk may hold
constexpr int kGradPairOutputs = 4 * (kGradTileBits + 1);   // per-tile sums of a PAIR mask (bins kernel)

// A chunk of masks whose bins are held in LDS together: members
// [first, first + count) of the member list, at most kGradAccMasks of them PAIR
// or DIAG masks (their positions in acc).  The masks of a near chunk have one of
// at most kGradSrcTiles values of x >> tile_bits (one staged source tile each;
// bit 30 of a member's koffs says which); their QUAD members come first,
// sorted by row class (mask_classes.hpp) with cnt[] masks per class.  A far
// chunk holds QUAD / PAIR masks that flip no row bit inside a tile, each
// reading its own source tile straight from global memory.  All members of a
// chunk run in one row layout (0: natural, 1: rotated, apply_h.hpp), in whose
// coordinates their records are given.
struct alignas(16) GChunk {
    uint32_t x_high, first, count, bin_count, n_acc, far, n_quad, layout;
    uint32_t acc[kGradAccMasks];
    uint32_t cnt[8];   // QUAD members per class, one byte per class
    uint32_t x_high2;  // near chunks: the second source tile (tile ^ x_high2), if n_src == 2
    uint32_t n_src;    // source tiles a near chunk stages (1 or 2; 0 for far chunks)
};
static_assert(sizeof(GChunk) % 16 == 0, "GChunk layout");

// Per-member record of a QUAD member of a near chunk.
struct alignas(16) GRec {
    uint32_t sel;    // byte selector gathering the lane bits of tid at q0..q3 (0x0c: not a lane bit)
    uint32_t zl;     // lane bits of zbase
    uint32_t xoff;   // x & lane mask: lane part of the source row
    uint32_t koffs;  // byte b < 3: index bit set by k bit b (0 if not flipped); bits 24-29: in-wave lane
                     // bits of x; bit 30: the chunk's source tile the member reads (also for PAIR / DIAG)
};

constexpr int kGradRecPad = 4;   // zero QUAD member records after the last one

struct GradChunks {
    std::vector<GChunk> chunks;
    std::vector<uint32_t> members;   // mask index of each member
    std::vector<uint32_t> local;     // first LDS bin of each member
    std::vector<GRec> grec;          // per member (zero for all but near QUAD members), plus kGradRecPad zero records
};

// masks: every mask in mask order, in the coordinates of its layout
// (layout_of[i]); members index this list.
GradChunks make_grad_chunks(const std::vector<MaskRec>& masks, const std::vector<uint8_t>& layout_of,
                            const std::vector<uint64_t>& bin_off, uint64_t n_bins, int tile_bits, int lane_bits);

// out = b (w - gamma y) + s z + c x ; acc += ca out.  Null pointers drop their term.
void cheb_rec(syk_dtype dtype, int64_t n, void* out, const void* w, const void* y, const void* z, const void* x,
              void* acc, double b, double gamma, double s, std::complex<double> c, std::complex<double> ca,
              hipStream_t st);

// bins_dev (device, n_bins complex) += sum_p w_p * bins of (g_p, v_p); complex128 states.
void grad_bins(syk_terms_s& h, const std::vector<const void*>& g, const std::vector<const void*>& v,
               const std::vector<double>& w, double* bins_dev, hipStream_t st);

}  // namespace syk
