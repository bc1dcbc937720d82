// Launch interface of the apply_H kernels.
#pragma once

#include "handle.hpp"

namespace syk {

// Mask record of the gradient kernel for one launch shape (tile_bits): what
// a mask needs that does not depend on the lane or the tile.  Loaded with one
// scalar load.
struct alignas(16) KRec {
    uint32_t xl;        // x & (tile rows - 1): row offset of the source inside the tile
    uint32_t qpack;     // flipped qubits, one per byte
    uint32_t zbase;     // Z string of the mask
    uint32_t meta;      // type << 28 | table index
    uint32_t bin0;      // first derivative bin of the mask
    uint32_t x_high;    // x >> tile_bits: source tile = tile ^ x_high
};
static_assert(sizeof(KRec) == 32, "KRec layout");

// Mask record of the apply kernel for one launch shape and element size, in
// the class-sorted order of its chunk (QApplyChunk).  The first four words are
// what the QUAD loops read per mask; the rest serves table staging and the
// PAIR / DIAG paths.
struct alignas(16) QRec {
    uint32_t sel;    // QUAD: byte selector gathering the lane bits of tid at q0..q3 (0x0c: not a lane bit);
                     // PAIR: byte offset of the mask's staged values in the chunk's table area
    uint32_t zl;     // lane bits of zbase
    uint32_t xoff;   // (x & lane mask) * element size: lane part of the source offset
    uint32_t koffs;  // QUAD: byte b = table byte offset of the index bit that k-bit b sets (0 if b is not flipped),
                     // except in the first record of a group: the offset of its lowest flipped k bit;
                     // PAIR / DIAG: the k bits of x
    uint32_t tab;    // index into the type's tables
    uint32_t xl;     // x & (tile rows - 1)
    uint32_t qpack;  // flipped qubits, one per byte
    uint32_t zbase;  // Z string of the mask
};
static_assert(sizeof(QRec) == 32, "QRec layout");

constexpr int kMaxKBits = 3;   // up to 8 rows per thread
constexpr int kQuadClasses = 27;   // 3^kMaxKBits (k-bit flipped / in the Z string / neither)

// One chunk of the apply kernel: masks sharing a source tile, QUAD masks first
// (groups of three by group class, then the others sorted by class), then PAIR
// (those that flip no k bit first, sorted by the k bits of their Z string),
// then DIAG.
struct alignas(16) QApplyChunk {
    uint32_t x_high;    // source tile = tile ^ x_high
    uint32_t first;     // first record (index into the QRec array)
    uint32_t new_tile;  // x_high differs from the previous chunk's
    uint32_t n_quad;
    uint32_t n_pair, n_diag;
    uint32_t pcnt[2];   // PAIR masks that flip no k bit, per k-bit pattern of zbase, one byte per pattern
    uint32_t cnt[8];    // byte c < 27: QUAD masks of class c outside groups; byte 27 + g: groups of class g
};
static_assert(sizeof(QApplyChunk) == 64, "QApplyChunk layout");

// Optional overrides of the launch shape (autotuner / benchmarks); 0 = default.
struct ApplyTuning {
    int tile_bits;
    int xcd_remap;
    int cols;        // columns per workgroup (1 or 2; 0 = default)
};

constexpr int kColsPerLaunch = 64;   // columns of a block served by one launch

struct ApplyPlan {
    int tile_bits;   // rows per workgroup tile = 2^tile_bits
    int slices;      // launches over column slices of kColsPerLaunch
    int nt;          // threads per workgroup
    int lb;          // lane bits: nt = 2^lb
    int rpt;         // tile rows per thread
    int xcd_remap;
    int two_layouts; // also run the masks that flip few rows of a tile on a bit-rotated copy
    int nc;          // columns per workgroup where a launch's columns pair up by realisation (1 or 2)
};

ApplyPlan plan_apply(int M, int nvec, syk_dtype dtype, const ApplyTuning* tune);

// The plan for a handle's tables of M qubits, honouring its
// syk_set_apply_tuning settings.
inline ApplyPlan plan_for(const syk_terms_s& h, int M, int nvec, syk_dtype dtype)
{
    ApplyTuning t{h.tune_tile_bits, h.tune_xcd, h.tune_cols};
    return plan_apply(M, nvec, dtype, h.tuned ? &t : nullptr);
}
inline ApplyPlan plan_for(const syk_terms_s& h, int nvec, syk_dtype dtype) { return plan_for(h, h.H.M, nvec, dtype); }

// Gradient mask records for tiles of 2^tile_bits rows, one per mask of `masks`
// in its order, with bin0 = bin_off[i].
std::vector<KRec> build_krecs(const std::vector<MaskRec>& masks, const std::vector<uint64_t>& bin_off, int tile_bits);

// Second row layout: row bits rotated right by tb (bit b -> b - tb mod M), so
// that the high qubits of the natural layout become the low bits of a tile.
// quad_in_rotated: a QUAD mask with fewer flipped qubits outside a tile there
// than in the natural layout (false for every other mask type).  rotate_mask:
// the same mask in rotated row coordinates (x, zbase and the qubit of every
// table index bit relabelled; coefficients unchanged).
bool quad_in_rotated(const MaskRec& m, int M, int tb);
MaskRec rotate_mask(const MaskRec& m, int M, int tb);

// dst[c] = src[c] viewed as a [2^log_h] x [2^log_w] row-major matrix and
// transposed (with add: dst[c] += ...), for ncols columns of dim elements.
// For log_h = M - tb, log_w = tb this moves every row to its rotated index.
void launch_transpose(syk_dtype dtype, const void* src, void* dst, int log_h, int log_w, int ncols, uint64_t dim,
                      bool add, hipStream_t s);

// out = H psi for nvec columns stored one after another; real_of_col: host array or NULL.
void launch_apply_h(const HamiltonianDev& H, syk_dtype dtype, int nvec, const int32_t* real_of_col,
                    const void* psi, void* out, const ApplyPlan& P, hipStream_t s);

// Bytes of the file-scope device scratch of the allocation-free apply.
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;

// launch_apply_h without any allocation: the rotated layout's two buffers come
// from the scratch array of `device` (the current device), and the handle's
// tables for this launch shape and its diagonal must exist already (SYK_EINVAL
// otherwise, as for plans whose buffers exceed kNoAllocScratchBytes).  Calls
// that overlap on one device race on the scratch.
void launch_apply_h_noalloc(const HamiltonianDev& H, int device, syk_dtype dtype, int nvec,
                            const int32_t* real_of_col, const void* psi, void* out, const ApplyPlan& P,
                            hipStream_t s);

}  // namespace syk
