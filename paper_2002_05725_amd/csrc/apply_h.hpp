// Launch interface of the apply_H kernels.
#pragma once

#include "handle.hpp"

namespace syk {

// Mask record of the single-vector kernels for one launch shape (tile_bits,
// threads): everything about a mask that does not depend on the lane or the
// tile, precomputed on the host.  Loaded with one scalar load.
struct alignas(16) KRec {
    uint32_t xl;        // x & (tile rows - 1): row offset of the source inside the tile
    uint32_t qpack;     // flipped qubits, one per byte
    uint32_t zbase;     // Z string of the mask
    uint32_t meta;      // type << 28 | path << 26 | table index
    uint32_t kinfo[2];  // QUAD, per row k: (index bits from k | sign bit from k << 4) << 5 (k % 6)
    uint32_t pad[2];    // pad[0]: first derivative bin of the mask
};
static_assert(sizeof(KRec) == 32, "KRec layout");

// QUAD paths: the table entry and sign of a thread's rows
enum : uint32_t {
    PATH_SAME = 0,   // ... are the same for all rows
    PATH_SIGN = 1,   // ... share the entry; only the sign depends on the row
    PATH_FULL = 2    // ... both depend on the row
};

// Optional overrides of the launch shape (autotuner / benchmarks); 0 = default.
struct ApplyTuning {
    int tile_bits;
    int threads;
    int xcd_remap;
};

constexpr int kColsPerLaunch = 64;   // columns of a block served by one launch

struct ApplyPlan {
    int tile_bits;   // rows per workgroup tile = 2^tile_bits
    int slices;      // launches over column slices of kColsPerLaunch
    int nt;          // threads per workgroup
    int rpt;         // tile rows per thread
    int xcd_remap;
};

ApplyPlan plan_apply(int M, int nvec, syk_dtype dtype, const ApplyTuning* tune);

// The plan for a handle, honouring its syk_set_apply_tuning settings.
inline ApplyPlan plan_for(const syk_terms_s& h, int nvec, syk_dtype dtype)
{
    ApplyTuning t{h.tune_tile_bits, h.tune_threads, h.tune_xcd};
    return plan_apply(h.H.M, nvec, dtype, h.tuned ? &t : nullptr);
}

struct ApplyPlan;
// Device mask records for a single-vector launch shape (built on first use).
const KRec* krecs_for(const HamiltonianDev& H, const ApplyPlan& P);

// out = H psi for nvec columns stored one after another; real_of_col: host array or NULL.
void launch_apply_h(const HamiltonianDev& H, syk_dtype dtype, int nvec, const int32_t* real_of_col,
                    const void* psi, void* out, const ApplyPlan& P, hipStream_t s);

}  // namespace syk
