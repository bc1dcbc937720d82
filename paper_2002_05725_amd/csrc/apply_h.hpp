// Launch interface of the apply_H kernels.
#pragma once

#include "handle.hpp"

namespace syk {

// Optional overrides of the launch shape (autotuner / benchmarks); 0 = default.
struct ApplyTuning {
    int tile_bits;
    int threads;
    int xcd_remap;
};

struct ApplyPlan {
    int tile_bits;   // rows per workgroup tile = 2^tile_bits
    int log_cw;      // interleaved columns per tile = 2^log_cw
    int slices;      // launches over column slices (nvec / 2^log_cw)
    int nt;          // threads per workgroup
    int rpt;         // tile elements per thread
    int xcd_remap;
    bool single;     // one column: the specialised single-vector kernel
};

ApplyPlan plan_apply(int M, int nvec, syk_dtype dtype, const ApplyTuning* tune);

// The plan for a handle, honouring its syk_set_apply_tuning settings.
inline ApplyPlan plan_for(const syk_terms_s& h, int nvec, syk_dtype dtype)
{
    ApplyTuning t{h.tune_tile_bits, h.tune_threads, h.tune_xcd};
    return plan_apply(h.H.M, nvec, dtype, h.tuned ? &t : nullptr);
}

// out = H psi for a [dim][nvec] block; real_of_col: host array or NULL.
void launch_apply_h(const HamiltonianDev& H, syk_dtype dtype, int nvec, const int32_t* real_of_col,
                    const void* psi, void* out, const ApplyPlan& P, hipStream_t s);

}  // namespace syk
