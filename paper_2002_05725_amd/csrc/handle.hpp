// The syk_terms handle: host tables, device tables and workspaces.
#pragma once

#include <map>
#include <memory>
#include <vector>

#include "terms.hpp"

namespace syk {

// Device view of the Hamiltonian tables used by the kernels.
struct HamiltonianDev {
    int N = 0, M = 0, n_real = 0, n_diag = 0;
    const MaskRec* masks = nullptr;
    const c128* tab4_d = nullptr;
    const c64* tab4_f = nullptr;
    const uint32_t* qinfo = nullptr;
    const c128* phi2_d = nullptr;
    const c64* phi2_f = nullptr;
    const double* w2_d = nullptr;
    const float* w2_f = nullptr;
    const uint32_t* dz = nullptr;
    const double* dw_d = nullptr;
    const float* dw_f = nullptr;
    // Host mask list (sorted by x) and derivative-bin offsets the per-launch-
    // shape tables are built from.
    const std::vector<MaskRec>* host_masks = nullptr;
    const std::vector<uint64_t>* bin_off = nullptr;
    // Per-launch-shape chunks and class-sorted records of the apply kernel.
    struct ApplyTables {
        DevBuf chunks, recs, far;
        int n_chunks = 0, n_far = 0;
    };
    mutable std::map<int, std::unique_ptr<ApplyTables>> apply_tables;
    // Rotated copies of psi and of the second layout's output (two-layout plans).
    mutable DevBuf rot_in, rot_out;
    // The diagonal of H per realisation (FP64, [n_real][2^M]), filled on the
    // first apply: it does not depend on the state.
    mutable DevBuf diag;
    mutable bool diag_ready = false;
};

// Named device workspaces, grown on demand and kept until the handle dies.
// With a cap (limit > 0), growing past it throws SYK_ENOMEM before allocating.
struct Workspace {
    std::map<std::string, std::unique_ptr<DevBuf>> bufs;
    size_t limit = 0;
    size_t total = 0;   // bytes held over all buffers
    void* get(const std::string& name, size_t bytes)
    {
        auto& b = bufs[name];
        if (!b) b.reset(new DevBuf());
        if (bytes > b->bytes) {
            const size_t after = total - b->bytes + bytes;
            if (limit > 0 && after > limit)
                throw Error(SYK_ENOMEM, "workspace of " + std::to_string(after) + " bytes exceeds the cap of " +
                                            std::to_string(limit) + " bytes (" + name + ")");
            total -= b->bytes;
            b->ensure(bytes);
            total += b->bytes;
        }
        return b->p;
    }
    // bytes already held under `name` (0 if none)
    size_t held(const std::string& name) const
    {
        auto it = bufs.find(name);
        return (it == bufs.end() || !it->second) ? 0 : it->second->bytes;
    }
    void release_all()
    {
        bufs.clear();
        total = 0;
    }
};

}  // namespace syk

struct syk_terms_s {
    int device = 0;
    syk::TermTables host;
    syk::DeviceTerms dev;
    syk::HamiltonianDev H;
    syk::Workspace ws;
    unsigned upload_slot = 0;       // ring position of small coefficient uploads
    std::map<int, std::unique_ptr<syk::DevBuf>> grad_chunks;   // per (tile_bits, layouts)
    std::map<int, int> grad_nchunks, grad_nmembers;
    // H restricted to each fermion-parity sector, built on first use
    struct Sector {
        syk::TermTables host;
        syk::DeviceTerms dev;
        syk::HamiltonianDev H;
    };
    std::unique_ptr<Sector> sectors[2];
    bool tuned = false;             // apply_H launch shape set by syk_set_apply_tuning
    int tune_tile_bits = 0, tune_xcd = 1, tune_cols = 0;
};

namespace syk {
// Tables of the sector-s Hamiltonian of a handle (built on first use).
const HamiltonianDev& sector_ham(syk_terms_s& h, int s);
}  // namespace syk
