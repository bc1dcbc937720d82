// Host-side term builder: couplings -> Pauli strings -> flip-mask groups.
#pragma once

#include <complex>
#include <map>
#include <memory>
#include <vector>

#include "common.hpp"

namespace syk {

// Kinds of flip mask x (the set of qubits a term flips).
enum MaskType : uint32_t { MASK_DIAG = 0, MASK_PAIR = 2, MASK_QUAD = 4 };

// One flip mask, as read by the apply kernel.  For every row r the mask adds
// D_x(r) psi[r ^ x] to (H psi)[r], with
//   QUAD: D_x(r) = (-1)^{popcount(r & zbase)} T[bits of r at q0..q3]
//   PAIR: D_x(r) = (-1)^{popcount(r & zbase)} sum_e Phi[bits of r at q0,q1][e] L_e(r),
//         L_e(r) = W_e + sum_c w_{e,c} r_c          (real, c over all qubits)
//   DIAG: D_0(r) = sum_n d_n (-1)^{popcount(r & dz_n)}
struct alignas(16) MaskRec {
    uint32_t x;        // qubits flipped
    uint32_t zbase;    // Z string shared by all terms of the mask
    uint32_t qpack;    // flipped qubits, ascending, one per byte (QUAD: 4, PAIR: 2)
    uint32_t type_tab; // type << 28 | index into the type's tables
};
static_assert(sizeof(MaskRec) == 16, "MaskRec layout");

__host__ __device__ inline uint32_t mask_q(uint32_t qpack, int i) { return (qpack >> (8 * i)) & 0xffu; }

// Masks with the same x >> tile_bits read the same source tile of psi; the
// gradient kernel cuts such runs into chunks of at most kChunkMasks masks.
constexpr int kChunkMasks = 64;

// Pauli string X^x Z^z times the phase i^ph (acts as |s> -> i^ph (-1)^{|s&z|} |s^x>).
struct Pauli {
    uint32_t x, z;
    int ph;
};

// chi_a without its 2^{-1/2}: X_k Z_{<k} for even a, i X_k Z_{<=k} for odd a (Y = iXZ).
inline Pauli majorana_pauli(int a)
{
    int k = a >> 1;
    uint32_t below = (1u << k) - 1u;
    if (a & 1) return {1u << k, below | (1u << k), 1};
    return {1u << k, below, 0};
}

// (X^x1 Z^z1)(X^x2 Z^z2) = (-1)^{|z1 & x2|} X^{x1^x2} Z^{z1^z2}
inline Pauli pauli_mul(const Pauli& A, const Pauli& B)
{
    int sign = __builtin_popcount(A.z & B.x) & 1;
    return {A.x ^ B.x, A.z ^ B.z, (A.ph + B.ph + 2 * sign) & 3};
}

// Where coupling n lives in the grouped form (for derivatives in the couplings).
struct TermRef {
    uint32_t mask;   // index in the sorted mask array
    uint32_t z;      // Z string of the term's Pauli string
    int ph;          // phase exponent: the term is J * i^ph / 4 * X^x Z^z
    int slot;        // PAIR: pair qubit c; DIAG: index in dz/dw; QUAD: unused
};

// Host copy of every table, in both precisions, plus device mirrors.
struct TermTables {
    int N = 0, M = 0, n_real = 0;
    int64_t n_terms = 0;
    std::vector<MaskRec> masks;          // sorted by x
    int n_quad = 0, n_pair = 0, n_diag = 0;
    // QUAD tables: [n_quad][n_real][16]; qinfo [n_quad]: (qpack, zbase) of each QUAD mask
    std::vector<c128> tab4;
    std::vector<uint32_t> qinfo;
    // PAIR tables: Phi [n_pair][16] (index bits*4 + e), weights [n_pair][n_real][4][M+1]
    // (entry M holds W_e, entry c holds w_{e,c})
    std::vector<c128> phi2;
    std::vector<double> w2;
    // DIAG terms: dz [n_diag], d [n_real][n_diag]
    std::vector<uint32_t> dz;
    std::vector<double> dw;
    // Coupling order -> grouped form; per-mask offsets into the derivative bins
    // (QUAD: 16 bins; PAIR: 4 + 4 M bins; DIAG: n_diag bins).
    std::vector<TermRef> terms;
    std::vector<uint64_t> bin_off;
    uint64_t n_bins = 0;
};

// Derivative bins of one mask (complex, FP64), filled by the gradient kernel:
//   QUAD  B[idx]            = sum_r conj(g[r]) (-1)^{|r & zbase|} v[r ^ x] over rows with bits idx at q0..q3
//   PAIR  B[idx], C_c[idx]  = the same over rows with bits idx at q0, q1 (C_c: only rows with r_c = 1)
//   DIAG  E_n               = sum_r conj(g[r]) (-1)^{|r & dz_n|} v[r]
// d/dJ_n Re <g|H v> for every coupling n, from the bins.
void couplings_from_bins(const TermTables& T, const double* bins /* n_bins (re, im) */, double* out);

void build_tables(int N, int n_real, const double* J, TermTables& out);

// Tables of H restricted to the fermion-parity sector s (rows with popcount
// parity s, indexed without their top qubit, whose bit is implied): M - 1
// qubits, masks over them, no derivative bins.
void build_sector_tables(const TermTables& full, int s, TermTables& out);

// Device-resident copies of the tables.
struct DeviceTerms {
    DevBuf masks, tab4_d, tab4_f, qinfo, phi2_d, phi2_f, w2_d, w2_f, dz, dw_d, dw_f;
};

// A QUAD mask whose flipped qubits are all tile bits.
struct alignas(16) FarRec {
    uint32_t x_high, qpack, zbase, tab;
};

}  // namespace syk
