// Matrix-free H psi for the Jordan-Wigner SYK Hamiltonian on gfx950.
//
// (H psi)[r] = sum_x D_x(r) psi[r ^ x] over the flip masks x of terms.hpp.
// A workgroup owns one tile of 2^tile_bits consecutive rows of one column of a
// block (columns are whole state vectors, one after another).  For a mask, every row of the tile reads
// the tile (tile ^ (x >> tile_bits)) of psi, permuted by x's low bits, so the
// masks are processed chunk by chunk in x order: the shared source tile is
// staged once into LDS with coalesced loads, every mask of the chunk gathers
// from LDS, and each thread keeps its rows' sums in registers and writes them
// once.
//
// Grid: (tiles, column groups); every workgroup serves NC consecutive columns
// of one realisation (NC = 1, or 2 for the two typical states a realisation
// carries in a block), so mask records, PAIR weights and DIAG terms are
// wave-uniform (scalar loads) and the chunk's QUAD tables are staged into LDS
// next to the NC source tiles.  Everything a mask decodes (record, table
// entries, lane index and sign, PAIR coefficients) is formed once and applied
// to every column.  Up to 64 columns per launch.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>

#include "apply_h.hpp"
#include "mask_classes.hpp"
#include "timing.hpp"

namespace syk {

namespace {

template <typename R>
struct KTerms {
    const cplx<R>* __restrict__ tab4;
    const uint32_t* __restrict__ qinfo;
    const cplx<R>* __restrict__ phi2;
    const R* __restrict__ w2;
    const double* __restrict__ diag;   // [n_real][dim]: the diagonal of H
    int n_real, M;
};

struct KLayout {
    const FarRec* __restrict__ far;   // QUAD masks flipping only tile bits
    int n_far;
    int n_chunks;
    int tile_bits;     // rows per tile = 2^tile_bits
    int lane_bits;     // threads per workgroup = 2^lane_bits
    uint64_t dim;      // rows per column
    int col0;          // first column of this launch (column = col0 + NC blockIdx.y + c)
    uint32_t n_tiles;  // dim >> tile_bits
    int xcd_remap;     // spread consecutive tiles over XCDs in contiguous ranges
    int32_t real[kColsPerLaunch];  // realisation of each column of the launch
};

static_assert(kColsPerLaunch == 64, "column slice");

// Workgroups are dispatched round-robin over the 8 XCDs; give XCD j the
// contiguous tile range [j n/8, (j+1) n/8) so that its L2 sees neighbouring
// tiles, whose source tiles overlap for low flip masks.
__device__ __forceinline__ uint32_t tile_of_block(uint32_t b, const KLayout& L)
{
    if (!L.xcd_remap || (L.n_tiles & 7u)) return b;
    return (b & 7u) * (L.n_tiles >> 3) + (b >> 3);
}

__device__ __forceinline__ uint32_t parity(uint32_t v) { return __popc(v) & 1u; }

// Flip the sign of x when s is 1 (s in {0, 1}).
__device__ __forceinline__ double flip(double x, uint32_t s)
{
    return __hiloint2double(__double2hiint(x) ^ (int)(s << 31), __double2loint(x));
}
__device__ __forceinline__ float flip(float x, uint32_t s) { return __int_as_float(__float_as_int(x) ^ (int)(s << 31)); }

__device__ __forceinline__ uint32_t bit(uint32_t r, uint32_t q) { return (r >> q) & 1u; }

// Sign flip when the count c is odd: adding c << 31 to the word holding the
// sign bit changes that bit exactly when c is odd.  Written as one
// v_lshl_add_u32 per word (plain C lets the compiler share the shift between
// words, one instruction more per table entry pair).
__device__ __forceinline__ uint32_t add_lsb31(uint32_t w, uint32_t c)
{
    uint32_t r;
    asm("v_lshl_add_u32 %0, %1, 31, %2" : "=v"(r) : "v"(c), "v"(w));
    return r;
}
__device__ __forceinline__ double flip_odd(double x, uint32_t c)
{
    return __hiloint2double((int)add_lsb31((uint32_t)__double2hiint(x), c), __double2loint(x));
}
__device__ __forceinline__ float flip_odd(float x, uint32_t c) { return __uint_as_float(add_lsb31(__float_as_uint(x), c)); }

// 4-bit QUAD table index: bit m = bit q_m of r.
__device__ __forceinline__ uint32_t quad_index(uint32_t r, uint32_t qpack)
{
    return bit(r, mask_q(qpack, 0)) | (bit(r, mask_q(qpack, 1)) << 1) | (bit(r, mask_q(qpack, 2)) << 2) |
           (bit(r, mask_q(qpack, 3)) << 3);
}

}  // namespace

namespace {

// Thread layout: row rl = tid + (k << lb) of the tile (nt = 2^lb threads,
// lb = 8 whenever a thread owns several rows, k < RPT).  A row index splits into
// lane bits (tid), k bits (the same for every lane) and tile bits (the same for
// the workgroup).
//
// QUAD masks: the tile bits of every table index and sign are folded into the
// tables while they are staged.  Inside a chunk the host sorts the QUAD masks
// by class: for each k bit, whether the mask flips it, has it in its Z string,
// or neither.  Within a class the source offset of every row and the sign each
// row adds are compile-time constants, and the rows use one table entry per
// subset of the flipped k bits.  The lane part of the table index is a byte
// gather of tid's bits (v_perm) and a dot product with the powers of two
// (v_dot4), the lane part of the sign one popcount.
constexpr int kLaneBits = 8;

// Masks per chunk of the apply kernel: complex128 keeps the LDS of a
// 2048-row tile at 40 KiB so that four workgroups share a CU.
constexpr int apply_chunk_masks(uint32_t esz) { return esz == 16 ? 32 : 64; }

template <typename R, int RPT, int NC>
struct ApplyLds {
    cplx<R> src[NC * (RPT << kLaneBits)];   // column c's tile at c * (RPT << kLaneBits)
    cplx<R> tabs[apply_chunk_masks(sizeof(cplx<R>)) * 16];
};

// Waves per SIMD the kernel is compiled for: four with one column and 8 rows
// per thread; two columns double the sums (three waves for complex64, two for
// complex128, whose two 32 KiB tiles allow two workgroups per CU anyway).
constexpr int apply_waves(int rpt, int nc, int rbytes)
{
    return rpt != 8 ? 1 : nc == 1 ? 4 : rbytes == 8 ? 2 : 3;
}

template <typename R>
__device__ __forceinline__ void cmac(R& pr, R& pi, R a, R b, const cplx<R>& v)
{
    pr = fma(a, v.re, pr);
    pr = fma(-b, v.im, pr);
    pi = fma(a, v.im, pi);
    pi = fma(b, v.re, pi);
}

template <typename R, int RPT, int NC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(apply_waves(RPT, NC, sizeof(R)))))
k_apply(KTerms<R> T, const QApplyChunk* __restrict__ chunks,
                                               const QRec* __restrict__ rec, KLayout L,
                                               const cplx<R>* __restrict__ psi, cplx<R>* __restrict__ out)
{
    constexpr int KB = ilog2c(RPT);
    constexpr uint32_t esz = sizeof(cplx<R>);
    // byte weights of the four gathered index bits: esz * 2^m
    constexpr uint32_t kDotW = (esz) | (2 * esz) << 8 | (4 * esz) << 16 | (8 * esz) << 24;
    // kept in a VGPR, so that v_dot4 can take the per-mask table offset from an
    // SGPR (one scalar operand per instruction); not for two complex64 columns,
    // whose kernel is short of VGPRs at three waves (1.2% slower with it)
    uint32_t dotw = kDotW;
    if constexpr (NC == 1 || sizeof(R) == 8) asm("" : "+v"(dotw));
    __shared__ ApplyLds<R, RPT, NC> S;
    constexpr uint32_t TS = RPT << kLaneBits;   // rows of a column's tile
    const char* src_b = reinterpret_cast<const char*>(S.src);
    const char* tab_b = reinterpret_cast<const char*>(S.tabs);
    auto src_at = [&](uint32_t off) { return *reinterpret_cast<const cplx<R>*>(src_b + off); };
    auto tab_at = [&](uint32_t off) { return *reinterpret_cast<const cplx<R>*>(tab_b + off); };

    const uint32_t lb = (RPT > 1) ? (uint32_t)kLaneBits : (uint32_t)L.lane_bits;
    const uint32_t nt = 1u << lb;
    const uint32_t tile = tile_of_block(blockIdx.x, L);
    const uint32_t tid = threadIdx.x;
    const int rc = L.real[blockIdx.y * NC];   // the same for all NC columns
    const int M = T.M;
    const uint32_t base = tile << L.tile_bits;
    psi += (uint64_t)(L.col0 + blockIdx.y * NC) * L.dim;   // this workgroup's first column
    out += (uint64_t)(L.col0 + blockIdx.y * NC) * L.dim;

    // bits 0..3 and 4..7 of tid, one per byte
    uint32_t B0 = 0, B1 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        B0 |= ((tid >> i) & 1u) << (8 * i);
        B1 |= ((tid >> (4 + i)) & 1u) << (8 * i);
    }
    const uint32_t tid_b = tid * esz;

    // complex128 sums directly in pr/pi; complex64 sums each chunk in FP32 and
    // carries the running total in FP64.
    constexpr bool kSplit = sizeof(R) < sizeof(double);
    double acc_re[NC][RPT], acc_im[NC][RPT];
    R pr[NC][RPT], pi[NC][RPT];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            acc_re[c][k] = acc_im[c][k] = 0.0;
            pr[c][k] = pi[c][k] = R(0);
        }
    auto carry = [&]() {   // complex64: chunk sums into the FP64 running totals
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                acc_re[c][k] += (double)pr[c][k];
                acc_im[c][k] += (double)pi[c][k];
                pr[c][k] = pi[c][k] = R(0);
            }
    };
    // column c's source row at byte offset off of its tile
    auto src_row = [&](int c, uint32_t off) { return src_at(off + (uint32_t)c * TS * esz); };

    for (int g = 0; g < L.n_chunks; ++g) {
        const QApplyChunk C = chunks[g];
        uint32_t n_flat = 0;   // flat PAIR masks (no flipped k bit), first among the PAIR records
#pragma unroll
        for (int b = 0; b < 8; ++b) n_flat += (C.pcnt[b >> 2] >> (8 * (b & 3))) & 0xffu;
        __syncthreads();   // previous chunk is done with src / tabs
        if (C.new_tile) {
            const uint64_t sbase = (uint64_t)(tile ^ C.x_high) << L.tile_bits;
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int k = 0; k < RPT; ++k)
                    S.src[c * TS + tid + k * nt] = (psi + c * L.dim)[sbase + tid + k * nt];
        }
        // Staged QUAD table entry i of slot j: sign_tile * T[i ^ index_tile].
        for (uint32_t e = tid; e < C.n_quad * 16; e += nt) {
            const QRec& qr = rec[C.first + (e >> 4)];
            const uint32_t qt = qr.tab, qp = qr.qpack, zb = qr.zbase;   // in this layout's coordinates
            const cplx<R> c = T.tab4[((size_t)qt * T.n_real + rc) * 16 + ((e & 15u) ^ quad_index(base, qp))];
            const uint32_t sg = parity(base & zb);
            cplx<R> o;
            o.re = flip(c.re, sg);
            o.im = flip(c.im, sg);
            S.tabs[e] = o;
        }
        // PAIR slots (after the QUAD tables): for each row k and term e, the part
        // of L_e(r) that does not depend on the lane, t_{k,e} = W_e + sum over
        // tile and k bits c of w_{e,c} r_c.  One slot holds RPT * 4 values (flat
        // masks, below, only row 0).
        for (uint32_t v = tid; v < C.n_pair * (RPT * 4); v += nt) {
            const uint32_t p = v / (RPT * 4), k = (v >> 2) % RPT, e = v & 3u;
            if (p < n_flat && k != 0) continue;   // flat masks use row 0 only
            const QRec& pq = rec[C.first + C.n_quad + p];
            const R* w = T.w2 + (((size_t)pq.tab * T.n_real + rc) * 4 + e) * (M + 1);
            const uint32_t rb = base | (k << lb);
            R acc = w[M];
            for (int c = (int)lb; c < M; ++c)
                if ((rb >> c) & 1u) acc += w[c];
            reinterpret_cast<R*>(reinterpret_cast<char*>(S.tabs) + pq.sel)[k * 4 + e] = acc;
        }
        __syncthreads();

        uint32_t mi = C.first;
        // The next QUAD record is loaded one mask ahead (records run one past
        // the end): complex128 at the start of a mask, complex64 after its FMAs
        // (an outstanding scalar load makes every LDS wait a full wait).
        constexpr bool kEarlyRecord = sizeof(R) == 8;
        QRec qn = rec[mi];
        // Groups of three QUAD masks (same lane flips, J = 1 or 2 flipped k
        // bits in all three ways): the lane index, the lane sign and the source
        // rows are read once for the three.  Member j's table is the (m + j)-th
        // of the chunk; the index bits of its flipped k bits sit at kof and
        // 2 kof (kof: the first record's koffs).  The next member's table
        // entries are read while the previous member's FMAs run.
        if constexpr (KB == kMaxKBits) {
            auto group_loop = [&](auto gcls) {
                constexpr int GC = decltype(gcls)::value;
                constexpr int J = 1 + (GC >> 1), P = GC & 1;
                constexpr int NE = 1 << J;   // table entries per member
                const uint32_t n = (C.cnt[(kQuadClasses + GC) >> 2] >> (8 * ((kQuadClasses + GC) & 3))) & 0xffu;
                for (uint32_t i = 0; i < n; ++i, mi += 3) {
                    const QRec q = qn;
                    if constexpr (kEarlyRecord) qn = rec[mi + 3];
                    const uint32_t ia = __builtin_amdgcn_udot4(__builtin_amdgcn_perm(B1, B0, q.sel), dotw,
                                                               (mi - C.first) * 16u * esz, false);
                    const uint32_t sl = (uint32_t)__popc(tid & q.zl);   // lane sign: its parity
                    const uint32_t kof = q.koffs;
                    auto load_member = [&](auto jc, cplx<R> (&t)[NE]) {
                        constexpr uint32_t j = decltype(jc)::value;
#pragma unroll
                        for (int e = 0; e < NE; ++e)
                            t[e] = tab_at(ia + (uint32_t)e * kof + j * 16u * esz);
                    };
                    auto member_fma = [&](auto jc, cplx<R> (&t)[NE], const cplx<R> (&v)[NC][RPT]) {
                        constexpr int j = decltype(jc)::value;
                        constexpr int XK = group_xk(J, j), ZK = group_zk(XK, P);
#pragma unroll
                        for (int e = 0; e < NE; ++e) {
                            t[e].re = flip_odd(t[e].re, sl);
                            t[e].im = flip_odd(t[e].im, sl);
                        }
#pragma unroll
                        for (int c = 0; c < NC; ++c)
#pragma unroll
                            for (int k = 0; k < RPT; ++k) {
                                const cplx<R> te = t[pack_bits3(k & XK, XK)];
                                const bool neg = (popc3(k & ZK) & 1) != 0;
                                const R a = neg ? -te.re : te.re, b = neg ? -te.im : te.im;
                                cmac(pr[c][k], pi[c][k], a, b, v[c][k ^ XK]);
                            }
                    };
                    using I0 = std::integral_constant<int, 0>;
                    using I1 = std::integral_constant<int, 1>;
                    using I2 = std::integral_constant<int, 2>;
                    cplx<R> ta[NE], tb[NE];
                    load_member(I0{}, ta);
                    __builtin_amdgcn_sched_barrier(0);
                    const uint32_t sb = tid_b ^ q.xoff;
                    cplx<R> v[NC][RPT];
#pragma unroll
                    for (int c = 0; c < NC; ++c)
#pragma unroll
                        for (int k = 0; k < RPT; ++k) v[c][k] = src_row(c, sb + ((uint32_t)k << kLaneBits) * esz);
                    __builtin_amdgcn_sched_barrier(0);
                    if constexpr (J == 1) {
                        load_member(I1{}, tb);
                        member_fma(I0{}, ta, v);
                        __builtin_amdgcn_sched_barrier(0);
                        load_member(I2{}, ta);
                        member_fma(I1{}, tb, v);
                        __builtin_amdgcn_sched_barrier(0);
                        member_fma(I2{}, ta, v);
                    } else {
                        // four entries per member: no read-ahead (register pressure)
                        member_fma(I0{}, ta, v);
                        __builtin_amdgcn_sched_barrier(0);
                        load_member(I1{}, tb);
                        member_fma(I1{}, tb, v);
                        __builtin_amdgcn_sched_barrier(0);
                        load_member(I2{}, ta);
                        member_fma(I2{}, ta, v);
                    }
                    if constexpr (!kEarlyRecord) {
                        __builtin_amdgcn_sched_barrier(0);
                        qn = rec[mi + 3];
                    }
                }
            };
            for_each_class(group_loop, std::make_integer_sequence<int, kQuadGroupClasses>{});
        }
        auto class_loop = [&](auto cls) {
            constexpr int CL = decltype(cls)::value;
            constexpr uint32_t XK = (uint32_t)class_bits(CL, KB, 1);   // k bits the masks flip
            constexpr uint32_t ZK = (uint32_t)class_bits(CL, KB, 2);   // k bits in their Z string
            const uint32_t n = (C.cnt[CL >> 2] >> (8 * (CL & 3))) & 0xffu;
            for (uint32_t i = 0; i < n; ++i, ++mi) {
                const QRec q = qn;
                if constexpr (kEarlyRecord) qn = rec[mi + 1];
                const uint32_t ia = __builtin_amdgcn_udot4(__builtin_amdgcn_perm(B1, B0, q.sel), dotw,
                                                           (mi - C.first) * 16u * esz, false);
                const uint32_t sl = (uint32_t)__popc(tid & q.zl);   // lane sign: its parity
                cplx<R> te[RPT];   // entry for the k bits in p = k & XK
#pragma unroll
                for (int p = 0; p < RPT; ++p) {
                    if ((p & ~(int)XK) != 0) continue;
                    uint32_t off = 0;
#pragma unroll
                    for (int b = 0; b < KB; ++b)
                        if ((p >> b) & 1) off += (q.koffs >> (8 * b)) & 0xffu;
                    te[p] = tab_at(ia + off);
                }
                // table entries first, then the source rows in row order, so
                // that each row's FMAs wait only for its own load
                __builtin_amdgcn_sched_barrier(0);
                const uint32_t sb = tid_b ^ q.xoff;
                cplx<R> v[NC][RPT];
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int k = 0; k < RPT; ++k) v[c][k] = src_row(c, sb + (((uint32_t)k ^ XK) << kLaneBits) * esz);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int p = 0; p < RPT; ++p) {
                    if ((p & ~(int)XK) != 0) continue;
                    te[p].re = flip_odd(te[p].re, sl);
                    te[p].im = flip_odd(te[p].im, sl);
                }
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        const cplx<R> t = te[k & (int)XK];
                        const bool neg = (__builtin_popcount((uint32_t)k & ZK) & 1) != 0;
                        const R a = neg ? -t.re : t.re, b = neg ? -t.im : t.im;
                        cmac(pr[c][k], pi[c][k], a, b, v[c][k]);
                    }
                if constexpr (!kEarlyRecord) {
                    __builtin_amdgcn_sched_barrier(0);
                    qn = rec[mi + 1];
                }
            }
        };
        for_each_class(class_loop, std::make_integer_sequence<int, ipow3(KB)>{});

        // PAIR: D = (-1)^{|r & zbase|} sum_e phi_e (-1)^{s_q0 e_0 + s_q1 e_1} L_e(r),
        // phi_e = Phi[idx = 3][e] (the entry with s_q0 = s_q1 = 0), L_e(r) =
        // W_e + sum_c w_{e,c} r_c: the lane bits here, the rest staged per row k.
        // The lane part of a thread's rows: l_e = sum over lane bits c of w_{e,c} tid_c.
        auto lane_forms = [&](const QRec& q, R (&l)[4]) {
            const R* w = T.w2 + ((size_t)q.tab * T.n_real + rc) * 4 * (M + 1);
#pragma unroll
            for (int e = 0; e < 4; ++e) l[e] = R(0);
#pragma unroll
            for (int c = 0; c < kLaneBits; ++c) {
                if (c >= (int)lb) break;
                const R b = (R)((tid >> c) & 1u);
#pragma unroll
                for (int e = 0; e < 4; ++e) l[e] = fma(w[e * (M + 1) + c], b, l[e]);
            }
        };
        // Flat PAIR masks (no flipped k bit), by the k bits ZK of their Z string
        // (compile-time row signs).  The qubit signs s_q0, s_q1 and the lane and
        // tile parts of the Z-string sign are the same on all of a thread's rows,
        // and L_e is linear in the k bits:
        //   D_k = (-1)^{|k & ZK|} (A + sum over set bits b of k of Om_b),
        //   A = (-1)^{s} sum_e phi_e sigma_e (l_e + t_{0,e}),
        //   Om_b = (-1)^{s} sum_e phi_e sigma_e w_{e,lb+b},
        // sigma_e = (-1)^{s_q0 e_0 + s_q1 e_1}: one complex add per row.
        auto flat_loop = [&](auto cls) {
            constexpr int ZK = decltype(cls)::value;
            const uint32_t n = (C.pcnt[ZK >> 2] >> (8 * (ZK & 3))) & 0xffu;
            for (uint32_t i = 0; i < n; ++i, ++mi) {
                const QRec q = rec[mi];
                const R* w = T.w2 + ((size_t)q.tab * T.n_real + rc) * 4 * (M + 1);
                const cplx<R>* ph = T.phi2 + (size_t)q.tab * 16 + 12;
                R l[4];
                lane_forms(q, l);
                const R* t0 = reinterpret_cast<const R*>(tab_b + q.sel);   // t_{0,e}
                const uint32_t rl = tid | base;
                const uint32_t sa = bit(rl, mask_q(q.qpack, 0)) ^ 1u, sbb = bit(rl, mask_q(q.qpack, 1)) ^ 1u;
                const uint32_t s = parity(rl & q.zbase);
                // sum_e phi_e sigma_e y_e, signed by s
                auto combine = [&](R y0, R y1, R y2, R y3) {
                    const R b1 = flip(y1, sa), b2 = flip(y2, sbb), b3 = flip(y3, sa ^ sbb);
                    cplx<R> o;
                    o.re = flip(ph[0].re * y0 + ph[1].re * b1 + ph[2].re * b2 + ph[3].re * b3, s);
                    o.im = flip(ph[0].im * y0 + ph[1].im * b1 + ph[2].im * b2 + ph[3].im * b3, s);
                    return o;
                };
                cplx<R> X[RPT];
                X[0] = combine(l[0] + t0[0], l[1] + t0[1], l[2] + t0[2], l[3] + t0[3]);
#pragma unroll
                for (int b = 0; b < KB; ++b) {
                    const int c = (int)lb + b;
                    const cplx<R> om = combine(w[c], w[(M + 1) + c], w[2 * (M + 1) + c], w[3 * (M + 1) + c]);
#pragma unroll
                    for (int k = 1 << b; k < (2 << b); ++k) {
                        X[k].re = X[k - (1 << b)].re + om.re;
                        X[k].im = X[k - (1 << b)].im + om.im;
                    }
                }
                const uint32_t sb = tid_b ^ q.xoff;
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        const bool neg = (__builtin_popcount((uint32_t)k & (uint32_t)ZK) & 1) != 0;
                        const cplx<R> v = src_row(c, sb + ((uint32_t)k << kLaneBits) * esz);
                        cmac(pr[c][k], pi[c][k], neg ? -X[k].re : X[k].re, neg ? -X[k].im : X[k].im, v);
                    }
            }
        };
        if (RPT > 1) {
            for_each_class(flat_loop, std::make_integer_sequence<int, RPT>{});
        } else {
            flat_loop(std::integral_constant<int, 0>{});
        }
        for (uint32_t i = n_flat; i < C.n_pair; ++i, ++mi) {
            const QRec q = rec[mi];
            const cplx<R>* ph = T.phi2 + (size_t)q.tab * 16 + 12;
            R l[4];
            lane_forms(q, l);
            const uint32_t q0 = mask_q(q.qpack, 0), q1 = mask_q(q.qpack, 1);
            const uint32_t rl = tid | base;
            const uint32_t sa_l = bit(rl, q0) ^ 1u, sb_l = bit(rl, q1) ^ 1u, s_l = parity(rl & q.zbase);
            const uint32_t sb = tid_b ^ q.xoff;
            const R* tk = reinterpret_cast<const R*>(tab_b + q.sel);
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const uint32_t kr = (uint32_t)k << lb;
                const uint32_t sa = sa_l ^ bit(kr, q0), sbb = sb_l ^ bit(kr, q1);
                const uint32_t s = s_l ^ parity(kr & q.zbase);
                const R a0 = l[0] + tk[k * 4 + 0];
                const R a1 = flip(l[1] + tk[k * 4 + 1], sa);
                const R a2 = flip(l[2] + tk[k * 4 + 2], sbb);
                const R a3 = flip(l[3] + tk[k * 4 + 3], sa ^ sbb);
                const R dre = flip(ph[0].re * a0 + ph[1].re * a1 + ph[2].re * a2 + ph[3].re * a3, s);
                const R dim = flip(ph[0].im * a0 + ph[1].im * a1 + ph[2].im * a2 + ph[3].im * a3, s);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const cplx<R> v = src_row(c, sb + (((uint32_t)k ^ q.koffs) << lb) * esz);
                    cmac(pr[c][k], pi[c][k], dre, dim, v);
                }
            }
        }
        // DIAG (source = own row): the precomputed diagonal of H
        for (uint32_t i = 0; i < C.n_diag; ++i, ++mi) {
            const double* dg = T.diag + (uint64_t)rc * L.dim + base + tid;
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const R d = (R)dg[(uint32_t)k << lb];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const cplx<R> v = src_row(c, tid_b + ((uint32_t)k << lb) * esz);
                    pr[c][k] = fma(d, v.re, pr[c][k]);
                    pi[c][k] = fma(d, v.im, pi[c][k]);
                }
            }
        }
        if (kSplit) carry();
    }

    // QUAD masks that flip only tile bits: D_x is one number per tile, the
    // source rows are the same rows of tile ^ x_high.  Streamed straight from
    // global memory with the next mask's rows loaded one mask ahead.
    if (L.n_far > 0) {
        cplx<R> vn[NC][RPT];
        FarRec fn = L.far[0];
        const cplx<R>* sp = psi + ((uint64_t)(tile ^ fn.x_high) << L.tile_bits);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int k = 0; k < RPT; ++k) vn[c][k] = (sp + c * L.dim)[tid + k * nt];
        for (int f = 0; f < L.n_far; ++f) {
            const FarRec fc = fn;
            cplx<R> v[NC][RPT];
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int k = 0; k < RPT; ++k) v[c][k] = vn[c][k];
            if (f + 1 < L.n_far) {
                fn = L.far[f + 1];
                sp = psi + ((uint64_t)(tile ^ fn.x_high) << L.tile_bits);
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int k = 0; k < RPT; ++k) vn[c][k] = (sp + c * L.dim)[tid + k * nt];
            }
            const cplx<R> t = T.tab4[((size_t)fc.tab * T.n_real + rc) * 16 + quad_index(base, fc.qpack)];
            const uint32_t s = parity(base & fc.zbase);
            const R tr = flip(t.re, s), ti = flip(t.im, s);
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int k = 0; k < RPT; ++k) cmac(pr[c][k], pi[c][k], tr, ti, v[c][k]);
            if (kSplit && (f & 63) == 63) carry();
        }
        if (kSplit) carry();
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            cplx<R> o;
            o.re = kSplit ? (R)acc_re[c][k] : pr[c][k];
            o.im = kSplit ? (R)acc_im[c][k] : pi[c][k];
            (out + c * L.dim)[(uint64_t)base + tid + k * nt] = o;
        }
}

// dst = transpose of src viewed as a [2^log_h] x [2^log_w] matrix (row-major),
// column by column of a block: dst[c][lo << log_h | hi] (+)= src[c][hi << log_w | lo].
// 32 x 32 tiles through LDS so that both sides are read and written along
// contiguous rows.  With ADD, complex64 sums are formed in FP64 and rounded once.
template <typename R, bool ADD>
__global__ void __launch_bounds__(256) k_transpose(const cplx<R>* __restrict__ src, cplx<R>* __restrict__ dst,
                                                   int log_h, int log_w, uint64_t dim)
{
    __shared__ cplx<R> t[32][33];
    const uint32_t lw = (uint32_t)log_w - 5u;
    const uint64_t bx = blockIdx.x & ((1u << lw) - 1u);   // tile column (lo / 32)
    const uint64_t by = blockIdx.x >> lw;                 // tile row (hi / 32)
    src += (uint64_t)blockIdx.y * dim;
    dst += (uint64_t)blockIdx.y * dim;
    const uint32_t tx = threadIdx.x & 31u, ty = threadIdx.x >> 5;
#pragma unroll
    for (uint32_t j = ty; j < 32; j += 8) t[j][tx] = src[((by * 32 + j) << log_w) | (bx * 32 + tx)];
    __syncthreads();
#pragma unroll
    for (uint32_t j = ty; j < 32; j += 8) {
        const uint64_t o = ((bx * 32 + j) << log_h) | (by * 32 + tx);
        cplx<R> v = t[tx][j];
        if (ADD) {
            const cplx<R> d = dst[o];
            v.re = (R)((double)v.re + (double)d.re);
            v.im = (R)((double)v.im + (double)d.im);
        }
        dst[o] = v;
    }
}

// diag[c][r] = sum_n dw[c][n] (-1)^{|r & dz_n|} for realisation c = blockIdx.y:
// the diagonal of H (the masks with x = 0), FP64.
__global__ void __launch_bounds__(256) k_diag_fill(const uint32_t* __restrict__ dz, const double* __restrict__ dw,
                                                   int n_diag, uint64_t dim, double* __restrict__ diag)
{
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= dim) return;
    const double* d = dw + (size_t)blockIdx.y * n_diag;
    double s = 0.0;
    for (int n = 0; n < n_diag; ++n) s += (__popc((uint32_t)r & dz[n]) & 1u) ? -d[n] : d[n];
    diag[(uint64_t)blockIdx.y * dim + r] = s;
}

// Fills H.diag the first time it is needed (on the stream, then waits for it).
void ensure_diag(const HamiltonianDev& H, hipStream_t s)
{
    if (H.diag_ready) return;
    const uint64_t dim = (uint64_t)1 << H.M;
    H.diag.ensure((size_t)H.n_real * dim * sizeof(double));
    const dim3 grid((uint32_t)((dim + 255) / 256), (uint32_t)H.n_real);
    hipLaunchKernelGGL(k_diag_fill, grid, dim3(256), 0, s, H.dz, H.dw_d, H.n_diag, dim, H.diag.as<double>());
    SYK_HIP(hipGetLastError());
    SYK_HIP(hipStreamSynchronize(s));   // once per handle: later calls may come on other streams
    H.diag_ready = true;
}

}  // namespace

void launch_transpose(syk_dtype dtype, const void* src, void* dst, int log_h, int log_w, int ncols, uint64_t dim,
                      bool add, hipStream_t s)
{
    if (log_h < 5 || log_w < 5 || log_h + log_w > 40) throw Error(SYK_EINVAL, "transpose: unsupported shape");
    dim3 grid((uint32_t)((dim >> 10)), ncols), block(256);
    if (dtype == SYK_C128) {
        auto* i = static_cast<const c128*>(src);
        auto* o = static_cast<c128*>(dst);
        if (add) hipLaunchKernelGGL((k_transpose<double, true>), grid, block, 0, s, i, o, log_h, log_w, dim);
        else hipLaunchKernelGGL((k_transpose<double, false>), grid, block, 0, s, i, o, log_h, log_w, dim);
    } else {
        auto* i = static_cast<const c64*>(src);
        auto* o = static_cast<c64*>(dst);
        if (add) hipLaunchKernelGGL((k_transpose<float, true>), grid, block, 0, s, i, o, log_h, log_w, dim);
        else hipLaunchKernelGGL((k_transpose<float, false>), grid, block, 0, s, i, o, log_h, log_w, dim);
    }
    SYK_HIP(hipGetLastError());
}

namespace {

template <typename R>
void launch_t(const ApplyPlan& P, const KTerms<R>& T, const QApplyChunk* chunks, const QRec* rec, KLayout L,
              int ncols, int nc, const void* psi, void* out, hipStream_t s)
{
    auto* in = static_cast<const cplx<R>*>(psi);
    auto* o = static_cast<cplx<R>*>(out);
    if (nc == 2) {
        // the caller has checked that the columns pair up by realisation
        if (ncols % 2 != 0) throw Error(SYK_EINVAL, "apply_H: odd column count for two columns per workgroup");
        dim3 grid(L.n_tiles, ncols / 2), block(P.nt);
        switch (P.rpt) {
        case 4: hipLaunchKernelGGL((k_apply<R, 4, 2>), grid, block, 0, s, T, chunks, rec, L, in, o); break;
        case 8: hipLaunchKernelGGL((k_apply<R, 8, 2>), grid, block, 0, s, T, chunks, rec, L, in, o); break;
        default: throw Error(SYK_EINVAL, "apply_H: two columns per workgroup need 4 or 8 rows per thread");
        }
    } else {
        dim3 grid(L.n_tiles, ncols), block(P.nt);
        switch (P.rpt) {
        case 1: hipLaunchKernelGGL((k_apply<R, 1, 1>), grid, block, 0, s, T, chunks, rec, L, in, o); break;
        case 2: hipLaunchKernelGGL((k_apply<R, 2, 1>), grid, block, 0, s, T, chunks, rec, L, in, o); break;
        case 4: hipLaunchKernelGGL((k_apply<R, 4, 1>), grid, block, 0, s, T, chunks, rec, L, in, o); break;
        case 8: hipLaunchKernelGGL((k_apply<R, 8, 1>), grid, block, 0, s, T, chunks, rec, L, in, o); break;
        default: throw Error(SYK_EINVAL, "apply_H: unsupported rows per thread");
        }
    }
    SYK_HIP(hipGetLastError());
}

// Chunks and class-sorted records of the apply kernel for tiles of 2^tile_bits
// rows, 2^lane_bits threads and elements of esz bytes.  masks must be sorted by
// x; QUAD masks that neither flip nor sign-depend on a row bit inside a tile go
// to the far list.
void build_apply_tables(const std::vector<MaskRec>& masks_in, int tile_bits, int lane_bits, uint32_t esz,
                        std::vector<QApplyChunk>& chunks, std::vector<QRec>& recs, std::vector<FarRec>& far)
{
    const uint32_t row_mask = (1u << tile_bits) - 1u;
    const uint32_t lane_mask = (1u << lane_bits) - 1u;
    const int kb = tile_bits - lane_bits;
    if (kb < 0 || kb > kMaxKBits) throw Error(SYK_EINVAL, "apply_H: unsupported rows per thread");
    const uint32_t kbits_mask = (1u << kb) - 1u;
    auto quad_class_of = [&](const MaskRec& m) { return quad_class(m.x, m.zbase, lane_bits, kb); };
    auto type_of = [](const MaskRec& m) { return m.type_tab >> 28; };
    auto xk_of = [&](const MaskRec& m) { return (m.x >> lane_bits) & kbits_mask; };
    // PAIR masks flipping no k bit, and the k-bit pattern of their Z string
    auto is_k_bit = [&](uint32_t q) { return q >= (uint32_t)lane_bits && q < (uint32_t)tile_bits; };
    auto flat_pair = [&](const MaskRec& m) {
        return type_of(m) == MASK_PAIR && !is_k_bit(mask_q(m.qpack, 0)) && !is_k_bit(mask_q(m.qpack, 1));
    };
    auto zk_of = [&](const MaskRec& m) { return (int)((m.zbase >> lane_bits) & kbits_mask); };
    // table slots (16 entries each) a mask stages
    auto slots_of = [&](const MaskRec& m) { return type_of(m) == MASK_DIAG ? 0u : 1u; };
    // Inside a run of one x_high: by lane flips, then by k flips, so that the
    // masks of a group are adjacent (a chunk boundary rarely splits one).
    std::vector<MaskRec> masks = masks_in;
    std::stable_sort(masks.begin(), masks.end(), [&](const MaskRec& a, const MaskRec& b) {
        const uint32_t ha = a.x >> tile_bits, hb = b.x >> tile_bits;
        if (ha != hb) return ha < hb;
        const uint32_t la = a.x & lane_mask, lb2 = b.x & lane_mask;
        if (la != lb2) return la < lb2;
        return xk_of(a) < xk_of(b);
    });
    size_t i = 0;
    uint32_t prev_high = 0xffffffffu;
    while (i < masks.size()) {
        // masks of one chunk: same x_high, at most apply_chunk_masks(esz)
        std::vector<uint32_t> mem;
        const uint32_t xh = masks[i].x >> tile_bits;
        const uint32_t cap = (uint32_t)apply_chunk_masks(esz);   // masks and table slots per chunk
        uint32_t used = 0;
        while (i < masks.size() && (masks[i].x >> tile_bits) == xh && mem.size() < cap) {
            const MaskRec& m = masks[i];
            // far: coefficient constant over a tile (no flipped qubit and no Z-string bit inside it)
            if (type_of(m) == MASK_QUAD && (m.x & row_mask) == 0u && (m.zbase & row_mask) == 0u) {
                far.push_back({m.x >> tile_bits, m.qpack, m.zbase, m.type_tab & 0x0fffffffu});
            } else {
                if (used + slots_of(m) > cap) break;
                used += slots_of(m);
                mem.push_back((uint32_t)i);
            }
            ++i;
        }
        if (mem.empty()) continue;
        const size_t nm = mem.size();
        // records (the PAIR / DIAG table offsets follow the final order)
        std::vector<QRec> rr(nm);
        std::vector<int> key(nm);
        for (size_t u = 0; u < nm; ++u) {
            const MaskRec& m = masks[mem[u]];
            const uint32_t t = type_of(m);
            QRec r{};
            r.zl = m.zbase & lane_mask;
            r.xoff = (m.x & lane_mask) * esz;
            r.tab = m.type_tab & 0x0fffffffu;
            r.xl = m.x & row_mask;
            r.qpack = m.qpack;
            r.zbase = m.zbase;
            if (t == MASK_QUAD) {
                for (int q = 0; q < 4; ++q) {
                    const uint32_t qb = mask_q(m.qpack, q);
                    r.sel |= (qb < (uint32_t)lane_bits ? qb : 0x0cu) << (8 * q);
                    const int b = (int)qb - lane_bits;
                    if (b >= 0 && b < kb) r.koffs |= ((1u << q) * esz) << (8 * b);
                }
                key[u] = 1000 + quad_class_of(m);
            } else {
                r.koffs = (m.x >> lane_bits) & kbits_mask;
                key[u] = t == MASK_PAIR ? (flat_pair(m) ? 2000 + zk_of(m) : 2500) : 3000;
            }
            rr[u] = r;
        }
        // Groups: three QUAD masks with the same lane flips that flip J = 1 or
        // 2 k bits in all three ways, whose classes are those of a group class
        // and whose records agree on what the kernel reads once per group.
        std::vector<int> gcls(nm, -1), gid(nm, 0), gpos(nm, 0);
        uint32_t group_kof[256] = {};
        int ng = 0;
        if (kb == kMaxKBits) {
            std::map<std::pair<uint32_t, int>, std::vector<size_t>> cand;
            for (size_t u = 0; u < nm; ++u) {
                const MaskRec& m = masks[mem[u]];
                const int J = __builtin_popcount(xk_of(m));
                if (type_of(m) == MASK_QUAD && (J == 1 || J == 2)) cand[{m.x & lane_mask, J}].push_back(u);
            }
            for (const auto& kv : cand) {
                const int J = kv.first.second;
                const std::vector<size_t>& v = kv.second;
                if (v.size() != 3) continue;
                size_t mj[3];
                bool ok = true;
                for (int j = 0; j < 3 && ok; ++j) {
                    ok = false;
                    for (size_t u : v)
                        if ((int)xk_of(masks[mem[u]]) == group_xk(J, j)) {
                            mj[j] = u;
                            ok = true;
                        }
                }
                if (!ok) continue;
                int gc = -1;
                for (int P = 0; P < 2 && gc < 0; ++P) {
                    const int g = 2 * (J - 1) + P;
                    bool all = true;
                    for (int j = 0; j < 3; ++j) all = all && quad_class_of(masks[mem[mj[j]]]) == group_member_class(g, j);
                    if (all) gc = g;
                }
                if (gc < 0) continue;
                const QRec& r0 = rr[mj[0]];
                const uint32_t kof = r0.koffs & 0xffu;   // index-bit offset of member 0's lowest flipped k bit
                ok = kof != 0u;
                for (int j = 0; j < 3 && ok; ++j) {
                    const QRec& r = rr[mj[j]];
                    ok = r.sel == r0.sel && r.zl == r0.zl && r.xoff == r0.xoff;
                    uint32_t want = 0, t = 0;
                    for (int b = 0; b < kMaxKBits; ++b)
                        if ((group_xk(J, j) >> b) & 1) want |= (kof << t++) << (8 * b);
                    ok = ok && r.koffs == want;
                }
                if (!ok) continue;
                for (int j = 0; j < 3; ++j) {
                    gcls[mj[j]] = gc;
                    gid[mj[j]] = ng;
                    gpos[mj[j]] = j;
                }
                group_kof[ng++] = kof;
            }
        }
        std::vector<size_t> ord(nm);
        for (size_t u = 0; u < nm; ++u) ord[u] = u;
        auto okey = [&](size_t u) {
            return gcls[u] >= 0 ? std::make_tuple(gcls[u], gid[u], gpos[u]) : std::make_tuple(key[u], 0, 0);
        };
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return okey(a) < okey(b); });
        QApplyChunk c{};
        c.x_high = xh;
        c.first = (uint32_t)recs.size();
        c.new_tile = (xh != prev_high) ? 1u : 0u;
        prev_high = xh;
        uint32_t slot = 0;
        for (size_t u : ord) {
            const MaskRec& m = masks[mem[u]];
            const uint32_t t = type_of(m);
            QRec r = rr[u];
            if (t == MASK_QUAD) {
                ++c.n_quad;
                if (gcls[u] >= 0) {
                    if (gpos[u] == 0) {
                        const int g = kQuadClasses + gcls[u];
                        c.cnt[g >> 2] += 1u << (8 * (g & 3));
                        r.koffs = group_kof[gid[u]];
                    }
                } else {
                    const int cls = quad_class_of(m);
                    c.cnt[cls >> 2] += 1u << (8 * (cls & 3));
                }
            } else {
                r.sel = slot * 16u * esz;
                if (t == MASK_PAIR) {
                    ++c.n_pair;
                    if (flat_pair(m)) {
                        const int zk = zk_of(m);
                        c.pcnt[zk >> 2] += 1u << (8 * (zk & 3));
                    }
                } else {
                    ++c.n_diag;
                }
            }
            slot += slots_of(m);
            recs.push_back(r);
        }
        chunks.push_back(c);
    }
    recs.push_back(QRec{});   // one record past the end: loads may run one ahead
}

// Bit rotation of the second layout: bits s..M-1 of a row become bits
// 0..M-s-1 and bits 0..s-1 become the top bits.
inline uint32_t rotate_bits(uint32_t v, int M, int s)
{
    return (v >> s) | ((v & ((1u << s) - 1u)) << (M - s));
}

}  // namespace

bool quad_in_rotated(const MaskRec& m, int M, int tb)
{
    if ((m.type_tab >> 28) != MASK_QUAD) return false;
    const uint32_t row_mask = (1u << tb) - 1u;
    const int out_a = __builtin_popcount(m.x & ~row_mask);
    const int out_b = __builtin_popcount(rotate_bits(m.x, M, tb) & ~row_mask);
    return out_b < out_a;
}

MaskRec rotate_mask(const MaskRec& m, int M, int tb)
{
    MaskRec r = m;
    r.x = rotate_bits(m.x, M, tb);
    r.zbase = rotate_bits(m.zbase, M, tb);
    r.qpack = 0;   // table index bit q stays bit q; only its qubit moves
    for (int q = 0; q < 4; ++q) {
        const int b = (int)mask_q(m.qpack, q);   // 31: placeholder of an unused index bit
        r.qpack |= (uint32_t)(b == 31 ? 31 : b >= tb ? b - tb : b + (M - tb)) << (8 * q);
    }
    return r;
}

namespace {

// Masks of one layout, in that layout's row coordinates and sorted by x.  With
// two layouts, a QUAD mask goes to the rotated layout (1) when fewer of its
// flipped qubits lie outside a tile there; everything else stays in layout 0.
// A relabelling of qubits keeps every coefficient: only x, zbase and the
// qubit of each table index bit move.
std::vector<MaskRec> layout_masks(const std::vector<MaskRec>& masks, int M, int tb, bool two, int layout)
{
    std::vector<MaskRec> out;
    for (const MaskRec& m : masks) {
        const int in_b = two && quad_in_rotated(m, M, tb);
        if (in_b != layout) continue;
        out.push_back(layout == 0 ? m : rotate_mask(m, M, tb));
    }
    std::stable_sort(out.begin(), out.end(), [](const MaskRec& a, const MaskRec& b) { return a.x < b.x; });
    return out;
}

}  // namespace

std::vector<KRec> build_krecs(const std::vector<MaskRec>& masks, const std::vector<uint64_t>& bin_off, int tile_bits)
{
    const uint32_t row_mask = (1u << tile_bits) - 1u;
    std::vector<KRec> out(masks.size());
    for (size_t i = 0; i < masks.size(); ++i) {
        const MaskRec& m = masks[i];
        const uint32_t type = m.type_tab >> 28, tab = m.type_tab & 0x0fffffffu;
        KRec k{};
        k.xl = m.x & row_mask;
        k.qpack = m.qpack;
        k.zbase = m.zbase;
        k.meta = type << 28 | tab;
        k.bin0 = (uint32_t)bin_off[i];
        k.x_high = m.x >> tile_bits;
        out[i] = k;
    }
    return out;
}

namespace {

int apply_tables_key(const ApplyPlan& P, uint32_t esz, int layout)
{
    return (((P.tile_bits * 16 + P.lb) * 32 + (int)esz) * 2 + P.two_layouts) * 2 + layout;
}

const HamiltonianDev::ApplyTables& apply_tables_for(const HamiltonianDev& H, const ApplyPlan& P, uint32_t esz,
                                                    int layout)
{
    const int key = apply_tables_key(P, esz, layout);
    auto it = H.apply_tables.find(key);
    if (it == H.apply_tables.end()) {
        std::vector<QApplyChunk> ch;
        std::vector<QRec> rc;
        std::vector<FarRec> far;
        const std::vector<MaskRec> masks = layout_masks(*H.host_masks, H.M, P.tile_bits, P.two_layouts != 0, layout);
        build_apply_tables(masks, P.tile_bits, P.lb, esz, ch, rc, far);
        std::unique_ptr<HamiltonianDev::ApplyTables> t(new HamiltonianDev::ApplyTables());
        t->n_chunks = (int)ch.size();
        t->n_far = (int)far.size();
        if (!ch.empty()) {
            t->chunks.ensure(ch.size() * sizeof(QApplyChunk));
            SYK_HIP(hipMemcpy(t->chunks.p, ch.data(), ch.size() * sizeof(QApplyChunk), hipMemcpyHostToDevice));
        }
        if (!far.empty()) {
            t->far.ensure(far.size() * sizeof(FarRec));
            SYK_HIP(hipMemcpy(t->far.p, far.data(), far.size() * sizeof(FarRec), hipMemcpyHostToDevice));
        }
        t->recs.ensure(rc.size() * sizeof(QRec));
        SYK_HIP(hipMemcpy(t->recs.p, rc.data(), rc.size() * sizeof(QRec), hipMemcpyHostToDevice));
        it = H.apply_tables.emplace(key, std::move(t)).first;
    }
    return *it->second;
}

}  // namespace

ApplyPlan plan_apply(int M, int nvec, syk_dtype dtype, const ApplyTuning* tune)
{
    ApplyPlan P{};
    P.slices = (nvec + kColsPerLaunch - 1) / kColsPerLaunch;
    // 2048-row source tiles (256 threads, 8 rows each); smaller tiles when the
    // columns would not fill the chip.
    int tb = std::min(M, 11);
    while (tb > 8 && ((int64_t)1 << (M - tb)) * nvec < 2048) --tb;
    if (tune && tune->tile_bits > 0) tb = std::min(tune->tile_bits, M);
    // 8 lane bits; a thread owns 2^(tile_bits - 8) rows, at most 8
    if (tb > kLaneBits + kMaxKBits) throw Error(SYK_EINVAL, "apply_H: tile_bits above 11");
    P.tile_bits = tb;
    P.lb = std::min(tb, kLaneBits);
    P.nt = 1 << P.lb;
    P.rpt = 1 << (tb - P.lb);
    P.xcd_remap = tune ? tune->xcd_remap : 1;
    // Two columns of one realisation per workgroup (where a launch's columns
    // pair up) need a whole 256-thread workgroup with at least 4 rows per
    // thread.  By default complex64 takes them: its 8-row kernel holds both
    // columns' sums at three waves per SIMD and decodes each mask once for
    // both; complex128 would drop to two waves per SIMD and gains nothing.
    const bool explicit_cols = tune && tune->cols > 0;
    P.nc = explicit_cols ? tune->cols : (dtype == SYK_C64 ? 2 : 1);
    if (P.nc == 2 && P.rpt < 4) {
        if (explicit_cols && tune->tile_bits > 0)
            throw Error(SYK_EINVAL, "apply_H: two columns per workgroup need tile_bits >= 10");
        P.nc = 1;
    }
    // QUAD masks whose four qubits all lie above the tile would each stream a
    // whole tile from global memory; with at least C(7,4) of them, run the
    // masks that sit better in the rotated layout there.
    P.two_layouts = (M - tb >= 7 && tb >= 8) ? 1 : 0;
    return P;
}

namespace {
void launch_apply_impl(const HamiltonianDev& H, syk_dtype dtype, int nvec, const int32_t* real_of_col,
                       const void* psi, void* out, const ApplyPlan& P, hipStream_t s, void* rot_in, void* rot_out,
                       bool timed);
}  // namespace

// Scratch of the allocation-free apply (syk_apply_H_noalloc): the rotated
// copy of psi and the rotated layout's output of one call, side by side.  Each
// device holds its own copy for the life of the process; host code reaches it
// only through the address hipGetSymbolAddress returns on that device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

void* noalloc_scratch_ptr(int device)
{
    static std::mutex mu;
    static std::map<int, void*> ptr;   // per device, set once with that device current
    std::lock_guard<std::mutex> l(mu);
    auto it = ptr.find(device);
    if (it != ptr.end()) return it->second;
    int cur = -1;
    SYK_HIP(hipGetDevice(&cur));
    if (cur != device) throw Error(SYK_EINVAL, "apply_H_noalloc: the handle's device is not the current device");
    void* p = nullptr;
    SYK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(SYK_EHIP, "apply_H_noalloc: no device address for the scratch array");
    ptr.emplace(device, p);
    return p;
}

void launch_apply_h_noalloc(const HamiltonianDev& H, int device, syk_dtype dtype, int nvec,
                            const int32_t* real_of_col, const void* psi, void* out, const ApplyPlan& P,
                            hipStream_t s)
{
    const size_t esz = elem_bytes(dtype);
    const uint64_t dim = (uint64_t)1 << H.M;
    const size_t half = (size_t)std::min(nvec, kColsPerLaunch) * dim * esz;
    if (P.two_layouts && 2 * half > kNoAllocScratchBytes)
        throw Error(SYK_EINVAL, "apply_H_noalloc: the rotated layout needs " + std::to_string(2 * half) +
                                    " bytes of scratch, above the maximum of " +
                                    std::to_string(kNoAllocScratchBytes));
    // everything the handle builds on first use must exist already
    auto have = [&](int layout) { return H.apply_tables.count(apply_tables_key(P, (uint32_t)esz, layout)) != 0; };
    if (!H.diag_ready || !have(0) || (P.two_layouts && !have(1)))
        throw Error(SYK_EINVAL, "apply_H_noalloc: the handle has no tables for this dtype and block width yet "
                                "(call syk_apply_H once with them first)");
    char* sp = P.two_layouts ? static_cast<char*>(noalloc_scratch_ptr(device)) : nullptr;
    launch_apply_impl(H, dtype, nvec, real_of_col, psi, out, P, s, sp, sp ? sp + half : nullptr, false);
}

void launch_apply_h(const HamiltonianDev& H, syk_dtype dtype, int nvec, const int32_t* real_of_col,
                    const void* psi, void* out, const ApplyPlan& P, hipStream_t s)
{
    const bool two = P.two_layouts != 0;
    if (two) {
        const size_t bytes = (size_t)std::min(nvec, kColsPerLaunch) * ((uint64_t)1 << H.M) * elem_bytes(dtype);
        H.rot_in.ensure(bytes);
        H.rot_out.ensure(bytes);
    }
    ensure_diag(H, s);
    launch_apply_impl(H, dtype, nvec, real_of_col, psi, out, P, s, two ? H.rot_in.p : nullptr,
                      two ? H.rot_out.p : nullptr, true);
}

namespace {

// The launches of one apply_H call; rot_in / rot_out: state-sized buffers of
// min(nvec, 64) columns for two-layout plans.  Allocates nothing.
void launch_apply_impl(const HamiltonianDev& H, syk_dtype dtype, int nvec, const int32_t* real_of_col,
                       const void* psi, void* out, const ApplyPlan& P, hipStream_t s, void* rot_in, void* rot_out,
                       bool timed)
{
    const int M = H.M;
    if (P.lb > kLaneBits || (P.rpt > 1 && P.lb != kLaneBits) || P.nt != (1 << P.lb) ||
        (P.nc != 1 && (P.nc != 2 || P.rpt < 4)) ||
        (P.rpt << P.lb) != (1 << P.tile_bits) || P.tile_bits > M ||
        (P.two_layouts && (P.tile_bits < 5 || M - P.tile_bits < 5)))
        throw Error(SYK_EINVAL, "apply_H: inconsistent launch shape");
    const size_t esz = elem_bytes(dtype);
    const uint64_t dim = (uint64_t)1 << M;
    const HamiltonianDev::ApplyTables& A = apply_tables_for(H, P, (uint32_t)esz, 0);
    const HamiltonianDev::ApplyTables* B = P.two_layouts ? &apply_tables_for(H, P, (uint32_t)esz, 1) : nullptr;
    if (B && (!rot_in || !rot_out)) throw Error(SYK_EINVAL, "apply_H: no buffers for the rotated layout");
    if (timed) timing_begin(s);
    for (int sl = 0; sl < P.slices; ++sl) {
        KLayout L{};
        L.tile_bits = P.tile_bits;
        L.lane_bits = P.lb;
        L.dim = dim;
        L.col0 = 0;
        L.n_tiles = (uint32_t)(dim >> P.tile_bits);
        L.xcd_remap = P.xcd_remap;
        const int col0 = sl * kColsPerLaunch;
        const int ncols = std::min(kColsPerLaunch, nvec - col0);
        for (int c = 0; c < ncols; ++c) L.real[c] = real_of_col ? real_of_col[col0 + c] : 0;
        // two columns per workgroup only where every pair of the slice shares its realisation
        int nc = P.nc;
        if (nc == 2 && ncols % 2 != 0) nc = 1;
        for (int c = 0; nc == 2 && c < ncols; c += 2)
            if (L.real[c] != L.real[c + 1]) nc = 1;
        const char* in_c = static_cast<const char*>(psi) + (size_t)col0 * dim * esz;
        char* out_c = static_cast<char*>(out) + (size_t)col0 * dim * esz;
        auto run = [&](const HamiltonianDev::ApplyTables& Tb, const void* src, void* dst) {
            L.far = Tb.far.as<FarRec>();
            L.n_far = Tb.n_far;
            L.n_chunks = Tb.n_chunks;
            const auto* ch = Tb.chunks.as<QApplyChunk>();
            const auto* rc = Tb.recs.as<QRec>();
            if (dtype == SYK_C128) {
                KTerms<double> T{H.tab4_d, H.qinfo, H.phi2_d, H.w2_d, H.diag.as<double>(), H.n_real, M};
                launch_t<double>(P, T, ch, rc, L, ncols, nc, src, dst, s);
            } else {
                KTerms<float> T{H.tab4_f, H.qinfo, H.phi2_f, H.w2_f, H.diag.as<double>(), H.n_real, M};
                launch_t<float>(P, T, ch, rc, L, ncols, nc, src, dst, s);
            }
        };
        if (B) {
            // rows r -> rotate_bits(r): a [2^(M-s)] x [2^s] transpose
            launch_transpose(dtype, in_c, rot_in, M - P.tile_bits, P.tile_bits, ncols, dim, false, s);
            run(*B, rot_in, rot_out);
            run(A, in_c, out_c);
            launch_transpose(dtype, rot_out, out_c, P.tile_bits, M - P.tile_bits, ncols, dim, true, s);
        } else {
            run(A, in_c, out_c);
        }
    }
    if (timed) timing_end(s);
}

}  // namespace

}  // namespace syk
