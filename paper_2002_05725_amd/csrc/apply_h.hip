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
// Grid: (tiles, columns); every workgroup serves one column and that column's
// realisation, so mask records, PAIR weights and DIAG terms are wave-uniform
// (scalar loads) and the chunk's QUAD tables are staged into LDS next to the
// source tile.  Up to 64 columns per launch.
#include "apply_h.hpp"
#include "timing.hpp"

namespace syk {

namespace {

template <typename R>
struct KTerms {
    const MaskRec* __restrict__ masks;
    const Group* __restrict__ groups;
    const cplx<R>* __restrict__ tab4;
    const uint32_t* __restrict__ qinfo;
    const cplx<R>* __restrict__ phi2;
    const R* __restrict__ w2;
    const uint32_t* __restrict__ dz;
    const R* __restrict__ dw;
    int n_groups, n_diag, n_real, M;
};

struct KLayout {
    const FarRec* __restrict__ far;   // QUAD masks flipping only tile bits
    int n_far;
    int tile_bits;     // rows per tile = 2^tile_bits
    uint64_t dim;      // rows per column
    int col0;          // first column of this launch (column = col0 + blockIdx.y)
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

// 4-bit QUAD table index: bit m = bit q_m of r.
__device__ __forceinline__ uint32_t quad_index(uint32_t r, uint32_t qpack)
{
    return bit(r, mask_q(qpack, 0)) | (bit(r, mask_q(qpack, 1)) << 1) | (bit(r, mask_q(qpack, 2)) << 2) |
           (bit(r, mask_q(qpack, 3)) << 3);
}

}  // namespace

namespace {

// Thread layout of the single-vector kernel: row rl = tid + k * nt of the tile
// (nt = 2^lane_bits threads, k < RPT).  A row index splits into lane bits
// (tid, per lane), row bits (k, the same for every lane) and tile bits (base,
// the same for the workgroup).  The tile bits of every QUAD table index and
// sign are folded into the tables while they are staged; the row bits come
// from the mask record; only the lane bits are computed per thread, once per
// mask.
template <typename R, int RPT>
__global__ void __launch_bounds__(RPT >= 8 ? 256 : 1024) k_apply_single(KTerms<R> T, const KRec* __restrict__ krec, KLayout L,
                                                       const cplx<R>* __restrict__ psi, cplx<R>* __restrict__ out)
{
    static_assert(RPT <= 12, "row info holds 12 rows");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const uint32_t nt = blockDim.x;
    const uint32_t tile_elems = nt * RPT;               // == 2^tile_bits
    cplx<R>* src = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* tabs = src + tile_elems;                   // kChunkMasks x 16 entries

    const uint32_t tile = tile_of_block(blockIdx.x, L);
    const uint32_t row_mask = (1u << L.tile_bits) - 1u;
    const uint32_t kmask = row_mask & ~(nt - 1u);       // row bits that vary with k
    const uint32_t tid = threadIdx.x;
    const int rc = L.real[blockIdx.y];
    const int M = T.M;
    const uint32_t base = tile << L.tile_bits;
    psi += (uint64_t)(L.col0 + blockIdx.y) * L.dim;   // this workgroup's column
    out += (uint64_t)(L.col0 + blockIdx.y) * L.dim;

    // complex128 sums directly in pr/pi; complex64 sums each chunk in FP32 and
    // carries the running total in FP64.
    constexpr bool kSplit = sizeof(R) < sizeof(double);
    double acc_re[RPT], acc_im[RPT];
    R pr[RPT], pi[RPT];
    uint32_t roff[RPT];   // LDS byte offset of the thread's rows
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        acc_re[k] = acc_im[k] = 0.0;
        pr[k] = pi[k] = R(0);
        roff[k] = (tid + k * nt) * (uint32_t)sizeof(cplx<R>);
    }
    auto lds = [&](uint32_t byte_off) -> cplx<R> {
        return *reinterpret_cast<const cplx<R>*>(smem_raw + byte_off);
    };

    for (int g = 0; g < T.n_groups; ++g) {
        const Group G = T.groups[g];
        __syncthreads();   // previous chunk is done with src / tabs
        if (G.new_tile) {
            const uint64_t sbase = (uint64_t)(tile ^ G.x_high) << L.tile_bits;
#pragma unroll
            for (int k = 0; k < RPT; ++k) src[tid + k * nt] = psi[sbase + tid + k * nt];
        }
        // Staged QUAD table entry i of mask j: sign_tile * T[i ^ index_tile].
        for (uint32_t e = tid; e < G.n_quad * 16; e += nt) {
            const uint32_t qt = G.quad_first + (e >> 4);
            const uint32_t qp = T.qinfo[2 * qt], zb = T.qinfo[2 * qt + 1];
            const cplx<R> c = T.tab4[((size_t)qt * T.n_real + rc) * 16 + ((e & 15u) ^ quad_index(base, qp))];
            const uint32_t sg = parity(base & zb);
            cplx<R> o;
            o.re = flip(c.re, sg);
            o.im = flip(c.im, sg);
            tabs[e] = o;
        }
        __syncthreads();

        for (uint32_t mi = G.first; mi < G.first + G.count; ++mi) {
            const KRec m = krec[mi];
            const uint32_t type = m.meta >> 28;
            const uint32_t tab = m.meta & 0x03ffffffu;
            const uint32_t xlb = m.xl * (uint32_t)sizeof(cplx<R>);
            if (type == MASK_QUAD) {
                const uint32_t path = (m.meta >> 26) & 3u;
                const cplx<R>* tq = tabs + (tab - G.quad_first) * 16;
                const uint32_t il = quad_index(tid, m.qpack);   // lane bits of the index
                const uint32_t sl = parity(tid & m.zbase);      // lane bits of the sign
                if (path != PATH_FULL) {
                    const cplx<R> t = tq[il];
                    const R tr = flip(t.re, sl), ti = flip(t.im, sl);
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        const uint32_t sk = (path == PATH_SIGN) ? (m.kinfo[k / 6] >> (5 * (k % 6) + 4)) & 1u : 0u;
                        const R a = flip(tr, sk), b = flip(ti, sk);
                        const cplx<R> v = lds(roff[k] ^ xlb);
                        pr[k] = fma(a, v.re, pr[k]);
                        pr[k] = fma(-b, v.im, pr[k]);
                        pi[k] = fma(a, v.im, pi[k]);
                        pi[k] = fma(b, v.re, pi[k]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        const uint32_t ki = (m.kinfo[k / 6] >> (5 * (k % 6))) & 31u;
                        const cplx<R> t = tq[il | (ki & 15u)];
                        const uint32_t s = sl ^ (ki >> 4);
                        const R a = flip(t.re, s), b = flip(t.im, s);
                        const cplx<R> v = lds(roff[k] ^ xlb);
                        pr[k] = fma(a, v.re, pr[k]);
                        pr[k] = fma(-b, v.im, pr[k]);
                        pi[k] = fma(a, v.im, pi[k]);
                        pi[k] = fma(b, v.re, pi[k]);
                    }
                }
            } else if (type == MASK_PAIR) {
                // D = (-1)^{|r & zbase|} sum_e phi_e (-1)^{s_q0 e_0 + s_q1 e_1} L_e(r),
                // phi_e = Phi[idx = 3][e] (the entry with s_q0 = s_q1 = 0),
                // L_e(r) = W_e + sum_c w_{e,c} r_c split into lane/tile bits (once)
                // and row bits (per k).
                const R* w = T.w2 + ((size_t)tab * T.n_real + rc) * 4 * (M + 1);
                const cplx<R>* ph = T.phi2 + (size_t)tab * 16 + 12;
                R l0 = w[M], l1 = w[(M + 1) + M], l2 = w[2 * (M + 1) + M], l3 = w[3 * (M + 1) + M];
                for (int c = 0; c < M; ++c) {
                    if ((1u << c) & kmask) continue;
                    const R b = (R)bit(tid | base, c);
                    l0 = fma(w[c], b, l0);
                    l1 = fma(w[(M + 1) + c], b, l1);
                    l2 = fma(w[2 * (M + 1) + c], b, l2);
                    l3 = fma(w[3 * (M + 1) + c], b, l3);
                }
                const uint32_t sl = parity(tid & m.zbase);
                const uint32_t q0 = mask_q(m.qpack, 0), q1 = mask_q(m.qpack, 1);
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const uint32_t ru = base | (k * nt);
                    R k0 = l0, k1 = l1, k2 = l2, k3 = l3;
                    for (uint32_t rb = ru & kmask; rb; rb &= rb - 1) {
                        const int c = __ffs(rb) - 1;
                        k0 += w[c];
                        k1 += w[(M + 1) + c];
                        k2 += w[2 * (M + 1) + c];
                        k3 += w[3 * (M + 1) + c];
                    }
                    const uint32_t r = tid | ru;
                    const uint32_t sa = bit(r, q0) ^ 1u, sb = bit(r, q1) ^ 1u;
                    k1 = flip(k1, sa);
                    k2 = flip(k2, sb);
                    k3 = flip(k3, sa ^ sb);
                    const uint32_t s = sl ^ parity(ru & m.zbase);
                    const R dre = flip(ph[0].re * k0 + ph[1].re * k1 + ph[2].re * k2 + ph[3].re * k3, s);
                    const R dim = flip(ph[0].im * k0 + ph[1].im * k1 + ph[2].im * k2 + ph[3].im * k3, s);
                    const cplx<R> v = lds(roff[k] ^ xlb);
                    pr[k] = fma(dre, v.re, pr[k]);
                    pr[k] = fma(-dim, v.im, pr[k]);
                    pi[k] = fma(dre, v.im, pi[k]);
                    pi[k] = fma(dim, v.re, pi[k]);
                }
            } else {  // MASK_DIAG
                const R* d = T.dw + (size_t)rc * T.n_diag;
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const uint32_t r = base | (tid + k * nt);
                    const cplx<R> v = lds(roff[k] ^ xlb);
                    R s = R(0);
                    for (int n = 0; n < T.n_diag; ++n) s += flip(d[n], parity(r & T.dz[n]));
                    pr[k] = fma(s, v.re, pr[k]);
                    pi[k] = fma(s, v.im, pi[k]);
                }
            }
        }
        if (kSplit) {
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                acc_re[k] += (double)pr[k];
                acc_im[k] += (double)pi[k];
                pr[k] = pi[k] = R(0);
            }
        }
    }

    // QUAD masks that flip only tile bits: D_x is one number per tile, the
    // source rows are the same rows of tile ^ x_high.  Streamed straight from
    // global memory with the next mask's rows loaded one mask ahead.
    if (L.n_far > 0) {
        cplx<R> vn[RPT];
        FarRec fn = L.far[0];
        const cplx<R>* sp = psi + ((uint64_t)(tile ^ fn.x_high) << L.tile_bits);
#pragma unroll
        for (int k = 0; k < RPT; ++k) vn[k] = sp[tid + k * nt];
        for (int f = 0; f < L.n_far; ++f) {
            const FarRec fc = fn;
            cplx<R> v[RPT];
#pragma unroll
            for (int k = 0; k < RPT; ++k) v[k] = vn[k];
            if (f + 1 < L.n_far) {
                fn = L.far[f + 1];
                sp = psi + ((uint64_t)(tile ^ fn.x_high) << L.tile_bits);
#pragma unroll
                for (int k = 0; k < RPT; ++k) vn[k] = sp[tid + k * nt];
            }
            const cplx<R> t = T.tab4[((size_t)fc.tab * T.n_real + rc) * 16 + quad_index(base, fc.qpack)];
            const uint32_t s = parity(base & fc.zbase);
            const R tr = flip(t.re, s), ti = flip(t.im, s);
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                pr[k] = fma(tr, v[k].re, pr[k]);
                pr[k] = fma(-ti, v[k].im, pr[k]);
                pi[k] = fma(tr, v[k].im, pi[k]);
                pi[k] = fma(ti, v[k].re, pi[k]);
            }
            if (kSplit && (f & 63) == 63) {
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    acc_re[k] += (double)pr[k];
                    acc_im[k] += (double)pi[k];
                    pr[k] = pi[k] = R(0);
                }
            }
        }
        if (kSplit) {
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                acc_re[k] += (double)pr[k];
                acc_im[k] += (double)pi[k];
                pr[k] = pi[k] = R(0);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        cplx<R> o;
        o.re = kSplit ? (R)acc_re[k] : pr[k];
        o.im = kSplit ? (R)acc_im[k] : pi[k];
        out[(uint64_t)base + tid + k * nt] = o;
    }
}

inline int ilog2(int64_t v)
{
    int l = 0;
    while ((int64_t(1) << (l + 1)) <= v) ++l;
    return l;
}

template <typename R>
void launch_t(const ApplyPlan& P, const KTerms<R>& T, const KRec* krec, KLayout L, int ncols, const void* psi,
              void* out, hipStream_t s)
{
    dim3 grid(L.n_tiles, ncols), block(P.nt);
    const size_t lds = ((size_t)1 << P.tile_bits) * sizeof(cplx<R>) + (size_t)kChunkMasks * 16 * sizeof(cplx<R>);
    auto* in = static_cast<const cplx<R>*>(psi);
    auto* o = static_cast<cplx<R>*>(out);
    switch (P.rpt) {
    case 1: hipLaunchKernelGGL((k_apply_single<R, 1>), grid, block, lds, s, T, krec, L, in, o); break;
    case 2: hipLaunchKernelGGL((k_apply_single<R, 2>), grid, block, lds, s, T, krec, L, in, o); break;
    case 4: hipLaunchKernelGGL((k_apply_single<R, 4>), grid, block, lds, s, T, krec, L, in, o); break;
    case 8: hipLaunchKernelGGL((k_apply_single<R, 8>), grid, block, lds, s, T, krec, L, in, o); break;
    default: throw Error(SYK_EINVAL, "apply_H: unsupported rows per thread");
    }
    SYK_HIP(hipGetLastError());
}

// Mask records for launch shape (tile_bits, nt), in mask order.
std::vector<KRec> build_krecs(const std::vector<MaskRec>& masks, const std::vector<uint64_t>& bin_off, int tile_bits,
                             int nt)
{
    const uint32_t row_mask = (1u << tile_bits) - 1u;
    const uint32_t kmask = row_mask & ~((uint32_t)nt - 1u);
    const int rpt = (1 << tile_bits) / nt;
    std::vector<KRec> out(masks.size());
    for (size_t i = 0; i < masks.size(); ++i) {
        const MaskRec& m = masks[i];
        KRec k{};
        k.xl = m.x & row_mask;
        k.qpack = m.qpack;
        k.zbase = m.zbase;
        const uint32_t type = m.type_tab >> 28, tab = m.type_tab & 0x0fffffffu;
        uint32_t path = PATH_SAME;
        if (type == MASK_QUAD) {
            if (m.x & kmask) path = PATH_FULL;
            else if (m.zbase & kmask) path = PATH_SIGN;
            for (int r = 0; r < rpt && r < 12; ++r) {
                const uint32_t ru = (uint32_t)r * (uint32_t)nt;
                uint32_t ik = 0;
                for (int j = 0; j < 4; ++j) ik |= ((ru >> mask_q(m.qpack, j)) & 1u) << j;
                const uint32_t sk = (uint32_t)__builtin_popcount(ru & m.zbase) & 1u;
                k.kinfo[r / 6] |= (ik | sk << 4) << (5 * (r % 6));
            }
        }
        if (tab >= (1u << 26)) throw Error(SYK_EUNSUPPORTED, "apply_H: too many masks");
        k.meta = type << 28 | path << 26 | tab;
        k.pad[0] = (uint32_t)bin_off[i];
        out[i] = k;
    }
    return out;
}

}  // namespace

const KRec* krecs_for(const HamiltonianDev& H, const ApplyPlan& P)
{
    const int key = P.tile_bits * 4096 + P.nt;
    auto it = H.krecs.find(key);
    if (it == H.krecs.end()) {
        if (H.bin_off->size() != H.host_masks->size()) throw Error(SYK_EINVAL, "apply_H: handle tables incomplete");
        std::vector<KRec> v = build_krecs(*H.host_masks, *H.bin_off, P.tile_bits, P.nt);
        std::unique_ptr<DevBuf> b(new DevBuf());
        b->ensure(v.size() * sizeof(KRec));
        SYK_HIP(hipMemcpy(b->p, v.data(), v.size() * sizeof(KRec), hipMemcpyHostToDevice));
        it = H.krecs.emplace(key, std::move(b)).first;
    }
    return it->second->as<KRec>();
}

ApplyPlan plan_apply(int M, int nvec, syk_dtype dtype, const ApplyTuning* tune)
{
    ApplyPlan P{};
    P.slices = (nvec + kColsPerLaunch - 1) / kColsPerLaunch;
    // 2048-row source tiles with 512 threads (4 rows each): measured best at
    // N=44 and N=52; smaller tiles when the columns would not fill the chip.
    int tb = std::min(M, 11);
    while (tb > 8 && ((int64_t)1 << (M - tb)) * nvec < 2048) --tb;
    int nt_pref = 512;
    if (tune && tune->tile_bits > 0) {
        // at most 64 KiB of LDS per tile
        const int lim = (dtype == SYK_C128) ? 12 : 13;
        tb = std::max(0, std::min(std::min(tune->tile_bits, M), lim));
    }
    if (tune && tune->threads > 0) nt_pref = tune->threads;
    P.tile_bits = tb;
    const int elems = 1 << tb;
    // up to 8 rows per thread with <= 256 threads, 4 rows beyond
    auto rpt_cap = [](int nt) { return nt > 256 ? 4 : 8; };
    P.nt = std::min(nt_pref, elems);
    while (elems / P.nt > rpt_cap(P.nt) && P.nt < 1024) P.nt *= 2;
    P.rpt = elems / P.nt;
    if (P.rpt > rpt_cap(P.nt) || P.rpt * P.nt != elems)
        throw Error(SYK_EINVAL, "apply_H: tile does not fit the launch shape");
    P.xcd_remap = tune ? tune->xcd_remap : 1;
    return P;
}

void launch_apply_h(const HamiltonianDev& H, syk_dtype dtype, int nvec, const int32_t* real_of_col,
                    const void* psi, void* out, const ApplyPlan& P, hipStream_t s)
{
    const int M = H.M;
    const Group* groups = H.groups_for(P.tile_bits, true);
    const int n_groups = H.n_groups_for(P.tile_bits, true);
    const FarRec* far = H.far_for(P.tile_bits);
    const int n_far = H.n_far_for(P.tile_bits);
    const KRec* krec = krecs_for(H, P);
    timing_begin(s);
    for (int sl = 0; sl < P.slices; ++sl) {
        KLayout L{};
        L.far = far;
        L.n_far = n_far;
        L.tile_bits = P.tile_bits;
        L.dim = (uint64_t)1 << M;
        L.col0 = sl * kColsPerLaunch;
        L.n_tiles = (uint32_t)(((uint64_t)1 << M) >> P.tile_bits);
        L.xcd_remap = P.xcd_remap;
        const int ncols = std::min(kColsPerLaunch, nvec - L.col0);
        for (int c = 0; c < ncols; ++c) L.real[c] = real_of_col ? real_of_col[L.col0 + c] : 0;
        if (dtype == SYK_C128) {
            KTerms<double> T{H.masks, groups, H.tab4_d, H.qinfo, H.phi2_d, H.w2_d, H.dz, H.dw_d,
                             n_groups, H.n_diag, H.n_real, M};
            launch_t<double>(P, T, krec, L, ncols, psi, out, s);
        } else {
            KTerms<float> T{H.masks, groups, H.tab4_f, H.qinfo, H.phi2_f, H.w2_f, H.dz, H.dw_f,
                            n_groups, H.n_diag, H.n_real, M};
            launch_t<float>(P, T, krec, L, ncols, psi, out, s);
        }
    }
    timing_end(s);
}

}  // namespace syk
