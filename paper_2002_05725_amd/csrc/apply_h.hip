// Matrix-free H psi for the Jordan-Wigner SYK Hamiltonian on gfx950.
//
// (H psi)[r] = sum_x D_x(r) psi[r ^ x] over the flip masks x of terms.hpp.
// A workgroup owns one tile of 2^tile_bits consecutive rows (times up to 64
// interleaved columns of a block).  For a mask, every row of the tile reads
// the tile (tile ^ (x >> tile_bits)) of psi, permuted by x's low bits, so the
// masks are processed chunk by chunk in x order: the shared source tile is
// staged once into LDS with coalesced loads, every mask of the chunk gathers
// from LDS, and each thread keeps its rows' sums in registers and writes them
// once.
//
// Two kernels:
//  * k_apply_single: one column, one realisation.  Mask records, PAIR weights
//    and DIAG terms are wave-uniform (scalar loads); the chunk's QUAD tables are
//    staged into LDS next to the source tile.
//  * k_apply_block: up to 64 interleaved columns, each with its realisation.
#include "apply_h.hpp"
#include "timing.hpp"

namespace syk {

namespace {

template <typename R>
struct KTerms {
    const MaskRec* __restrict__ masks;
    const Group* __restrict__ groups;
    const cplx<R>* __restrict__ tab4;
    const cplx<R>* __restrict__ phi2;
    const R* __restrict__ w2;
    const uint32_t* __restrict__ dz;
    const R* __restrict__ dw;
    int n_groups, n_diag, n_real, M;
};

struct KLayout {
    int tile_bits;     // rows per tile = 2^tile_bits
    int log_cw;        // columns per tile = 2^log_cw
    int64_t ld;        // row stride of psi/out in elements (= nvec)
    int col0;          // first column of this launch
    uint32_t n_tiles;  // dim >> tile_bits
    int xcd_remap;     // spread consecutive tiles over XCDs in contiguous ranges
    int32_t real[64];  // realisation of each column of the slice
};

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

template <typename R, int RPT>
__global__ void __launch_bounds__(256) k_apply_single(KTerms<R> T, KLayout L, const cplx<R>* __restrict__ psi,
                                                       cplx<R>* __restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nt = blockDim.x;
    const int tile_elems = nt * RPT;                   // == 2^tile_bits
    cplx<R>* src = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* tabs = src + tile_elems;                  // kChunkMasks x 16 entries

    const uint32_t tile = tile_of_block(blockIdx.x, L);
    const uint32_t row_mask = (1u << L.tile_bits) - 1u;
    const int rc = L.real[0];
    const int M = T.M;
    const uint32_t base = tile << L.tile_bits;

    double acc_re[RPT], acc_im[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) acc_re[k] = acc_im[k] = 0.0;

    for (int g = 0; g < T.n_groups; ++g) {
        const Group G = T.groups[g];
        __syncthreads();   // previous chunk is done with src / tabs
        if (G.new_tile) {
            const uint64_t sbase = (uint64_t)(tile ^ G.x_high) << L.tile_bits;
#pragma unroll
            for (int k = 0; k < RPT; ++k) src[threadIdx.x + k * nt] = psi[sbase + threadIdx.x + k * nt];
        }
        for (int e = threadIdx.x; e < (int)G.n_quad * 16; e += nt)
            tabs[e] = T.tab4[((size_t)(G.quad_first + (e >> 4)) * T.n_real + rc) * 16 + (e & 15)];
        __syncthreads();

        R pr[RPT], pi[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) pr[k] = pi[k] = R(0);

        for (uint32_t mi = G.first; mi < G.first + G.count; ++mi) {
            const MaskRec m = T.masks[mi];
            const uint32_t xl = m.x & row_mask;
            const uint32_t type = m.type_tab >> 28;
            const uint32_t tab = m.type_tab & 0x0fffffffu;
            if (type == MASK_QUAD) {
                const cplx<R>* tq = tabs + (tab - G.quad_first) * 16;
                const uint32_t q0 = m.q[0], q1 = m.q[1], q2 = m.q[2], q3 = m.q[3];
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const uint32_t rl = threadIdx.x + k * nt;
                    const uint32_t r = base | rl;
                    const cplx<R> v = src[rl ^ xl];
                    const uint32_t idx = bit(r, q0) | (bit(r, q1) << 1) | (bit(r, q2) << 2) | (bit(r, q3) << 3);
                    const cplx<R> t = tq[idx];
                    const uint32_t s = parity(r & m.zbase);
                    const R tr = flip(t.re, s), ti = flip(t.im, s);
                    pr[k] = fma(tr, v.re, pr[k]);
                    pr[k] = fma(-ti, v.im, pr[k]);
                    pi[k] = fma(tr, v.im, pi[k]);
                    pi[k] = fma(ti, v.re, pi[k]);
                }
            } else if (type == MASK_PAIR) {
                // D = (-1)^{|r & zbase|} sum_e phi_e (-1)^{s_q0 e_0 + s_q1 e_1} L_e(r),
                // phi_e = Phi[idx = 3][e] (the entry with s_q0 = s_q1 = 0).
                const R* w = T.w2 + ((size_t)tab * T.n_real + rc) * 4 * (M + 1);
                const cplx<R>* ph = T.phi2 + (size_t)tab * 16 + 12;
                const uint32_t q0 = m.q[0], q1 = m.q[1];
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const uint32_t rl = threadIdx.x + k * nt;
                    const uint32_t r = base | rl;
                    const cplx<R> v = src[rl ^ xl];
                    R l0 = w[M], l1 = w[(M + 1) + M], l2 = w[2 * (M + 1) + M], l3 = w[3 * (M + 1) + M];
                    for (int c = 0; c < M; ++c) {
                        const R b = (R)bit(r, c);
                        l0 = fma(w[c], b, l0);
                        l1 = fma(w[(M + 1) + c], b, l1);
                        l2 = fma(w[2 * (M + 1) + c], b, l2);
                        l3 = fma(w[3 * (M + 1) + c], b, l3);
                    }
                    const uint32_t sa = bit(r, q0) ^ 1u, sb = bit(r, q1) ^ 1u;
                    l1 = flip(l1, sa);
                    l2 = flip(l2, sb);
                    l3 = flip(l3, sa ^ sb);
                    R dre = ph[0].re * l0 + ph[1].re * l1 + ph[2].re * l2 + ph[3].re * l3;
                    R dim = ph[0].im * l0 + ph[1].im * l1 + ph[2].im * l2 + ph[3].im * l3;
                    const uint32_t s = parity(r & m.zbase);
                    dre = flip(dre, s);
                    dim = flip(dim, s);
                    pr[k] = fma(dre, v.re, pr[k]);
                    pr[k] = fma(-dim, v.im, pr[k]);
                    pi[k] = fma(dre, v.im, pi[k]);
                    pi[k] = fma(dim, v.re, pi[k]);
                }
            } else {  // MASK_DIAG
                const R* d = T.dw + (size_t)rc * T.n_diag;
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const uint32_t rl = threadIdx.x + k * nt;
                    const uint32_t r = base | rl;
                    const cplx<R> v = src[rl ^ xl];
                    R s = R(0);
                    for (int n = 0; n < T.n_diag; ++n) s += flip(d[n], parity(r & T.dz[n]));
                    pr[k] = fma(s, v.re, pr[k]);
                    pi[k] = fma(s, v.im, pi[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            acc_re[k] += (double)pr[k];
            acc_im[k] += (double)pi[k];
        }
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        cplx<R> o;
        o.re = (R)acc_re[k];
        o.im = (R)acc_im[k];
        out[(uint64_t)base + threadIdx.x + k * nt] = o;
    }
}

template <typename R, int RPT>
__global__ void __launch_bounds__(256) k_apply_block(KTerms<R> T, KLayout L, const cplx<R>* __restrict__ psi,
                                                      cplx<R>* __restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R>* src = reinterpret_cast<cplx<R>*>(smem_raw);

    const int nt = blockDim.x;
    const int cw_mask = (1 << L.log_cw) - 1;
    const uint32_t tile = tile_of_block(blockIdx.x, L);
    const uint32_t row_mask = (1u << L.tile_bits) - 1u;

    int lin[RPT];
    uint32_t row[RPT];
    int col[RPT];
    int rc[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        lin[k] = threadIdx.x + k * nt;
        col[k] = lin[k] & cw_mask;
        row[k] = (tile << L.tile_bits) | (uint32_t)(lin[k] >> L.log_cw);
        int r = 0;
        for (int c = 0; c <= cw_mask; ++c)
            if (c == col[k]) r = L.real[c];
        rc[k] = r;
    }

    double acc_re[RPT], acc_im[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) acc_re[k] = acc_im[k] = 0.0;

    const int M = T.M;
    for (int g = 0; g < T.n_groups; ++g) {
        const Group G = T.groups[g];
        if (G.new_tile) {
            const uint32_t stile = tile ^ G.x_high;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const uint64_t srow = ((uint64_t)stile << L.tile_bits) | (uint32_t)(lin[k] >> L.log_cw);
                src[lin[k]] = psi[srow * L.ld + L.col0 + col[k]];
            }
            __syncthreads();
        }

        R pr[RPT], pi[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) pr[k] = pi[k] = R(0);

        for (uint32_t mi = G.first; mi < G.first + G.count; ++mi) {
            const MaskRec m = T.masks[mi];
            const int xl_sh = (int)((m.x & row_mask) << L.log_cw);
            const uint32_t type = m.type_tab >> 28;
            const uint32_t tab = m.type_tab & 0x0fffffffu;
            if (type == MASK_QUAD) {
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const cplx<R> v = src[lin[k] ^ xl_sh];
                    const uint32_t r = row[k];
                    const uint32_t idx = bit(r, m.q[0]) | (bit(r, m.q[1]) << 1) | (bit(r, m.q[2]) << 2) |
                                         (bit(r, m.q[3]) << 3);
                    const cplx<R> t = T.tab4[((size_t)tab * T.n_real + rc[k]) * 16 + idx];
                    const uint32_t s = parity(r & m.zbase);
                    const R tr = flip(t.re, s), ti = flip(t.im, s);
                    pr[k] = fma(tr, v.re, pr[k]);
                    pr[k] = fma(-ti, v.im, pr[k]);
                    pi[k] = fma(tr, v.im, pi[k]);
                    pi[k] = fma(ti, v.re, pi[k]);
                }
            } else if (type == MASK_PAIR) {
                const cplx<R>* ph = T.phi2 + (size_t)tab * 16 + 12;
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const cplx<R> v = src[lin[k] ^ xl_sh];
                    const uint32_t r = row[k];
                    const R* w = T.w2 + ((size_t)tab * T.n_real + rc[k]) * 4 * (M + 1);
                    R l0 = w[M], l1 = w[(M + 1) + M], l2 = w[2 * (M + 1) + M], l3 = w[3 * (M + 1) + M];
                    for (int c = 0; c < M; ++c) {
                        const R b = (R)bit(r, c);
                        l0 = fma(w[c], b, l0);
                        l1 = fma(w[(M + 1) + c], b, l1);
                        l2 = fma(w[2 * (M + 1) + c], b, l2);
                        l3 = fma(w[3 * (M + 1) + c], b, l3);
                    }
                    const uint32_t sa = bit(r, m.q[0]) ^ 1u, sb = bit(r, m.q[1]) ^ 1u;
                    l1 = flip(l1, sa);
                    l2 = flip(l2, sb);
                    l3 = flip(l3, sa ^ sb);
                    R dre = ph[0].re * l0 + ph[1].re * l1 + ph[2].re * l2 + ph[3].re * l3;
                    R dim = ph[0].im * l0 + ph[1].im * l1 + ph[2].im * l2 + ph[3].im * l3;
                    const uint32_t s = parity(r & m.zbase);
                    dre = flip(dre, s);
                    dim = flip(dim, s);
                    pr[k] = fma(dre, v.re, pr[k]);
                    pr[k] = fma(-dim, v.im, pr[k]);
                    pi[k] = fma(dre, v.im, pi[k]);
                    pi[k] = fma(dim, v.re, pi[k]);
                }
            } else {  // MASK_DIAG
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const cplx<R> v = src[lin[k] ^ xl_sh];
                    const uint32_t r = row[k];
                    const R* d = T.dw + (size_t)rc[k] * T.n_diag;
                    R s = R(0);
                    for (int n = 0; n < T.n_diag; ++n) s += flip(d[n], parity(r & T.dz[n]));
                    pr[k] = fma(s, v.re, pr[k]);
                    pi[k] = fma(s, v.im, pi[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            acc_re[k] += (double)pr[k];
            acc_im[k] += (double)pi[k];
        }
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        cplx<R> o;
        o.re = (R)acc_re[k];
        o.im = (R)acc_im[k];
        out[(uint64_t)row[k] * L.ld + L.col0 + col[k]] = o;
    }
}

inline int ilog2(int64_t v)
{
    int l = 0;
    while ((int64_t(1) << (l + 1)) <= v) ++l;
    return l;
}

template <typename R>
void launch_t(const ApplyPlan& P, const KTerms<R>& T, KLayout L, const void* psi, void* out, hipStream_t s)
{
    dim3 grid(L.n_tiles), block(P.nt);
    const size_t tile = ((size_t)1 << (P.tile_bits + P.log_cw)) * sizeof(cplx<R>);
    auto* in = static_cast<const cplx<R>*>(psi);
    auto* o = static_cast<cplx<R>*>(out);
    if (P.single) {
        const size_t lds = tile + (size_t)kChunkMasks * 16 * sizeof(cplx<R>);
        switch (P.rpt) {
        case 1: hipLaunchKernelGGL((k_apply_single<R, 1>), grid, block, lds, s, T, L, in, o); break;
        case 2: hipLaunchKernelGGL((k_apply_single<R, 2>), grid, block, lds, s, T, L, in, o); break;
        case 4: hipLaunchKernelGGL((k_apply_single<R, 4>), grid, block, lds, s, T, L, in, o); break;
        case 8: hipLaunchKernelGGL((k_apply_single<R, 8>), grid, block, lds, s, T, L, in, o); break;
        case 16: hipLaunchKernelGGL((k_apply_single<R, 16>), grid, block, lds, s, T, L, in, o); break;
        default: throw Error(SYK_EINVAL, "apply_H: unsupported rows per thread");
        }
    } else {
        switch (P.rpt) {
        case 1: hipLaunchKernelGGL((k_apply_block<R, 1>), grid, block, tile, s, T, L, in, o); break;
        case 2: hipLaunchKernelGGL((k_apply_block<R, 2>), grid, block, tile, s, T, L, in, o); break;
        case 4: hipLaunchKernelGGL((k_apply_block<R, 4>), grid, block, tile, s, T, L, in, o); break;
        case 8: hipLaunchKernelGGL((k_apply_block<R, 8>), grid, block, tile, s, T, L, in, o); break;
        case 16: hipLaunchKernelGGL((k_apply_block<R, 16>), grid, block, tile, s, T, L, in, o); break;
        default: throw Error(SYK_EINVAL, "apply_H: unsupported rows per thread");
        }
    }
    SYK_HIP(hipGetLastError());
}

}  // namespace

ApplyPlan plan_apply(int M, int nvec, syk_dtype dtype, const ApplyTuning* tune)
{
    ApplyPlan P{};
    int cw = 1;
    if (nvec <= 64 && (nvec & (nvec - 1)) == 0) cw = nvec;
    else if (nvec % 64 == 0) cw = 64;
    P.log_cw = ilog2(cw);
    P.slices = nvec / cw;
    P.single = (nvec == 1);
    // LDS source tile of 16 KiB (two or more workgroups per CU).
    const int max_elems_log = (dtype == SYK_C128) ? 10 : 11;
    int tb = std::min(M, max_elems_log - P.log_cw);
    if (tb < 0) tb = 0;
    // Keep enough workgroups to fill 256 CUs several times over.
    while (tb > 0 && ((int64_t)1 << (M - tb)) * P.slices < 2048 && ((int64_t)1 << (tb + P.log_cw)) > 256) --tb;
    int nt_pref = 256;
    if (tune && tune->tile_bits > 0) {
        // at most 64 KiB of LDS per tile
        const int lim = ((dtype == SYK_C128) ? 12 : 13) - P.log_cw;
        tb = std::max(0, std::min(std::min(tune->tile_bits, M), lim));
    }
    if (tune && tune->threads > 0) nt_pref = tune->threads;
    P.tile_bits = tb;
    const int elems = 1 << (tb + P.log_cw);
    P.nt = std::min(nt_pref, elems);
    while (elems / P.nt > 16) P.nt *= 2;
    if (P.nt > 256) P.nt = 256;
    P.rpt = elems / P.nt;
    if (P.rpt > 16 || P.rpt * P.nt != elems) throw Error(SYK_EINVAL, "apply_H: tile does not fit the launch shape");
    P.xcd_remap = tune ? tune->xcd_remap : 1;
    return P;
}

void launch_apply_h(const HamiltonianDev& H, syk_dtype dtype, int nvec, const int32_t* real_of_col,
                    const void* psi, void* out, const ApplyPlan& P, hipStream_t s)
{
    const int M = H.M;
    const Group* groups = H.groups_for(P.tile_bits);
    const int n_groups = H.n_groups_for(P.tile_bits);
    const int cw = 1 << P.log_cw;
    timing_begin(s);
    for (int sl = 0; sl < P.slices; ++sl) {
        KLayout L{};
        L.tile_bits = P.tile_bits;
        L.log_cw = P.log_cw;
        L.ld = nvec;
        L.col0 = sl * cw;
        L.n_tiles = (uint32_t)(((uint64_t)1 << M) >> P.tile_bits);
        L.xcd_remap = P.xcd_remap;
        for (int c = 0; c < cw; ++c) L.real[c] = real_of_col ? real_of_col[L.col0 + c] : 0;
        if (dtype == SYK_C128) {
            KTerms<double> T{H.masks, groups, H.tab4_d, H.phi2_d, H.w2_d, H.dz, H.dw_d,
                             n_groups, H.n_diag, H.n_real, M};
            launch_t<double>(P, T, L, psi, out, s);
        } else {
            KTerms<float> T{H.masks, groups, H.tab4_f, H.phi2_f, H.w2_f, H.dz, H.dw_f,
                            n_groups, H.n_diag, H.n_real, M};
            launch_t<float>(P, T, L, psi, out, s);
        }
    }
    timing_end(s);
}

}  // namespace syk
