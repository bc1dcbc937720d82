// Matrix-free H psi for the Jordan-Wigner SYK Hamiltonian on gfx950.
//
// (H psi)[r] = sum_x D_x(r) psi[r ^ x] over the flip masks x of terms.hpp.
// A workgroup owns one tile of 2^tile_bits consecutive rows (times up to 64
// interleaved columns of a block).  For a mask, every row of the tile reads
// the tile (tile ^ (x >> tile_bits)) of psi, permuted by x's low bits, so the
// masks are processed group by group: the shared source tile is staged once
// into LDS with coalesced loads and every mask of the group gathers from LDS.
// Each thread keeps its rows' sums in registers and writes them once.
#include "apply_h.hpp"

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

__device__ __forceinline__ int parity(uint32_t v) { return __popc(v) & 1; }

template <typename R, int RPT>
__global__ void __launch_bounds__(256) k_apply_h(KTerms<R> T, KLayout L,
                                                  const cplx<R>* __restrict__ psi,
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
        const uint32_t stile = tile ^ G.x_high;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const uint64_t srow = ((uint64_t)stile << L.tile_bits) | (uint32_t)(lin[k] >> L.log_cw);
            src[lin[k]] = psi[srow * L.ld + L.col0 + col[k]];
        }
        __syncthreads();

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
                    const int idx = (int)(((r >> m.q[0]) & 1u) | (((r >> m.q[1]) & 1u) << 1) |
                                          (((r >> m.q[2]) & 1u) << 2) | (((r >> m.q[3]) & 1u) << 3));
                    const cplx<R> t = T.tab4[((size_t)tab * T.n_real + rc[k]) * 16 + idx];
                    R cr = t.re * v.re - t.im * v.im;
                    R ci = t.re * v.im + t.im * v.re;
                    if (parity(r & m.zbase)) { cr = -cr; ci = -ci; }
                    pr[k] += cr;
                    pi[k] += ci;
                }
            } else if (type == MASK_PAIR) {
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const cplx<R> v = src[lin[k] ^ xl_sh];
                    const uint32_t r = row[k];
                    const R* w = T.w2 + ((size_t)tab * T.n_real + rc[k]) * 4 * (M + 1);
                    R l0 = w[M], l1 = w[(M + 1) + M], l2 = w[2 * (M + 1) + M], l3 = w[3 * (M + 1) + M];
                    for (int c = 0; c < M; ++c) {
                        const R b = (R)((r >> c) & 1u);
                        l0 += w[c] * b;
                        l1 += w[(M + 1) + c] * b;
                        l2 += w[2 * (M + 1) + c] * b;
                        l3 += w[3 * (M + 1) + c] * b;
                    }
                    const int idx = (int)(((r >> m.q[0]) & 1u) | (((r >> m.q[1]) & 1u) << 1));
                    const cplx<R>* ph = T.phi2 + (size_t)tab * 16 + idx * 4;
                    const R dre = ph[0].re * l0 + ph[1].re * l1 + ph[2].re * l2 + ph[3].re * l3;
                    const R dim = ph[0].im * l0 + ph[1].im * l1 + ph[2].im * l2 + ph[3].im * l3;
                    R cr = dre * v.re - dim * v.im;
                    R ci = dre * v.im + dim * v.re;
                    if (parity(r & m.zbase)) { cr = -cr; ci = -ci; }
                    pr[k] += cr;
                    pi[k] += ci;
                }
            } else {  // MASK_DIAG
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const cplx<R> v = src[lin[k] ^ xl_sh];
                    const uint32_t r = row[k];
                    const R* d = T.dw + (size_t)rc[k] * T.n_diag;
                    R s = R(0);
                    for (int n = 0; n < T.n_diag; ++n) s += parity(r & T.dz[n]) ? -d[n] : d[n];
                    pr[k] += s * v.re;
                    pi[k] += s * v.im;
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
void launch_t(const ApplyPlan& P, const KTerms<R>& T, KLayout L, const void* psi, void* out,
              hipStream_t s)
{
    dim3 grid(L.n_tiles), block(P.nt);
    size_t lds = ((size_t)1 << (P.tile_bits + P.log_cw)) * sizeof(cplx<R>);
    auto* in = static_cast<const cplx<R>*>(psi);
    auto* o = static_cast<cplx<R>*>(out);
    switch (P.rpt) {
    case 1: hipLaunchKernelGGL((k_apply_h<R, 1>), grid, block, lds, s, T, L, in, o); break;
    case 2: hipLaunchKernelGGL((k_apply_h<R, 2>), grid, block, lds, s, T, L, in, o); break;
    case 4: hipLaunchKernelGGL((k_apply_h<R, 4>), grid, block, lds, s, T, L, in, o); break;
    case 8: hipLaunchKernelGGL((k_apply_h<R, 8>), grid, block, lds, s, T, L, in, o); break;
    case 16: hipLaunchKernelGGL((k_apply_h<R, 16>), grid, block, lds, s, T, L, in, o); break;
    default: throw Error(SYK_EINVAL, "apply_H: unsupported rows per thread");
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
    const int max_elems_log = (dtype == SYK_C128) ? 11 : 12;   // 32 KiB LDS tile
    int tb = std::min(M, max_elems_log - P.log_cw);
    if (tb < 0) tb = 0;
    // Keep enough workgroups to fill 256 CUs several times over.
    while (tb > 0 && ((int64_t)1 << (M - tb)) * P.slices < 2048 && ((int64_t)1 << (tb + P.log_cw)) > 256) --tb;
    if (tune && tune->tile_bits > 0) tb = std::min(tune->tile_bits, M);
    P.tile_bits = tb;
    const int elems = 1 << (tb + P.log_cw);
    P.nt = std::min(256, elems);
    P.rpt = elems / P.nt;
    if (tune && tune->threads > 0 && elems / tune->threads >= 1 && elems / tune->threads <= 16 &&
        elems % tune->threads == 0) {
        P.nt = tune->threads;
        P.rpt = elems / P.nt;
    }
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
    const size_t eb = elem_bytes(dtype);
    for (int sl = 0; sl < P.slices; ++sl) {
        KLayout L{};
        L.tile_bits = P.tile_bits;
        L.log_cw = P.log_cw;
        L.ld = nvec;
        L.col0 = sl * cw;
        L.n_tiles = (uint32_t)(((uint64_t)1 << M) >> P.tile_bits);
        L.xcd_remap = P.xcd_remap;
        for (int c = 0; c < cw; ++c) L.real[c] = real_of_col ? real_of_col[L.col0 + c] : 0;
        (void)eb;
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
}

}  // namespace syk
