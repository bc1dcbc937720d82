// Kernels of the Chebyshev propagator and of the coupling derivatives.
//
// k_cheb_rec: one step of the three-term recurrence T_{n+1} = 2 H~ T_n - T_{n-1}
// (and of its transpose, Clenshaw's recurrence), fused with the running sum.
//
// k_grad_bins: for pairs (g_p, v_p) with weights w_p, accumulates for every flip
// mask the bins of sum_p w_p conj(g_p[r]) (-1)^{|r & zbase|} v_p[r ^ x] that
// determine Re <g_p| Q_n v_p> for each coupling n of the mask (terms.hpp).  A
// workgroup sweeps a fixed set of 512-row tiles for one chunk of masks at a
// time with the chunk's bins in LDS, then writes them to its own slice of a
// partial buffer; k_bins_reduce adds the slices in a fixed order.
//
// The four waves of a workgroup split a chunk's QUAD masks (every fourth of
// its list to each), and a wave computes its masks over all rows of the tile
// (64 lanes x 8 rows).  QUAD bins depend on the row only through its bits at
// the four flipped qubits: the lanes of the wave that agree on those bits are
// summed with DPP row shifts and permlane swaps, and one lane per bin adds it
// to the bin, which no other wave touches.  PAIR and DIAG bins are linear in
// sum_p w_p conj(g_p[r]) v_p[r ^ x], which each thread sums over the pairs for
// its two rows of the tile; the rows are then laid out in LDS and every bin is
// formed by fixed threads in a fixed order.  No float atomics: the bins are the
// same bits on every run.
#include "grad.hpp"

#include <algorithm>
#include <cstring>

#include "mask_classes.hpp"

namespace syk {

namespace {

__device__ __forceinline__ uint32_t parity(uint32_t v) { return __popc(v) & 1u; }
__device__ __forceinline__ uint32_t bit(uint32_t r, uint32_t q) { return (r >> q) & 1u; }
__device__ __forceinline__ double flip(double x, uint32_t s)
{
    return __hiloint2double(__double2hiint(x) ^ (int)(s << 31), __double2loint(x));
}
__device__ __forceinline__ uint32_t quad_index(uint32_t r, uint32_t qpack)
{
    return bit(r, mask_q(qpack, 0)) | (bit(r, mask_q(qpack, 1)) << 1) | (bit(r, mask_q(qpack, 2)) << 2) |
           (bit(r, mask_q(qpack, 3)) << 3);
}

// v plus the value of the partner lane that differs from this lane in in-wave
// lane bit B.  Bits 0..3: a DPP row shift by 2^B, whose partner is this lane
// minus 2^B, so only lanes with bit B set receive the pair's sum.  Bits 4 and
// 5: the gfx950 permlane swaps (rows 2j <-> 2j+1 of 16 lanes; halves of 32
// lanes), which give every lane the sum.  All VALU: no LDS round trip.
template <int B>
__device__ __forceinline__ double add_partner(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    if constexpr (B < 4) {
        constexpr int ctrl = 0x110 + (1 << B);   // row_shr:2^B
        const int plo = __builtin_amdgcn_mov_dpp(lo, ctrl, 0xf, 0xf, true);
        const int phi = __builtin_amdgcn_mov_dpp(hi, ctrl, 0xf, 0xf, true);
        return v + __hiloint2double(phi, plo);
    } else if constexpr (B == 4) {
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
    } else {
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
    }
}

// Sums of a and of b over the lanes of this wave that agree with this lane on
// every in-wave lane bit set in keep (bits 0..5 of the lane index), complete
// in the lane group_rep picks out of each group.  keep must be wave-uniform,
// every lane of the workgroup must call it, and keep must include every lane
// bit at or above the workgroup's own lane bits (the exchanges would read the
// registers of lanes that do not run).
template <int B>
__device__ __forceinline__ void group_stage(double& a, double& b, uint32_t keep)
{
    if (!(keep & (1u << B))) {
        a = add_partner<B>(a);
        b = add_partner<B>(b);
    }
}
__device__ __forceinline__ void group_sum(double& a, double& b, uint32_t keep)
{
    group_stage<0>(a, b, keep);
    group_stage<1>(a, b, keep);
    group_stage<2>(a, b, keep);
    group_stage<3>(a, b, keep);
    group_stage<4>(a, b, keep);
    group_stage<5>(a, b, keep);
}

// The value of the lane that differs from this lane in lane bit B (0 or 1):
// a DPP quad permutation, both ways.
template <int B>
__device__ __forceinline__ double lane_xor(double v)
{
    constexpr int ctrl = B == 0 ? 0xb1 : 0x4e;   // quad_perm:[1,0,3,2] / [2,3,0,1]
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// The lane of a group_sum group that holds the sum: its bits 0..3 outside keep
// are set, its bits 4 and 5 outside keep clear.
__device__ __forceinline__ bool group_rep(uint32_t lane, uint32_t keep)
{
    return ((lane | keep) & 15u) == 15u && (lane & ~keep & 48u) == 0u;
}

// out = b (w - gamma y) + s z + c x ; acc += ca out (acc optional).  Null
// pointers drop their term.  out may alias z or x.
template <typename R>
__global__ void __launch_bounds__(256) k_cheb_rec(cplx<R>* out, const cplx<R>* __restrict__ w,
                                                  const cplx<R>* __restrict__ y, const cplx<R>* z,
                                                  const cplx<R>* x, cplx<R>* acc, double b, double gamma, double s,
                                                  double c_re, double c_im, double ca_re, double ca_im, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double re = 0.0, im = 0.0;
        if (w) {
            const cplx<R> wv = w[e];
            const cplx<R> yv = y[e];
            re = b * ((double)wv.re - gamma * (double)yv.re);
            im = b * ((double)wv.im - gamma * (double)yv.im);
        }
        if (z) {
            const cplx<R> zv = z[e];
            re += s * (double)zv.re;
            im += s * (double)zv.im;
        }
        if (x) {
            const cplx<R> xv = x[e];
            re += c_re * (double)xv.re - c_im * (double)xv.im;
            im += c_re * (double)xv.im + c_im * (double)xv.re;
        }
        cplx<R> o;
        o.re = (R)re;
        o.im = (R)im;
        out[e] = o;
        if (acc) {
            const cplx<R> a = acc[e];
            cplx<R> r;
            r.re = (R)((double)a.re + ca_re * re - ca_im * im);
            r.im = (R)((double)a.im + ca_re * im + ca_im * re);
            acc[e] = r;
        }
    }
}

struct GLayout {
    int tile_bits;                        // rows per tile = 2^tile_bits
    int lane_bits;                        // in-wave lane bits that index rows (6, fewer for tiny states)
    uint32_t n_tiles;
    uint32_t tile_groups, chunk_groups;   // grid = tile_groups x chunk_groups workgroups
    int n_chunks;
    int npairs;
    int M;
    int n_diag;
    uint64_t n_bins;
};

// Bins of one launch: four waves of 64 lanes; lane l owns rows l + 64 k
// (k < 2^KB) of every tile of 2^(lane_bits + KB) rows.  Each QUAD member of a
// chunk belongs to one wave (every fourth member of the chunk's class-sorted
// list), which computes it over all rows of the tile: its bins are only ever
// added to by that wave, one lane per bin and instruction, in program order.
// PAIR and DIAG masks sum sum_p w_p conj(g_p[r]) v_p[r ^ x] per row over the
// pairs (each row owned by one thread); at the end of a tile the rows are laid
// out in LDS and every bin is formed by fixed threads in a fixed row order.
// Nothing depends on timing, so the bins are the same bits on every run.
template <int KB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_grad_bins(const KRec* __restrict__ krec, const GChunk* __restrict__ chunks,
                                                    const uint32_t* __restrict__ members,
                                                    const uint32_t* __restrict__ local,
                                                    const GRec* __restrict__ grec,
                                                    const uint32_t* __restrict__ dz, GLayout L,
                                                    const c128* const* __restrict__ gs_nat,
                                                    const c128* const* __restrict__ vs_nat,
                                                    const c128* const* __restrict__ gs_rot,
                                                    const c128* const* __restrict__ vs_rot,
                                                    const double* __restrict__ wts, double* __restrict__ partial)
{
    constexpr int RPT = 1 << KB;
    constexpr int PP = kGradPairsPerStage;
    constexpr int TS = kGradTileRows;                        // LDS rows per staged pair (the largest tile)
    constexpr int SS = PP * TS;                              // one staged source tile of PP pairs
    constexpr int SR = kGradSrcTiles * PP > kGradAccMasks ? kGradSrcTiles * PP : kGradAccMasks;
    __shared__ __align__(16) c128 src[SR * TS];           // [slot][pair][row] source rows; PAIR / DIAG row sums
                                                           // at tile end
    __shared__ __align__(16) double bins[2 * kGradBinCap];
    __shared__ uint32_t fold[kChunkMasks + 4];
    __shared__ __align__(16) double part[2 * 4 * kGradPairOutputs];   // PAIR outputs of four row quarters

    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    // the same for every lane of the wave: member positions and records stay scalar
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t tile_rows = 1u << L.tile_bits;
    const bool live = lane < (1u << L.lane_bits);          // lanes above a tiny state own no rows
    // bits 0..3 and 4..5 of the lane, one per byte (table-index gather)
    uint32_t B0 = 0, B1 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        B0 |= ((lane >> i) & 1u) << (8 * i);
        B1 |= ((lane >> (4 + i)) & 1u) << (8 * i);
    }
    // workgroup (t, s) of the grid: tiles t, t + tile_groups, ...; chunks s, s + chunk_groups, ...
    const uint32_t tg = blockIdx.x % L.tile_groups, sg = blockIdx.x / L.tile_groups;
    double* mine = partial + (uint64_t)tg * L.n_bins * 2;

    for (int ch = (int)sg; ch < L.n_chunks; ch += (int)L.chunk_groups) {
        const GChunk C = chunks[ch];
        // the pair vectors in the chunk's row layout
        const c128* const* __restrict__ gs = C.layout ? gs_rot : gs_nat;
        const c128* const* __restrict__ vs = C.layout ? vs_rot : vs_nat;
        for (uint32_t e = tid; e < 2 * C.bin_count; e += 256) bins[e] = 0.0;
        __syncthreads();   // every bin is zero before any wave adds into it
        for (uint32_t tile = tg; tile < L.n_tiles; tile += L.tile_groups) {
            const uint32_t base = tile << L.tile_bits;
            if (!C.far) {
                // tile part of each QUAD member's bin index and sign
                __syncthreads();   // the previous tile's readers of fold are done
                for (uint32_t j = tid; j < C.n_quad; j += 256) {
                    const KRec m = krec[members[C.first + j]];
                    fold[j] = quad_index(base, m.qpack) | (parity(base & m.zbase) << 4);
                }
            }
            // PAIR / DIAG: sum_p w_p conj(g_p[r]) v_p[r ^ x] on the rows tid and tid + 256 of the tile
            double acc_re[kGradAccMasks][2], acc_im[kGradAccMasks][2];
#pragma unroll
            for (int j = 0; j < kGradAccMasks; ++j)
#pragma unroll
                for (int h = 0; h < 2; ++h) acc_re[j][h] = acc_im[j][h] = 0.0;

            // PP pairs at a time (the host pads the list with zero-weight pairs)
            for (int p0 = 0; p0 < L.npairs; p0 += PP) {
                c128 gk[PP][RPT];   // w_p g_p on the lane's rows (every wave loads all rows)
#pragma unroll
                for (int u = 0; u < PP; ++u) {
                    const c128* __restrict__ g = gs[p0 + u] + (base + lane);
                    const double wt = wts[p0 + u];
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        c128 x{0.0, 0.0};
                        if (live) x = g[64 * k];
                        gk[u][k].re = x.re * wt;
                        gk[u][k].im = x.im * wt;
                    }
                }
                if (!C.far) {
                    // the chunk's source tiles; rows past a tiny state are zeros
                    __syncthreads();   // previous users of src are done
#pragma unroll
                    for (int sl = 0; sl < kGradSrcTiles; ++sl) {
                        if (sl >= (int)C.n_src) break;
                        const uint64_t sbase = (uint64_t)(tile ^ (sl ? C.x_high2 : C.x_high)) << L.tile_bits;
#pragma unroll
                        for (int u = 0; u < PP; ++u) {
                            const c128* __restrict__ v = vs[p0 + u] + sbase;
#pragma unroll
                            for (int h = 0; h < TS / 256; ++h) {
                                const uint32_t e = tid + 256u * h;
                                c128& d = src[sl * SS + u * TS + e];
                                if (e < tile_rows) {
                                    d = v[e];
                                } else {
                                    d.re = 0.0;
                                    d.im = 0.0;
                                }
                            }
                        }
                    }
                    __syncthreads();
                }

                if (C.far) {
                    // far QUAD masks (no row bit of the tile flipped or in the sign): one bin
                    // per tile; every fourth member of the chunk to this wave
                    for (uint32_t j = C.first + wave; j < C.first + C.count; j += 4) {
                        const KRec m = krec[members[j]];
                        if ((m.meta >> 28) != MASK_QUAD) continue;
                        const uint64_t sb = (uint64_t)(tile ^ m.x_high) << L.tile_bits;
                        double ar = 0.0, ai = 0.0;
#pragma unroll
                        for (int u = 0; u < PP; ++u) {
                            const c128* __restrict__ v = vs[p0 + u];
#pragma unroll
                            for (int k = 0; k < RPT; ++k) {
                                c128 x{0.0, 0.0};
                                if (live) x = v[sb + lane + 64u * k];
                                ar = fma(gk[u][k].re, x.re, ar);
                                ar = fma(gk[u][k].im, x.im, ar);
                                ai = fma(gk[u][k].re, x.im, ai);
                                ai = fma(-gk[u][k].im, x.re, ai);
                            }
                        }
                        const uint32_t s = parity(base & m.zbase);
                        ar = flip(ar, s);
                        ai = flip(ai, s);
                        group_sum(ar, ai, 0u);
                        if (group_rep(lane, 0u)) {
                            double* mb = bins + 2 * (local[j] + quad_index(base, m.qpack));
                            mb[0] += ar;
                            mb[1] += ai;
                        }
                    }
                } else {
                    // near QUAD members, class by class: positions wave, wave + 4, ... of the
                    // class-sorted list (the next one's record and fold loaded ahead; both
                    // lists run four past the end)
                    uint32_t pos = wave, cls_end = 0;
                    GRec qn = grec[C.first + pos];
                    uint32_t fon = fold[pos];
                    auto class_loop = [&](auto cls) {
                        constexpr int CL = decltype(cls)::value;
                        constexpr uint32_t XK = (uint32_t)class_bits(CL, KB, 1);   // k bits the masks flip
                        constexpr uint32_t ZK = (uint32_t)class_bits(CL, KB, 2);   // k bits in their Z string
                        cls_end += (C.cnt[CL >> 2] >> (8 * (CL & 3))) & 0xffu;
                        for (; pos < cls_end; pos += 4) {
                            const GRec q = qn;
                            const uint32_t slot = pos;
                            const uint32_t fo = fon;
                            qn = grec[C.first + pos + 4];
                            fon = fold[pos + 4];
                            const uint32_t il = __builtin_amdgcn_udot4(__builtin_amdgcn_perm(B1, B0, q.sel), 0x08040201u,
                                                                       fo & 15u, false);
                            const uint32_t sl = (((uint32_t)__popc(lane & q.zl) ^ (fo >> 4)) & 1u) << 31;
                            const uint32_t keep = (q.koffs >> 24) & 63u;
                            double er[RPT], ei[RPT];   // by the flipped k bits p = k & XK
#pragma unroll
                            for (int pp = 0; pp < RPT; ++pp) er[pp] = ei[pp] = 0.0;
                            // lane part of the source row, in the member's staged tile
                            const uint32_t sb = (lane ^ q.xoff) + ((q.koffs >> 30) & 1u) * SS;
                            // source rows of row k (both pairs), read kAhead rows before their FMAs
                            constexpr int kAhead = 2;
                            c128 xs[kAhead + 1][PP];
                            auto read_row = [&](int k, c128 (&x)[PP]) {
#pragma unroll
                                for (int u = 0; u < PP; ++u) x[u] = src[u * TS + sb + (((uint32_t)k ^ XK) << 6)];
                            };
#pragma unroll
                            for (int k = 0; k < kAhead && k < RPT; ++k) read_row(k, xs[k]);
#pragma unroll
                            for (int k = 0; k < RPT; ++k) {
                                if (k + kAhead < RPT) read_row(k + kAhead, xs[(k + kAhead) % (kAhead + 1)]);
                                __builtin_amdgcn_sched_barrier(0);
                                // += (sign of row k) conj(w g) x, straight into the entry's sums
                                const bool neg = (__builtin_popcount((uint32_t)k & ZK) & 1) != 0;
                                double& a = er[k & (int)XK];
                                double& b = ei[k & (int)XK];
#pragma unroll
                                for (int u = 0; u < PP; ++u) {
                                    const c128 x = xs[k % (kAhead + 1)][u];
                                    const double gr = neg ? -gk[u][k].re : gk[u][k].re;
                                    const double gi = neg ? -gk[u][k].im : gk[u][k].im;
                                    a = fma(gr, x.re, a);
                                    a = fma(gi, x.im, a);
                                    b = fma(gr, x.im, b);
                                    b = fma(-gi, x.re, b);
                                }
                                __builtin_amdgcn_sched_barrier(0);
                            }
                            // entry pp (a subset of XK) goes to bin il + the index bits its k bits set
                            auto entry_idx = [&](int pp) {
                                uint32_t idx = il;
#pragma unroll
                                for (int b = 0; b < KB; ++b)
                                    if ((pp >> b) & 1) idx += (q.koffs >> (8 * b)) & 0xffu;
                                return idx;
                            };
                            // this wave is the only one that adds into the member's bins
                            auto bin_add = [&](uint32_t idx, double ar, double ai) {
                                double* mb = bins + 2 * (16 * slot + idx);
                                mb[0] += ar;
                                mb[1] += ai;
                            };
                            // Several entries and in-wave lane bit 0 or 1 outside keep:
                            // one exchange over that bit first (lanes with the bit clear
                            // keep the entries without XK's lowest bit, their partners
                            // those with it), so the remaining sums run on half as many
                            // values per lane.
                            constexpr int T0 = (int)(XK & (0u - XK));   // lowest bit of XK (0: one entry)
                            auto split_sums = [&](auto bc) {
                                constexpr int B = decltype(bc)::value;
                                const uint32_t side = (lane >> B) & 1u;
                                const uint32_t keep2 = keep | (1u << B);
                                const bool rep2 = group_rep(lane, keep2);
#pragma unroll
                                for (int pp = 0; pp < RPT; ++pp) {
                                    if ((pp & ~(int)XK) != 0 || (pp & T0) != 0) continue;
                                    const double a0 = flip31(er[pp], sl), b0 = flip31(ei[pp], sl);
                                    const double a1 = flip31(er[pp | T0], sl), b1 = flip31(ei[pp | T0], sl);
                                    double ar = side ? a1 : a0, ai = side ? b1 : b0;
                                    ar += lane_xor<B>(side ? a0 : a1);
                                    ai += lane_xor<B>(side ? b0 : b1);
                                    group_sum(ar, ai, keep2);
                                    if (rep2) bin_add(side ? entry_idx(pp | T0) : entry_idx(pp), ar, ai);
                                }
                            };
                            if (T0 != 0 && (keep & 1u) == 0u) {
                                split_sums(std::integral_constant<int, 0>{});
                            } else if (T0 != 0 && (keep & 2u) == 0u) {
                                split_sums(std::integral_constant<int, 1>{});
                            } else {
                                const bool rep = group_rep(lane, keep);   // one lane per bin
#pragma unroll
                                for (int pp = 0; pp < RPT; ++pp) {
                                    if ((pp & ~(int)XK) != 0) continue;
                                    double ar = flip31(er[pp], sl), ai = flip31(ei[pp], sl);
                                    group_sum(ar, ai, keep);
                                    if (rep) bin_add(entry_idx(pp), ar, ai);
                                }
                            }
                        }
                    };
                    for_each_class(class_loop, std::make_integer_sequence<int, ipow3(KB)>{});
                }
                // PAIR / DIAG rows of this thread, tid and tid + 256 of the tile: the
                // lane's rows k = wave and wave + 4 (w_p g_p already in gk)
#pragma unroll
                for (int j = 0; j < kGradAccMasks; ++j) {
                    if (j >= (int)C.n_acc) break;
                    const KRec ma = krec[members[C.first + C.acc[j]]];
                    const uint32_t slot_off = ((grec[C.first + C.acc[j]].koffs >> 30) & 1u) * SS;
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        if ((uint32_t)(k & 3) != wave || !live) continue;
                        const uint32_t rl = lane + 64u * (uint32_t)k;
                        double& ar = acc_re[j][k >> 2];
                        double& ai = acc_im[j][k >> 2];
#pragma unroll
                        for (int u = 0; u < PP; ++u) {
                            const c128 x = C.far ? vs[p0 + u][((uint64_t)(tile ^ ma.x_high) << L.tile_bits) + rl]
                                                 : src[slot_off + u * TS + (rl ^ ma.xl)];
                            ar = fma(gk[u][k].re, x.re, fma(gk[u][k].im, x.im, ar));
                            ai = fma(gk[u][k].re, x.im, fma(-gk[u][k].im, x.re, ai));
                        }
                    }
                }
            }

            // bins of the PAIR / DIAG masks from this tile's row sums
            if (C.n_acc > 0) {
                __syncthreads();   // every wave is done with src
                c128* rows = src;   // [kGradAccMasks][TS]
#pragma unroll
                for (int j = 0; j < kGradAccMasks; ++j) {
                    if (j >= (int)C.n_acc) break;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint32_t rl = tid + 256u * h;
                        if (rl < tile_rows) rows[j * TS + rl] = c128{acc_re[j][h], acc_im[j][h]};
                    }
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < kGradAccMasks; ++j) {
                    if (j >= (int)C.n_acc) break;
                    const KRec m = krec[members[C.first + C.acc[j]]];
                    double* mb = bins + 2 * local[C.first + C.acc[j]];
                    const c128* rj = rows + j * TS;
                    if ((m.meta >> 28) == MASK_PAIR) {
                        // output o: rows with bits idx = o & 3 at (q0, q1), and for o >= 4 also
                        // bit c = (o >> 2) - 1 of the tile row set; four threads per output sum
                        // a quarter of the rows each, then one thread adds the quarters in order
                        const uint32_t q0 = mask_q(m.qpack, 0), q1 = mask_q(m.qpack, 1);
                        const uint32_t nout = 4u * (uint32_t)(L.tile_bits + 1);
                        if (tid < 4 * nout) {
                            const uint32_t o = tid >> 2, qtr = tid & 3u, idx = o & 3u;
                            const int c = (int)(o >> 2) - 1;
                            const uint32_t n4 = tile_rows >> 2;
                            double sr = 0.0, si = 0.0;
                            for (uint32_t rl = qtr * n4; rl < (qtr + 1) * n4; ++rl) {
                                const uint32_t r = base | rl;
                                if ((bit(r, q0) | (bit(r, q1) << 1)) != idx) continue;
                                if (c >= 0 && !bit(rl, (uint32_t)c)) continue;
                                const c128 v = rj[rl];
                                const uint32_t s = parity(r & m.zbase);
                                sr += flip(v.re, s);
                                si += flip(v.im, s);
                            }
                            part[2 * tid] = sr;
                            part[2 * tid + 1] = si;
                        }
                        __syncthreads();
                        if (tid < nout) {
                            const uint32_t o = tid, idx = o & 3u;
                            const int c = (int)(o >> 2) - 1;
                            double sr = 0.0, si = 0.0;
#pragma unroll
                            for (int qtr = 0; qtr < 4; ++qtr) {
                                sr += part[2 * (4 * o + qtr)];
                                si += part[2 * (4 * o + qtr) + 1];
                            }
                            if (c >= 0) {
                                mb[2 * (4 + 4 * c + idx)] += sr;
                                mb[2 * (4 + 4 * c + idx) + 1] += si;
                            } else {
                                mb[2 * idx] += sr;
                                mb[2 * idx + 1] += si;
                                // tile bits of the row: the same for every row of the tile
                                for (int cq = L.tile_bits; cq < L.M; ++cq)
                                    if (bit(base, (uint32_t)cq)) {
                                        mb[2 * (4 + 4 * cq + idx)] += sr;
                                        mb[2 * (4 + 4 * cq + idx) + 1] += si;
                                    }
                            }
                        }
                        __syncthreads();   // part is free for the next mask
                    } else {   // MASK_DIAG: one thread per diagonal term, all rows in order
                        for (int n = (int)tid; n < L.n_diag; n += 256) {
                            double sr = 0.0, si = 0.0;
                            for (uint32_t rl = 0; rl < tile_rows; ++rl) {
                                const c128 v = rj[rl];
                                const uint32_t s = parity((base | rl) & dz[n]);
                                sr += flip(v.re, s);
                                si += flip(v.im, s);
                            }
                            mb[2 * n] += sr;
                            mb[2 * n + 1] += si;
                        }
                    }
                }
            }
        }
        __syncthreads();
        // each member's bins to their place in this workgroup's slice
        for (uint32_t j = C.first; j < C.first + C.count; ++j) {
            const uint32_t lo = local[j];
            const uint32_t hi = (j + 1 < C.first + C.count) ? local[j + 1] : C.bin_count;
            const uint64_t go = krec[members[j]].bin0;
            for (uint32_t e = tid; e < 2 * (hi - lo); e += 256) mine[2 * go + e] = bins[2 * lo + e];
        }
        __syncthreads();
    }
}

// out[i] += sum_b partial[b][i] for i < n (in block order b = 0, 1, ...).
__global__ void k_bins_reduce(const double* __restrict__ partial, int nblk, uint64_t n, double* __restrict__ out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(uint64_t)b * n + i];
    out[i] += s;
}

}  // namespace

GradChunks make_grad_chunks(const std::vector<MaskRec>& masks, const std::vector<uint8_t>& layout_of,
                            const std::vector<uint64_t>& bin_off, uint64_t n_bins, int tile_bits, int lane_bits)
{
    const uint32_t row_mask = (1u << tile_bits) - 1u;
    const uint32_t lane_mask = (1u << lane_bits) - 1u;
    const int kb = tile_bits - lane_bits;
    if (kb < 0 || kb > kMaxKBits || lane_bits > 8) throw Error(SYK_EINVAL, "gradient: unsupported launch shape");
    auto nbins = [&](uint32_t i) { return ((i + 1 < masks.size()) ? bin_off[i + 1] : n_bins) - bin_off[i]; };
    struct Build {
        GChunk c;
        std::vector<uint32_t> mem;
    };
    std::vector<Build> near, far;
    // each layout's masks in x order (consecutive masks of a chunk share x >> tile_bits)
    std::vector<uint32_t> order(masks.size());
    for (uint32_t i = 0; i < (uint32_t)masks.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return layout_of[a] != layout_of[b] ? layout_of[a] < layout_of[b] : masks[a].x < masks[b].x;
    });
    for (const uint32_t i : order) {
        const uint32_t type = masks[i].type_tab >> 28;
        const uint32_t xh = masks[i].x >> tile_bits;
        const uint64_t nb = nbins(i);
        if (nb > (uint64_t)kGradBinCap) throw Error(SYK_EUNSUPPORTED, "gradient: mask with too many bins");
        const bool accm = type != MASK_QUAD;
        const bool is_far = type != MASK_DIAG && (masks[i].x & row_mask) == 0u;
        std::vector<Build>& out = is_far ? far : near;
        // a near chunk takes a second source tile when its first group of masks ends
        bool same = !out.empty() && out.back().c.layout == layout_of[i];
        if (same && !is_far) {
            const GChunk& c = out.back().c;
            same = c.x_high == xh || (c.n_src == 2 && c.x_high2 == xh) || c.n_src < (uint32_t)kGradSrcTiles;
        }
        if (!same || out.back().c.count == (uint32_t)kChunkMasks ||
            out.back().c.bin_count + nb > (uint64_t)kGradBinCap ||
            (accm && out.back().c.n_acc == (uint32_t)kGradAccMasks)) {
            Build b{};
            b.c.x_high = is_far ? 0u : xh;
            b.c.n_src = is_far ? 0u : 1u;
            b.c.far = is_far ? 1u : 0u;
            b.c.layout = layout_of[i];
            out.push_back(b);
        }
        Build& b = out.back();
        if (!is_far && b.c.x_high != xh && (b.c.n_src < 2 || b.c.x_high2 != xh)) {
            b.c.x_high2 = xh;
            b.c.n_src = 2;
        }
        if (accm) ++b.c.n_acc;
        b.mem.push_back(i);
        ++b.c.count;
        b.c.bin_count += (uint32_t)nb;
    }
    near.insert(near.end(), far.begin(), far.end());
    GradChunks g;
    for (Build& b : near) {
        // near chunks: QUAD members by class, then PAIR / DIAG; far chunks keep mask order
        auto key = [&](uint32_t i) {
            const MaskRec& m = masks[i];
            if ((m.type_tab >> 28) != MASK_QUAD) return 1000;
            return b.c.far ? 0 : quad_class(m.x, m.zbase, lane_bits, kb);
        };
        std::stable_sort(b.mem.begin(), b.mem.end(), [&](uint32_t x, uint32_t y) { return key(x) < key(y); });
        b.c.first = (uint32_t)g.members.size();
        b.c.n_acc = 0;
        uint32_t lo = 0;
        for (uint32_t pos = 0; pos < b.mem.size(); ++pos) {
            const uint32_t i = b.mem[pos];
            const MaskRec& m = masks[i];
            GRec r{};
            // which of the chunk's staged source tiles the member reads
            if (!b.c.far && (m.x >> tile_bits) != b.c.x_high) r.koffs |= 1u << 30;
            if ((m.type_tab >> 28) == MASK_QUAD) {
                ++b.c.n_quad;
                if (!b.c.far) {
                    const int cls = quad_class(m.x, m.zbase, lane_bits, kb);
                    b.c.cnt[cls >> 2] += 1u << (8 * (cls & 3));
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t qb = mask_q(m.qpack, q);
                        r.sel |= (qb < (uint32_t)lane_bits ? qb : 0x0cu) << (8 * q);
                        const int kbit = (int)qb - lane_bits;
                        if (kbit >= 0 && kbit < kb) r.koffs |= (1u << q) << (8 * kbit);
                    }
                    r.zl = m.zbase & lane_mask;
                    r.xoff = m.x & lane_mask;
                    r.koffs |= (m.x & 63u) << 24;
                }
            } else {
                b.c.acc[b.c.n_acc++] = pos;
            }
            g.members.push_back(i);
            g.local.push_back(lo);
            g.grec.push_back(r);
            lo += (uint32_t)nbins(i);
        }
        g.chunks.push_back(b.c);
    }
    // records past the end: a wave loads its next member's record four positions ahead
    for (int k = 0; k < kGradRecPad; ++k) g.grec.push_back(GRec{});
    return g;
}

void cheb_rec(syk_dtype dtype, int64_t n, void* out, const void* w, const void* y, const void* z, const void* x,
              void* acc, double b, double gamma, double s, std::complex<double> c, std::complex<double> ca,
              hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    if (dtype == SYK_C128)
        hipLaunchKernelGGL(k_cheb_rec<double>, dim3((unsigned)blocks), dim3(256), 0, st, (c128*)out, (const c128*)w,
                           (const c128*)y, (const c128*)z, (const c128*)x, (c128*)acc, b, gamma, s, c.real(), c.imag(),
                           ca.real(), ca.imag(), n);
    else
        hipLaunchKernelGGL(k_cheb_rec<float>, dim3((unsigned)blocks), dim3(256), 0, st, (c64*)out, (const c64*)w,
                           (const c64*)y, (const c64*)z, (const c64*)x, (c64*)acc, b, gamma, s, c.real(), c.imag(),
                           ca.real(), ca.imag(), n);
    SYK_HIP(hipGetLastError());
}

void grad_bins(syk_terms_s& h, const std::vector<const void*>& g, const std::vector<const void*>& v,
               const std::vector<double>& w, double* bins_dev, hipStream_t st)
{
    const HamiltonianDev& H = h.H;
    const TermTables& T = h.host;
    const int npairs = (int)g.size();
    if (npairs == 0) return;
    require(npairs <= kGradMaxPairs && (int)v.size() == npairs && (int)w.size() == npairs, "gradient: bad pair list");
    // tiles of 512 rows (64 lanes x 8 rows per wave), fewer for small states
    const int M = H.M;
    const int tb = std::min(kGradTileBits, M);
    const int lb = std::min(tb, 6);
    const int kb = tb - lb;
    // QUAD masks whose four qubits lie above the tile would each stream a whole
    // tile; with at least C(7,4) of them, run those that sit better in the
    // bit-rotated row layout there (as apply_H does)
    const bool two = M - tb >= 7 && tb >= 8;
    // mask records, chunk records, member list, LDS bin offsets and QUAD member
    // records in one device buffer
    const int key = tb * 2 + (two ? 1 : 0);
    auto it = h.grad_chunks.find(key);
    if (it == h.grad_chunks.end()) {
        std::vector<MaskRec> lm(T.masks);
        std::vector<uint8_t> lay(T.masks.size(), 0);
        if (two)
            for (size_t i = 0; i < lm.size(); ++i)
                if (quad_in_rotated(T.masks[i], M, tb)) {
                    lm[i] = rotate_mask(T.masks[i], M, tb);
                    lay[i] = 1;
                }
        const std::vector<KRec> kr = build_krecs(lm, T.bin_off, tb);
        const GradChunks c = make_grad_chunks(lm, lay, T.bin_off, T.n_bins, tb, lb);
        const size_t kbytes = kr.size() * sizeof(KRec), cb = c.chunks.size() * sizeof(GChunk);
        const size_t gb = c.grec.size() * sizeof(GRec), mb = c.members.size() * sizeof(uint32_t);
        std::unique_ptr<DevBuf> b(new DevBuf());
        b->ensure(kbytes + cb + gb + 2 * mb);
        char* d = static_cast<char*>(b->p);
        SYK_HIP(hipMemcpy(d, kr.data(), kbytes, hipMemcpyHostToDevice));
        SYK_HIP(hipMemcpy(d + kbytes, c.chunks.data(), cb, hipMemcpyHostToDevice));
        SYK_HIP(hipMemcpy(d + kbytes + cb, c.grec.data(), gb, hipMemcpyHostToDevice));
        SYK_HIP(hipMemcpy(d + kbytes + cb + gb, c.members.data(), mb, hipMemcpyHostToDevice));
        SYK_HIP(hipMemcpy(d + kbytes + cb + gb + mb, c.local.data(), mb, hipMemcpyHostToDevice));
        h.grad_nchunks[key] = (int)c.chunks.size();
        h.grad_nmembers[key] = (int)c.members.size();
        it = h.grad_chunks.emplace(key, std::move(b)).first;
    }
    GLayout L{};
    L.tile_bits = tb;
    L.lane_bits = lb;
    L.n_tiles = (uint32_t)(((uint64_t)1 << M) >> tb);
    L.n_chunks = h.grad_nchunks[key];
    L.M = M;
    L.n_diag = H.n_diag;
    L.n_bins = T.n_bins;
    // tile groups own the partial slices; chunk groups split each tile's
    // chunks.  About 12,288 workgroups: with three resident per CU, many
    // short ones balance the uneven cost of chunks and leave no part-full last
    // round (N=44, 32 pairs: 555 ms with 2,048, 530 ms with 3,072, 522 ms).
    const int nblk = (int)std::min<uint32_t>(L.n_tiles, 512u);
    L.tile_groups = (uint32_t)nblk;
    L.chunk_groups = (uint32_t)std::max(1, std::min(L.n_chunks, 12288 / nblk));

    // rotated copies of the pair vectors for the masks of the second layout
    const uint64_t dim = (uint64_t)1 << M;
    std::vector<const void*> gr(npairs), vr(npairs);
    for (int p = 0; p < npairs; ++p) {
        gr[p] = g[p];
        vr[p] = v[p];
        if (!two) continue;
        void* a = h.ws.get("grad_rot_g" + std::to_string(p), dim * sizeof(c128));
        void* b = h.ws.get("grad_rot_v" + std::to_string(p), dim * sizeof(c128));
        launch_transpose(SYK_C128, g[p], a, M - tb, tb, 1, dim, false, st);
        launch_transpose(SYK_C128, v[p], b, M - tb, tb, 1, dim, false, st);
        gr[p] = a;
        vr[p] = b;
    }

    // pointer lists and weights: one small synchronous upload.  The list is
    // padded to a multiple of kGradPairsPerStage with copies of pair 0 of
    // weight 0 (their products are exact zeros).
    const int np = (npairs + kGradPairsPerStage - 1) / kGradPairsPerStage * kGradPairsPerStage;
    L.npairs = np;
    std::vector<uint64_t> host(5 * (size_t)np);
    for (int p = 0; p < np; ++p) {
        const int q = p < npairs ? p : 0;
        host[p] = (uint64_t)(uintptr_t)g[q];
        host[np + p] = (uint64_t)(uintptr_t)v[q];
        host[2 * np + p] = (uint64_t)(uintptr_t)gr[q];
        host[3 * np + p] = (uint64_t)(uintptr_t)vr[q];
        double wp = p < npairs ? w[p] : 0.0;
        std::memcpy(&host[4 * np + p], &wp, sizeof(double));
    }
    void* dlist = h.ws.get("grad_lists", host.size() * sizeof(uint64_t));
    SYK_HIP(hipMemcpyAsync(dlist, host.data(), host.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    SYK_HIP(hipStreamSynchronize(st));
    const c128* const* gl = (const c128* const*)dlist;
    const c128* const* vl = gl + np;
    const c128* const* glr = gl + 2 * np;
    const c128* const* vlr = gl + 3 * np;
    const double* wl = (const double*)(gl + 4 * np);

    double* partial = (double*)h.ws.get("grad_partial", (size_t)nblk * T.n_bins * 2 * sizeof(double));
    const KRec* krec = it->second->as<KRec>();
    const GChunk* chunks = reinterpret_cast<const GChunk*>(krec + T.masks.size());
    const GRec* grec = reinterpret_cast<const GRec*>(chunks + L.n_chunks);
    const uint32_t* members = reinterpret_cast<const uint32_t*>(grec + h.grad_nmembers[key] + kGradRecPad);
    const uint32_t* local = members + h.grad_nmembers[key];
    const dim3 grid(nblk * L.chunk_groups), block(256);
    switch (kb) {
    case 0: hipLaunchKernelGGL(k_grad_bins<0>, grid, block, 0, st, krec, chunks, members, local, grec, H.dz, L, gl, vl, glr, vlr, wl, partial); break;
    case 1: hipLaunchKernelGGL(k_grad_bins<1>, grid, block, 0, st, krec, chunks, members, local, grec, H.dz, L, gl, vl, glr, vlr, wl, partial); break;
    case 2: hipLaunchKernelGGL(k_grad_bins<2>, grid, block, 0, st, krec, chunks, members, local, grec, H.dz, L, gl, vl, glr, vlr, wl, partial); break;
    case 3: hipLaunchKernelGGL(k_grad_bins<3>, grid, block, 0, st, krec, chunks, members, local, grec, H.dz, L, gl, vl, glr, vlr, wl, partial); break;
    default: throw Error(SYK_EUNSUPPORTED, "gradient: launch shape");
    }
    SYK_HIP(hipGetLastError());
    const uint64_t n = 2 * T.n_bins;
    hipLaunchKernelGGL(k_bins_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, partial, nblk, n, bins_dev);
    SYK_HIP(hipGetLastError());
}

}  // namespace syk
