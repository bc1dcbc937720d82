// Host-side check of the derivative-bin kernel's tables (no GPU).
//
// Builds the gradient chunk tables with the library's host code
// (make_grad_chunks, build_krecs, the launch shape and row layouts the
// gradient uses) and evaluates the bins from them the way k_grad_bins reads
// them: the waves' shares of a near chunk's class-sorted QUAD members (every
// fourth position through the classes, each over all rows of the tile, lane
// by lane with the per-tile fold of index and sign), far chunks (each mask's
// own source tile), and the PAIR / DIAG row sums turned into bins per tile by
// the kernel's outputs (four row quarters per PAIR output, tile bits added
// afterwards; one sum per diagonal term).  Two (g, v) pairs with weights are
// summed.  It also checks what the kernel relies on: every lane of an in-wave
// sum group (lanes that differ only in bits outside keep) computes the same
// bin index, every QUAD member sits in the class its position says and is
// visited by exactly one wave per tile.  The result is compared with the bins'
// own definitions in natural row coordinates:
//   QUAD  B[idx]       = sum_p w_p sum_r conj(g_p[r]) (-1)^{|r & zbase|} v_p[r ^ x], rows with bits idx at q0..q3
//   PAIR  B[idx], C_c  = the same over rows with bits idx at q0, q1 (C_c: rows with r_c = 1)
//   DIAG  E_n          = sum_p w_p sum_r conj(g_p[r]) (-1)^{|r & dz_n|} v_p[r]
//
// Exit status 0 when every case agrees to 1e-12 relative and no check failed;
// one line per case on stdout.
#include "grad.hip"

#include <complex>
#include <cstdio>
#include <random>

using namespace syk;
typedef std::complex<double> C;

namespace {

inline uint32_t rot_bits(uint32_t v, int M, int s) { return (v >> s) | ((v & ((1u << s) - 1u)) << (M - s)); }

int run_case(int N)
{
    std::mt19937_64 gen((uint64_t)N * 977 + 5);
    std::normal_distribution<double> nd;
    const int nc = N * (N - 1) * (N - 2) * (N - 3) / 24;
    std::vector<double> J(nc);
    for (double& v : J) v = nd(gen) * 0.1;
    TermTables T;
    build_tables(N, 1, J.data(), T);
    const int M = N / 2;
    const uint64_t D = 1ull << M;
    constexpr int PP = 2;
    std::vector<std::vector<C>> g(PP, std::vector<C>(D)), v(PP, std::vector<C>(D));
    const double wt[PP] = {0.75, -1.25};
    for (int u = 0; u < PP; ++u)
        for (uint64_t r = 0; r < D; ++r) {
            g[u][r] = C(nd(gen), nd(gen));
            v[u][r] = C(nd(gen), nd(gen));
        }

    // definitions
    std::vector<C> ref(T.n_bins, 0.0);
    for (size_t i = 0; i < T.masks.size(); ++i) {
        const MaskRec& m = T.masks[i];
        const uint32_t type = m.type_tab >> 28;
        C* B = &ref[T.bin_off[i]];
        for (int u = 0; u < PP; ++u)
            for (uint64_t r = 0; r < D; ++r) {
                const C gv = wt[u] * std::conj(g[u][r]);
                if (type == MASK_DIAG) {
                    for (int n = 0; n < T.n_diag; ++n)
                        B[n] += ((__builtin_popcount((uint32_t)r & T.dz[n]) & 1) ? -1.0 : 1.0) * gv * v[u][r];
                    continue;
                }
                const C t = ((__builtin_popcount((uint32_t)r & m.zbase) & 1) ? -1.0 : 1.0) * gv * v[u][r ^ m.x];
                if (type == MASK_QUAD) {
                    int idx = 0;
                    for (int q = 0; q < 4; ++q) idx |= (int)((r >> mask_q(m.qpack, q)) & 1u) << q;
                    B[idx] += t;
                } else {
                    const int idx = (int)((r >> mask_q(m.qpack, 0)) & 1u) | (int)((r >> mask_q(m.qpack, 1)) & 1u) << 1;
                    B[idx] += t;
                    for (int c = 0; c < M; ++c)
                        if ((r >> c) & 1u) B[4 + 4 * c + idx] += t;
                }
            }
    }

    // the gradient's launch shape and layouts (as grad_bins sets them up)
    const int tb = std::min(kGradTileBits, M), lb = std::min(tb, 6), KB = tb - lb, RPT = 1 << KB;
    const bool two = M - tb >= 7 && tb >= 8;
    std::vector<MaskRec> lm(T.masks);
    std::vector<uint8_t> lay(T.masks.size(), 0);
    if (two)
        for (size_t i = 0; i < lm.size(); ++i)
            if (quad_in_rotated(T.masks[i], M, tb)) {
                lm[i] = rotate_mask(T.masks[i], M, tb);
                lay[i] = 1;
            }
    const std::vector<KRec> kr = build_krecs(lm, T.bin_off, tb);
    const GradChunks GC = make_grad_chunks(lm, lay, T.bin_off, T.n_bins, tb, lb);
    // the pair vectors in both layouts
    std::vector<std::vector<C>> g_rot(PP, std::vector<C>(D)), v_rot(PP, std::vector<C>(D));
    for (int u = 0; u < PP; ++u)
        for (uint64_t r = 0; r < D; ++r) {
            const uint64_t rr = two ? rot_bits((uint32_t)r, M, tb) : r;
            g_rot[u][rr] = g[u][r];
            v_rot[u][rr] = v[u][r];
        }

    std::vector<C> out(T.n_bins, 0.0);
    int index_errors = 0, visit_errors = 0;
    const uint32_t tile_rows = 1u << tb;
    for (const GChunk& c : GC.chunks) {
        const std::vector<std::vector<C>>& gs = c.layout ? g_rot : g;
        const std::vector<std::vector<C>>& vs = c.layout ? v_rot : v;
        std::vector<C> bins((size_t)c.bin_count, 0.0);
        for (uint32_t tile = 0; tile < (uint32_t)(D >> tb); ++tile) {
            const uint32_t base = tile << tb;
            std::vector<uint32_t> fold(c.n_quad);
            if (!c.far)
                for (uint32_t j = 0; j < c.n_quad; ++j) {
                    const KRec& m = kr[GC.members[c.first + j]];
                    uint32_t qi = 0;
                    for (int q = 0; q < 4; ++q) qi |= ((base >> mask_q(m.qpack, q)) & 1u) << q;
                    fold[j] = qi | ((uint32_t)(__builtin_popcount(base & m.zbase) & 1) << 4);
                }
            // the staged source tile a member reads: bit 30 of its koffs picks one of the chunk's two
            auto sbase_of = [&](uint32_t j) {
                const uint32_t xh = ((GC.grec[j].koffs >> 30) & 1u) ? c.x_high2 : c.x_high;
                if (!c.far && ((kr[GC.members[j]].x_high) != xh)) ++index_errors;
                return (uint64_t)(tile ^ xh) << tb;
            };
            auto gk = [&](int u, uint32_t lane, int k) {
                return lane < (1u << lb) ? wt[u] * gs[u][base + lane + 64u * (uint32_t)k] : C(0.0);
            };
            std::vector<int> visits(c.n_quad, 0);
            for (uint32_t wave = 0; wave < 4; ++wave) {
                if (c.far) {
                    // every fourth member of the chunk, QUAD only, over all rows of the tile
                    for (uint32_t j = c.first + wave; j < c.first + c.count; j += 4) {
                        const KRec& m = kr[GC.members[j]];
                        if ((m.meta >> 28) != MASK_QUAD) continue;
                        C a = 0.0;
                        for (uint32_t lane = 0; lane < (1u << lb); ++lane)
                            for (int k = 0; k < RPT; ++k)
                                for (int u = 0; u < PP; ++u)
                                    a += std::conj(gk(u, lane, k)) *
                                         vs[u][((uint64_t)(tile ^ m.x_high) << tb) + lane + 64u * (uint32_t)k];
                        if (__builtin_popcount(base & m.zbase) & 1) a = -a;
                        uint32_t idx = 0;
                        for (int q = 0; q < 4; ++q) idx |= ((base >> mask_q(m.qpack, q)) & 1u) << q;
                        bins.at(GC.local[j] + idx) += a;
                    }
                    continue;
                }
                // near QUAD members: positions wave, wave + 4, ... through the classes
                uint32_t pos = wave, cls_end = 0;
                for (int cl = 0; cl < ipow3(KB); ++cl) {
                    const int XK = class_bits(cl, KB, 1), ZK = class_bits(cl, KB, 2);
                    cls_end += (c.cnt[cl >> 2] >> (8 * (cl & 3))) & 0xffu;
                    for (; pos < cls_end; pos += 4) {
                        const uint32_t j = c.first + pos;
                        ++visits.at(pos);
                        const GRec& q = GC.grec[j];
                        if (quad_class(lm[GC.members[j]].x, lm[GC.members[j]].zbase, lb, KB) != cl) ++index_errors;
                        const uint32_t fo = fold[pos];
                        auto lane_idx = [&](uint32_t t) {
                            uint32_t a = 0;
                            for (int mq = 0; mq < 4; ++mq) {
                                const uint32_t b = (q.sel >> (8 * mq)) & 0xffu;
                                if (b < 8) a += ((t >> b) & 1u) << mq;
                            }
                            return a + (fo & 15u);
                        };
                        const uint32_t keep = (q.koffs >> 24) & 63u;
                        const uint64_t sbase = sbase_of(j);
                        for (uint32_t lane = 0; lane < 64; ++lane) {
                            const uint32_t il = lane_idx(lane);
                            // every lane of this lane's group computes the same index
                            const uint32_t rep = (lane & keep) | (~keep & 15u);
                            if (lane_idx(rep) != il) ++index_errors;
                            const bool sl = ((__builtin_popcount(lane & q.zl) ^ (fo >> 4)) & 1) != 0;
                            for (int pp = 0; pp < RPT; ++pp) {
                                if ((pp & ~XK) != 0) continue;
                                C e = 0.0;
                                for (int k = 0; k < RPT; ++k) {
                                    if ((k & XK) != pp) continue;
                                    const double neg = (__builtin_popcount((uint32_t)k & (uint32_t)ZK) & 1) ? -1.0 : 1.0;
                                    for (int u = 0; u < PP; ++u) {
                                        const uint32_t e_src = (lane ^ q.xoff) + ((uint32_t)(k ^ XK) << 6);
                                        const C x = e_src < tile_rows ? vs[u][sbase + e_src] : C(0.0);
                                        e += neg * std::conj(gk(u, lane, k)) * x;
                                    }
                                }
                                uint32_t idx = il;
                                for (int b = 0; b < KB; ++b)
                                    if ((pp >> b) & 1) idx += (q.koffs >> (8 * b)) & 0xffu;
                                bins.at(16 * pos + idx) += sl ? -e : e;
                            }
                        }
                    }
                }
            }
            if (!c.far)
                for (uint32_t p = 0; p < c.n_quad; ++p)
                    if (visits[p] != 1) ++visit_errors;
            // PAIR / DIAG: thread t sums the rows t and t + 256 over the pairs
            std::vector<C> rows((size_t)kGradAccMasks * tile_rows, 0.0);
            for (uint32_t a = 0; a < c.n_acc; ++a) {
                const KRec& m = kr[GC.members[c.first + c.acc[a]]];
                const uint64_t sbase = c.far ? 0 : sbase_of(c.first + c.acc[a]);
                for (uint32_t rl = 0; rl < tile_rows; ++rl)
                    for (int u = 0; u < PP; ++u) {
                        const C x = c.far ? vs[u][((uint64_t)(tile ^ m.x_high) << tb) + rl] : vs[u][sbase + (rl ^ m.xl)];
                        rows[(size_t)a * tile_rows + rl] += std::conj(wt[u] * gs[u][base + rl]) * x;
                    }
            }
            // per-tile outputs as the kernel forms them
            for (uint32_t a = 0; a < c.n_acc; ++a) {
                const KRec& m = kr[GC.members[c.first + c.acc[a]]];
                C* mb = &bins.at(GC.local[c.first + c.acc[a]]);
                const C* rj = &rows[(size_t)a * tile_rows];
                if ((m.meta >> 28) == MASK_PAIR) {
                    const uint32_t q0 = mask_q(m.qpack, 0), q1 = mask_q(m.qpack, 1);
                    for (uint32_t o = 0; o < 4u * (uint32_t)(tb + 1); ++o) {
                        const uint32_t idx = o & 3u;
                        const int cb = (int)(o >> 2) - 1;
                        C sum = 0.0;
                        for (int qtr = 0; qtr < 4; ++qtr) {
                            C part = 0.0;
                            for (uint32_t rl = qtr * (tile_rows / 4); rl < (qtr + 1) * (tile_rows / 4); ++rl) {
                                const uint32_t r = base | rl;
                                if ((((r >> q0) & 1u) | (((r >> q1) & 1u) << 1)) != idx) continue;
                                if (cb >= 0 && !((rl >> cb) & 1u)) continue;
                                part += (__builtin_popcount(r & m.zbase) & 1) ? -rj[rl] : rj[rl];
                            }
                            sum += part;
                        }
                        if (cb >= 0) {
                            mb[4 + 4 * cb + idx] += sum;
                        } else {
                            mb[idx] += sum;
                            for (int cq = tb; cq < M; ++cq)
                                if ((base >> cq) & 1u) mb[4 + 4 * cq + idx] += sum;
                        }
                    }
                } else {
                    for (int n = 0; n < T.n_diag; ++n)
                        for (uint32_t rl = 0; rl < tile_rows; ++rl)
                            mb[n] += (__builtin_popcount((base | rl) & T.dz[n]) & 1) ? -rj[rl] : rj[rl];
                }
            }
        }
        // each member's bins to their place
        for (uint32_t j = c.first; j < c.first + c.count; ++j) {
            const uint32_t lo = GC.local[j];
            const uint32_t hi = (j + 1 < c.first + c.count) ? GC.local[j + 1] : c.bin_count;
            const uint64_t go = kr[GC.members[j]].bin0;
            for (uint32_t e = 0; e < hi - lo; ++e) out[go + e] += bins[lo + e];
        }
    }
    double err = 0.0, mx = 0.0;
    for (uint64_t i = 0; i < T.n_bins; ++i) {
        err = std::max(err, std::abs(out[i] - ref[i]));
        mx = std::max(mx, std::abs(ref[i]));
    }
    const double rel = err / mx;
    std::printf("N=%d tile_bits=%d rows_per_lane=%d layouts=%d chunks=%zu bins=%llu rel_err=%.3e index_errors=%d "
                "visit_errors=%d\n",
                N, tb, RPT, two ? 2 : 1, GC.chunks.size(), (unsigned long long)T.n_bins, rel, index_errors,
                visit_errors);
    std::fflush(stdout);
    return (rel < 1e-12 && index_errors == 0 && visit_errors == 0) ? 0 : 1;
}

}  // namespace

int main()
{
    int bad = 0;
    for (int N : {8, 12, 16, 20, 28, 34}) bad += run_case(N);
    return bad;
}
