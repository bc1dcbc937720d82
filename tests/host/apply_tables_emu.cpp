// Host-side check of the apply kernel's QUAD tables (no GPU).
//
// Builds the chunk and record tables of the apply kernel with the library's
// own host code (build_apply_tables, both row layouts), then evaluates the QUAD
// part of H psi from those tables exactly as k_apply<R, 8> reads them: per tile
// and chunk, the staged tables (tile sign and tile index bits folded in), then
// for every lane and row the groups of three masks (one lane index, one lane
// sign, one set of source rows, compile-time member classes) and the single
// masks by class.  The result is compared with the direct sum over the QUAD
// masks, (-1)^{|r & zbase|} T_x[bits of r at the flipped qubits] psi[r ^ x].
//
// Exit status 0 when every case agrees to 1e-12 relative and groups were found
// where the sizes allow them; one line per case on stdout.
#include "apply_h.hip"

#include <complex>
#include <cstdio>
#include <random>

using namespace syk;
typedef std::complex<double> C;

namespace {

int run_case(int N, int tb, bool two, uint32_t esz)
{
    std::mt19937_64 g((uint64_t)N * 131 + esz + (two ? 7 : 0));
    std::normal_distribution<double> nd;
    const int nc = N * (N - 1) * (N - 2) * (N - 3) / 24;
    std::vector<double> J(nc);
    for (double& v : J) v = nd(g) * 0.1;
    TermTables T;
    build_tables(N, 1, J.data(), T);
    const int M = N / 2;
    const uint64_t D = 1ull << M;
    const uint32_t rows = 1u << tb;
    std::vector<C> psi(D);
    for (C& v : psi) v = C(nd(g), nd(g));

    std::vector<C> ref(D, 0.0);
    for (uint64_t r = 0; r < D; ++r)
        for (const MaskRec& m : T.masks) {
            if ((m.type_tab >> 28) != MASK_QUAD) continue;
            int idx = 0;
            for (int k = 0; k < 4; ++k) idx |= (int)((r >> mask_q(m.qpack, k)) & 1u) << k;
            const double sg = (__builtin_popcount((uint32_t)r & m.zbase) & 1) ? -1.0 : 1.0;
            const c128 t = T.tab4[(size_t)(m.type_tab & 0x0fffffffu) * 16 + idx];
            ref[r] += sg * C(t.re, t.im) * psi[r ^ m.x];
        }

    std::vector<C> out(D, 0.0);
    int groups = 0, bad_layout = 0;
    for (int layout = 0; layout < (two ? 2 : 1); ++layout) {
        const std::vector<MaskRec> ms = layout_masks(T.masks, M, tb, two, layout);
        std::vector<QApplyChunk> ch;
        std::vector<QRec> rc;
        std::vector<FarRec> far;
        build_apply_tables(ms, tb, kLaneBits, esz, ch, rc, far);
        // every record index a chunk's loops reach, plus the one-ahead record
        for (const QApplyChunk& c : ch) {
            if (c.first + c.n_quad + c.n_pair + c.n_diag >= rc.size()) ++bad_layout;
            if (c.n_quad + c.n_pair > (uint32_t)apply_chunk_masks(esz)) ++bad_layout;
        }
        auto to_layout = [&](uint64_t r) { return layout ? (uint64_t)rotate_bits((uint32_t)r, M, tb) : r; };
        std::vector<C> ps(D), o(D, 0.0);
        for (uint64_t r = 0; r < D; ++r) ps[to_layout(r)] = psi[r];
        for (uint32_t tile = 0; tile < (uint32_t)(D >> tb); ++tile) {
            const uint32_t base = tile << tb;
            std::vector<C> src(rows), tabs((size_t)apply_chunk_masks(esz) * 16);
            for (const QApplyChunk& c : ch) {
                const uint64_t sbase = (uint64_t)(tile ^ c.x_high) << tb;
                for (uint32_t r = 0; r < rows; ++r) src[r] = ps[sbase + r];
                for (uint32_t e = 0; e < c.n_quad * 16; ++e) {
                    const QRec& qr = rc[c.first + (e >> 4)];
                    uint32_t qi = 0;
                    for (int k = 0; k < 4; ++k) qi |= ((base >> mask_q(qr.qpack, k)) & 1u) << k;
                    const c128 t = T.tab4[(size_t)qr.tab * 16 + ((e & 15u) ^ qi)];
                    tabs[e] = ((__builtin_popcount(base & qr.zbase) & 1) ? -1.0 : 1.0) * C(t.re, t.im);
                }
                auto tab_at = [&](uint32_t off) { return tabs.at(off / esz); };
                for (uint32_t tid = 0; tid < 256; ++tid) {
                    // v_perm / v_dot4: lane part of the table byte offset
                    auto lane_index = [&](uint32_t sel) {
                        uint32_t a = 0;
                        for (int m = 0; m < 4; ++m) {
                            const uint32_t b = (sel >> (8 * m)) & 0xffu;
                            if (b < 8) a += ((tid >> b) & 1u) * (esz << m);
                        }
                        return a;
                    };
                    auto src_row = [&](const QRec& q, int k) { return src.at((tid ^ (q.xoff / esz)) + ((uint32_t)k << kLaneBits)); };
                    auto row_out = [&](int k) -> C& { return o[base + tid + ((uint32_t)k << kLaneBits)]; };
                    uint32_t mi = c.first;
                    for (int gc = 0; gc < kQuadGroupClasses; ++gc) {
                        const int Jg = 1 + (gc >> 1), P = gc & 1;
                        const int n = (int)((c.cnt[(kQuadClasses + gc) >> 2] >> (8 * ((kQuadClasses + gc) & 3))) & 0xffu);
                        if (tid == 0 && tile == 0) groups += n;
                        for (int i = 0; i < n; ++i, mi += 3) {
                            const QRec& q = rc[mi];
                            const uint32_t ia = lane_index(q.sel) + (mi - c.first) * 16u * esz;
                            const double sl = (__builtin_popcount(tid & q.zl) & 1) ? -1.0 : 1.0;
                            for (int j = 0; j < 3; ++j) {
                                const int XK = group_xk(Jg, j), ZK = group_zk(XK, P);
                                for (int k = 0; k < 8; ++k) {
                                    const int e = pack_bits3(k & XK, XK);
                                    C t = sl * tab_at(ia + (uint32_t)e * q.koffs + (uint32_t)j * 16u * esz);
                                    if (popc3(k & ZK) & 1) t = -t;
                                    // member j reads the group's source row k ^ XK
                                    row_out(k) += t * src_row(q, k ^ XK);
                                }
                            }
                        }
                    }
                    for (int cl = 0; cl < kQuadClasses; ++cl) {
                        const int XK = class_bits(cl, 3, 1), ZK = class_bits(cl, 3, 2);
                        const int n = (int)((c.cnt[cl >> 2] >> (8 * (cl & 3))) & 0xffu);
                        for (int i = 0; i < n; ++i, ++mi) {
                            const QRec& q = rc[mi];
                            const uint32_t ia = lane_index(q.sel) + (mi - c.first) * 16u * esz;
                            const double sl = (__builtin_popcount(tid & q.zl) & 1) ? -1.0 : 1.0;
                            for (int k = 0; k < 8; ++k) {
                                const int p = k & XK;
                                uint32_t off = 0;
                                for (int b = 0; b < 3; ++b)
                                    if ((p >> b) & 1) off += (q.koffs >> (8 * b)) & 0xffu;
                                C t = sl * tab_at(ia + off);
                                if (popc3(k & ZK) & 1) t = -t;
                                row_out(k) += t * src_row(q, k ^ XK);
                            }
                        }
                    }
                    if (mi != c.first + c.n_quad) ++bad_layout;   // QUAD records come first, all visited
                }
            }
            // masks that flip only qubits above the tile: one coefficient per tile
            for (const FarRec& f : far) {
                uint32_t qi = 0;
                for (int k = 0; k < 4; ++k) qi |= ((base >> mask_q(f.qpack, k)) & 1u) << k;
                const c128 t = T.tab4[(size_t)f.tab * 16 + qi];
                const double sg = (__builtin_popcount(base & f.zbase) & 1) ? -1.0 : 1.0;
                for (uint32_t r = 0; r < rows; ++r)
                    o[base + r] += sg * C(t.re, t.im) * ps[((uint64_t)(tile ^ f.x_high) << tb) + r];
            }
        }
        for (uint64_t r = 0; r < D; ++r) out[r] += o[to_layout(r)];
    }
    double err = 0.0, mx = 0.0;
    for (uint64_t r = 0; r < D; ++r) {
        err = std::max(err, std::abs(out[r] - ref[r]));
        mx = std::max(mx, std::abs(ref[r]));
    }
    const double rel = err / mx;
    std::printf("N=%d tile_bits=%d layouts=%d esz=%u groups(tile 0)=%d rel_err=%.3e table_errors=%d\n", N, tb,
                two ? 2 : 1, esz, groups, rel, bad_layout);
    std::fflush(stdout);
    return (rel < 1e-12 && groups > 0 && bad_layout == 0) ? 0 : 1;
}

}  // namespace

int main()
{
    int bad = 0;
    for (int N : {22, 24, 28})
        for (bool two : {false, true})
            for (uint32_t esz : {16u, 8u}) bad += run_case(N, 11, two, esz);
    return bad;
}
