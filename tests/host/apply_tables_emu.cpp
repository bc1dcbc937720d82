// Host-side check of the apply kernel's tables (no GPU).
//
// Builds the chunk and record tables of the apply kernel with the library's
// own host code (build_apply_tables, both row layouts), then evaluates H psi
// from those tables exactly as k_apply<R, 8> reads them: per tile and chunk,
// the staged QUAD tables (tile sign and tile index bits folded in) and PAIR row
// forms, then for every lane and row the groups of three QUAD masks (one lane
// index, one lane sign, one set of source rows, compile-time member classes),
// the single QUAD masks by class, the PAIR masks that flip no k bit (A plus the
// k-bit steps Om_b), the other PAIR masks row by row, and the diagonal.  The
// result is compared with the direct sum over the term tables:
// (-1)^{|r & zbase|} T_x[bits of r at the flipped qubits] psi[r ^ x] (QUAD),
// (-1)^{|r & zbase|} sum_e Phi[bits at q0, q1][e] L_e(r) psi[r ^ x] (PAIR),
// sum_n d_n (-1)^{|r & z_n|} psi[r] (DIAG).  For the parity sectors the same is
// done on the sector tables, whose direct sum is first compared with the full
// H applied to the sector state embedded in the full space.
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

// The direct sum over a set of term tables on M qubits (n_real = 1).
std::vector<C> direct_apply(const TermTables& T, int M, const std::vector<C>& psi)
{
    const uint64_t D = 1ull << M;
    std::vector<C> out(D, 0.0);
    for (uint64_t r = 0; r < D; ++r)
        for (const MaskRec& m : T.masks) {
            const uint32_t type = m.type_tab >> 28, tab = m.type_tab & 0x0fffffffu;
            const double sg = (__builtin_popcount((uint32_t)r & m.zbase) & 1) ? -1.0 : 1.0;
            if (type == MASK_QUAD) {
                int idx = 0;
                for (int k = 0; k < 4; ++k) idx |= (int)((r >> mask_q(m.qpack, k)) & 1u) << k;
                const c128 t = T.tab4[(size_t)tab * 16 + idx];
                out[r] += sg * C(t.re, t.im) * psi[r ^ m.x];
            } else if (type == MASK_PAIR) {
                const int idx = (int)((r >> mask_q(m.qpack, 0)) & 1u) | (int)((r >> mask_q(m.qpack, 1)) & 1u) << 1;
                C d = 0.0;
                for (int e = 0; e < 4; ++e) {
                    const double* w = &T.w2[((size_t)tab * 4 + e) * (M + 1)];
                    double Le = w[M];
                    for (int c = 0; c < M; ++c) Le += w[c] * (double)((r >> c) & 1u);
                    const c128 ph = T.phi2[(size_t)tab * 16 + idx * 4 + e];
                    d += C(ph.re, ph.im) * Le;
                }
                out[r] += sg * d * psi[r ^ m.x];
            } else {
                double d = 0.0;
                for (int n = 0; n < T.n_diag; ++n)
                    d += (__builtin_popcount((uint32_t)r & T.dz[n]) & 1) ? -T.dw[n] : T.dw[n];
                out[r] += d * psi[r];
            }
        }
    return out;
}

// sector < 0: the full tables of N Majoranas; sector 0 / 1: the tables of that
// fermion-parity sector (M - 1 qubits), which are first checked against the
// full H on the embedded state.
int run_case(int N, int tb, bool two, uint32_t esz, int sector)
{
    std::mt19937_64 g((uint64_t)N * 131 + esz + (two ? 7 : 0) + 1000 * (uint64_t)(sector + 1));
    std::normal_distribution<double> nd;
    const int nc = N * (N - 1) * (N - 2) * (N - 3) / 24;
    std::vector<double> J(nc);
    for (double& v : J) v = nd(g) * 0.1;
    TermTables TF, TS;
    build_tables(N, 1, J.data(), TF);
    if (sector >= 0) build_sector_tables(TF, sector, TS);
    const TermTables& T = sector >= 0 ? TS : TF;
    const int M = sector >= 0 ? N / 2 - 1 : N / 2;
    const uint64_t D = 1ull << M;
    const uint32_t rows = 1u << tb;
    std::vector<C> psi(D);
    for (C& v : psi) v = C(nd(g), nd(g));

    auto diag_at = [&](uint64_t r) {
        double d = 0.0;
        for (int n = 0; n < T.n_diag; ++n) d += (__builtin_popcount((uint32_t)r & T.dz[n]) & 1) ? -T.dw[n] : T.dw[n];
        return d;
    };
    auto wrow = [&](uint32_t tab, int e) { return &T.w2[((size_t)tab * 4 + e) * (M + 1)]; };
    const std::vector<C> ref = direct_apply(T, M, psi);
    double sector_err = 0.0;
    if (sector >= 0) {
        // sector row u is the full row u + 2^M (parity(u) ^ s); H keeps the parity
        auto full_row = [&](uint64_t u) { return u + ((uint64_t)((__builtin_popcountll(u) & 1) ^ sector) << M); };
        std::vector<C> pf(2 * D, 0.0);
        for (uint64_t u = 0; u < D; ++u) pf[full_row(u)] = psi[u];
        const std::vector<C> hf = direct_apply(TF, M + 1, pf);
        double e = 0.0, off = 0.0, mx = 0.0;
        for (uint64_t u = 0; u < D; ++u) {
            e = std::max(e, std::abs(hf[full_row(u)] - ref[u]));
            off = std::max(off, std::abs(hf[full_row(u) ^ (1ull << M)]));   // the other sector's row
            mx = std::max(mx, std::abs(ref[u]));
        }
        sector_err = std::max(e, off) / mx;
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
        const uint32_t rsz = esz / 2;   // bytes of one real component
        for (const QApplyChunk& c : ch) {
            if (c.first + c.n_quad + c.n_pair + c.n_diag >= rc.size()) ++bad_layout;
            if (c.n_quad + c.n_pair > (uint32_t)apply_chunk_masks(esz)) ++bad_layout;
            // PAIR slots: after the QUAD tables, inside the table area
            for (uint32_t p = 0; p < c.n_pair; ++p) {
                const uint32_t sel = rc[c.first + c.n_quad + p].sel;
                if (sel < c.n_quad * 16u * esz || sel + 8u * 4u * rsz > (uint32_t)apply_chunk_masks(esz) * 16u * esz)
                    ++bad_layout;
            }
        }
        auto to_layout = [&](uint64_t r) { return layout ? (uint64_t)rotate_bits((uint32_t)r, M, tb) : r; };
        std::vector<C> ps(D), o(D, 0.0);
        for (uint64_t r = 0; r < D; ++r) ps[to_layout(r)] = psi[r];
        for (uint32_t tile = 0; tile < (uint32_t)(D >> tb); ++tile) {
            const uint32_t base = tile << tb;
            std::vector<C> src(rows), tabs((size_t)apply_chunk_masks(esz) * 16);
            std::vector<double> pst((size_t)apply_chunk_masks(esz) * 16 * esz / rsz);
            for (const QApplyChunk& c : ch) {
                uint32_t n_flat = 0;
                for (int b = 0; b < 8; ++b) n_flat += (c.pcnt[b >> 2] >> (8 * (b & 3))) & 0xffu;
                // PAIR row forms: W_e + the tile and k bits of the row (flat masks: row 0 only)
                for (uint32_t p = 0; p < c.n_pair; ++p) {
                    const QRec& pq = rc[c.first + c.n_quad + p];
                    for (int k = 0; k < (p < n_flat ? 1 : 8); ++k)
                        for (int e = 0; e < 4; ++e) {
                            const double* w = wrow(pq.tab, e);
                            const uint32_t rb = base | ((uint32_t)k << kLaneBits);
                            double acc = w[M];
                            for (int cq = kLaneBits; cq < M; ++cq)
                                if ((rb >> cq) & 1u) acc += w[cq];
                            pst.at(pq.sel / rsz + k * 4 + e) = acc;
                        }
                }
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
                    // PAIR: D = (-1)^{|r & zbase|} sum_e phi_e sigma_e L_e(r), phi_e the entry
                    // with both qubit bits set, sigma_e the signs of the bits that are 0
                    auto sigma = [](int e, uint32_t sa, uint32_t sb) {
                        return (((e & 1) ? sa : 0u) ^ ((e & 2) ? sb : 0u)) ? -1.0 : 1.0;
                    };
                    auto lane_forms = [&](const QRec& q, double (&l)[4]) {
                        for (int e = 0; e < 4; ++e) {
                            l[e] = 0.0;
                            for (int cq = 0; cq < kLaneBits; ++cq) l[e] += wrow(q.tab, e)[cq] * (double)((tid >> cq) & 1u);
                        }
                    };
                    const uint32_t rl = tid | base;
                    for (int zk = 0; zk < 8; ++zk) {
                        const int n = (int)((c.pcnt[zk >> 2] >> (8 * (zk & 3))) & 0xffu);
                        for (int i = 0; i < n; ++i, ++mi) {
                            const QRec& q = rc[mi];
                            const uint32_t q0 = mask_q(q.qpack, 0), q1 = mask_q(q.qpack, 1);
                            const uint32_t sa = ((rl >> q0) & 1u) ^ 1u, sb = ((rl >> q1) & 1u) ^ 1u;
                            const double s = (__builtin_popcount(rl & q.zbase) & 1) ? -1.0 : 1.0;
                            double l[4];
                            lane_forms(q, l);
                            auto combine = [&](const double (&y)[4]) {
                                C o = 0.0;
                                for (int e = 0; e < 4; ++e) {
                                    const c128 ph = T.phi2[(size_t)q.tab * 16 + 12 + e];
                                    o += C(ph.re, ph.im) * (sigma(e, sa, sb) * y[e]);
                                }
                                return s * o;
                            };
                            C X[8];
                            double y0[4];
                            for (int e = 0; e < 4; ++e) y0[e] = l[e] + pst.at(q.sel / rsz + e);
                            X[0] = combine(y0);
                            for (int b = 0; b < 3; ++b) {
                                double yb[4];
                                for (int e = 0; e < 4; ++e) yb[e] = wrow(q.tab, e)[kLaneBits + b];
                                const C om = combine(yb);
                                for (int k = 1 << b; k < (2 << b); ++k) X[k] = X[k - (1 << b)] + om;
                            }
                            for (int k = 0; k < 8; ++k) {
                                const double neg = (popc3(k & zk) & 1) ? -1.0 : 1.0;
                                row_out(k) += neg * X[k] * src_row(q, k);
                            }
                        }
                    }
                    for (uint32_t i = n_flat; i < c.n_pair; ++i, ++mi) {
                        const QRec& q = rc[mi];
                        const uint32_t q0 = mask_q(q.qpack, 0), q1 = mask_q(q.qpack, 1);
                        double l[4];
                        lane_forms(q, l);
                        for (int k = 0; k < 8; ++k) {
                            const uint32_t r = rl | ((uint32_t)k << kLaneBits);
                            const uint32_t sa = ((r >> q0) & 1u) ^ 1u, sb = ((r >> q1) & 1u) ^ 1u;
                            const double s = (__builtin_popcount(r & q.zbase) & 1) ? -1.0 : 1.0;
                            C d = 0.0;
                            for (int e = 0; e < 4; ++e) {
                                const c128 ph = T.phi2[(size_t)q.tab * 16 + 12 + e];
                                d += C(ph.re, ph.im) * (sigma(e, sa, sb) * (l[e] + pst.at(q.sel / rsz + k * 4 + e)));
                            }
                            row_out(k) += s * d * src_row(q, k ^ (int)q.koffs);
                        }
                    }
                    for (uint32_t i = 0; i < c.n_diag; ++i, ++mi)
                        for (int k = 0; k < 8; ++k) {
                            const uint32_t r = rl | ((uint32_t)k << kLaneBits);   // own row (x = 0: layout 0, own tile)
                            row_out(k) += diag_at(r) * src.at(tid + ((uint32_t)k << kLaneBits));
                        }
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
    std::printf("N=%d sector=%d tile_bits=%d layouts=%d esz=%u groups(tile 0)=%d rel_err=%.3e sector_err=%.3e "
                "table_errors=%d\n", N, sector, tb, two ? 2 : 1, esz, groups, rel, sector_err, bad_layout);
    std::fflush(stdout);
    return (rel < 1e-12 && sector_err < 1e-12 && groups > 0 && bad_layout == 0) ? 0 : 1;
}

}  // namespace

int main()
{
    int bad = 0;
    for (int N : {22, 24, 28})
        for (bool two : {false, true})
            for (uint32_t esz : {16u, 8u}) bad += run_case(N, 11, two, esz, -1);
    // parity sectors (M - 1 qubits)
    for (int s : {0, 1})
        for (bool two : {false, true}) bad += run_case(24, 11, two, 16u, s);
    bad += run_case(28, 11, true, 8u, 1);
    return bad;
}
