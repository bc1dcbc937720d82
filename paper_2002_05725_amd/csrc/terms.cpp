// Term builder.  Each coupling J_ijkl of Eq. 1 multiplies chi_i chi_j chi_k chi_l;
// under the Jordan-Wigner map of the SI this product is one Pauli string
// (1/4) i^ph X^x Z^z.  Terms are grouped by their flip mask x: every mask has
// even weight (the SI's conserved fermion parity) and |x| is 4, 2 or 0.
#include "terms.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <unordered_map>

namespace syk {

namespace {

struct Term {
    Pauli p;
    int64_t n;   // coupling index
};

inline std::complex<double> iphase(int ph)
{
    static const std::complex<double> v[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
    return v[ph & 3];
}

void fail(const std::string& m) { throw Error(SYK_EUNSUPPORTED, "term structure: " + m); }

}  // namespace

void build_tables(int N, int n_real, const double* J, TermTables& T)
{
    const int M = N / 2;
    T.N = N;
    T.M = M;
    T.n_real = n_real;

    Pauli chi[64];
    for (int a = 0; a < N; ++a) chi[a] = majorana_pauli(a);

    // Every quartet as a Pauli string, bucketed by flip mask.
    std::unordered_map<uint32_t, std::vector<Term>> by_x;
    int64_t n = 0;
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j)
            for (int k = j + 1; k < N; ++k)
                for (int l = k + 1; l < N; ++l, ++n) {
                    Pauli p = pauli_mul(pauli_mul(chi[i], chi[j]), pauli_mul(chi[k], chi[l]));
                    by_x[p.x].push_back({p, n});
                }
    T.n_terms = n;

    std::vector<uint32_t> xs;
    xs.reserve(by_x.size());
    for (auto& kv : by_x) xs.push_back(kv.first);
    std::sort(xs.begin(), xs.end());

    T.masks.clear();
    T.tab4.clear();
    T.qinfo.clear();
    T.phi2.clear();
    T.w2.clear();
    T.dz.clear();
    T.dw.clear();
    T.n_quad = T.n_pair = T.n_diag = 0;
    T.terms.assign((size_t)n, TermRef{});
    T.bin_off.clear();
    T.n_bins = 0;

    const size_t NQ = (size_t)n;
    auto coef = [&](const Term& t, int r) {   // J * i^ph / 4 for realisation r
        return J[(size_t)r * NQ + t.n] * 0.25 * iphase(t.p.ph);
    };

    for (uint32_t x : xs) {
        const std::vector<Term>& ts = by_x[x];
        const int w = __builtin_popcount(x);
        const uint32_t mask_index = (uint32_t)T.masks.size();
        for (const Term& t : ts) T.terms[t.n] = TermRef{mask_index, t.p.z, t.p.ph, -1};
        T.bin_off.push_back(T.n_bins);
        T.n_bins += (w == 4) ? 16 : (w == 2) ? 4 + 4 * (uint64_t)M : (uint64_t)ts.size();
        MaskRec rec{};
        rec.x = x;
        int qn = 0;
        uint32_t q[4] = {0, 0, 0, 0};
        for (int b = 0; b < M; ++b)
            if (x >> b & 1u) {
                q[qn] = (uint32_t)b;
                rec.qpack |= (uint32_t)b << (8 * qn);
                ++qn;
            }

        if (w == 4) {
            // All 16 terms share their Z string outside the flipped qubits.
            if (ts.size() != 16) fail("weight-4 mask without 16 terms");
            uint32_t zb = ts[0].p.z & ~x;
            for (const Term& t : ts)
                if ((t.p.z & ~x) != zb) fail("weight-4 mask with differing Z strings");
            rec.zbase = zb;
            rec.type_tab = (uint32_t)MASK_QUAD << 28 | (uint32_t)T.n_quad;
            // T[idx]: idx bit m = bit q_m of the output row r; the source row
            // s = r ^ x has the opposite bits there.
            for (int r = 0; r < n_real; ++r)
                for (int idx = 0; idx < 16; ++idx) {
                    uint32_t s_loc = 0;
                    for (int m = 0; m < 4; ++m)
                        if (!((idx >> m) & 1)) s_loc |= 1u << q[m];
                    std::complex<double> acc = 0.0;
                    for (const Term& t : ts) {
                        double sg = (__builtin_popcount(s_loc & t.p.z) & 1) ? -1.0 : 1.0;
                        acc += sg * coef(t, r);
                    }
                    T.tab4.push_back({acc.real(), acc.imag()});
                }
            T.qinfo.push_back(rec.qpack);
            T.qinfo.push_back(rec.zbase);
            ++T.n_quad;
        } else if (w == 2) {
            // Terms chi_A chi_B chi_2c chi_2c+1: Z string = zbase ^ (bits at
            // q0, q1) ^ (1 << c), with c not flipped.  e = (z_q0, z_q1).
            const uint32_t qa = q[0], qb = q[1];
            // chi_A chi_B contributes the Z string on the qubits strictly
            // between q0 and q1 (plus bits at q0, q1); the pair adds Z_c.
            // Checked term by term below.
            const uint32_t zb = ((1u << qb) - 1u) & ~((1u << (qa + 1)) - 1u);
            rec.zbase = zb;
            rec.type_tab = (uint32_t)MASK_PAIR << 28 | (uint32_t)T.n_pair;
            // Phase class of each e must be uniform (real or imaginary).
            int cls[4] = {-1, -1, -1, -1};
            std::vector<double> wts((size_t)n_real * 4 * (M + 1), 0.0);
            for (const Term& t : ts) {
                uint32_t extra = (t.p.z & ~x) ^ zb;
                if (__builtin_popcount(extra) != 1 || (extra & x)) fail("weight-2 term without a single Z_c");
                int c = __builtin_ctz(extra);
                T.terms[t.n].slot = c;
                int e = (int)((t.p.z >> qa) & 1u) | (int)((t.p.z >> qb) & 1u) << 1;
                int c_cls = t.p.ph & 1;              // 0: real phase, 1: imaginary
                double sgn = (t.p.ph & 2) ? -1.0 : 1.0;
                if (cls[e] < 0) cls[e] = c_cls;
                if (cls[e] != c_cls) fail("weight-2 mask with mixed phase class");
                for (int r = 0; r < n_real; ++r) {
                    double v = J[(size_t)r * NQ + t.n] * 0.25 * sgn;
                    // sigma_c = 1 - 2 r_c:  v sigma_c = v - 2 v r_c
                    wts[((size_t)r * 4 + e) * (M + 1) + M] += v;
                    wts[((size_t)r * 4 + e) * (M + 1) + c] += -2.0 * v;
                }
            }
            // Phi[idx][e] = i^cls_e (-1)^{s_q0 e_0 + s_q1 e_1}, s = opposite of r's bits.
            for (int idx = 0; idx < 4; ++idx)
                for (int e = 0; e < 4; ++e) {
                    int sa = !((idx >> 0) & 1), sb = !((idx >> 1) & 1);
                    double sg = (((sa & (e & 1)) ^ (sb & (e >> 1))) & 1) ? -1.0 : 1.0;
                    std::complex<double> ph = (cls[e] == 1) ? std::complex<double>(0, sg)
                                                            : std::complex<double>(sg, 0);
                    if (cls[e] < 0) ph = 0.0;
                    T.phi2.push_back({ph.real(), ph.imag()});
                }
            T.w2.insert(T.w2.end(), wts.begin(), wts.end());
            ++T.n_pair;
        } else if (w == 0) {
            rec.zbase = 0;
            rec.type_tab = (uint32_t)MASK_DIAG << 28;
            T.n_diag = (int)ts.size();
            T.dz.resize(ts.size());
            T.dw.assign((size_t)n_real * ts.size(), 0.0);
            for (size_t m = 0; m < ts.size(); ++m) {
                T.dz[m] = ts[m].p.z;
                T.terms[ts[m].n].slot = (int)m;
                if (ts[m].p.ph & 1) fail("diagonal term with imaginary phase");
                double sgn = (ts[m].p.ph & 2) ? -1.0 : 1.0;
                for (int r = 0; r < n_real; ++r) T.dw[(size_t)r * ts.size() + m] = J[(size_t)r * NQ + ts[m].n] * 0.25 * sgn;
            }
        } else {
            fail("flip mask of odd or large weight");
        }
        T.masks.push_back(rec);
    }
}

void couplings_from_bins(const TermTables& T, const double* bins, double* out)
{
    typedef std::complex<double> C;
    auto bin = [&](uint64_t i) { return C(bins[2 * i], bins[2 * i + 1]); };
    const int M = T.M;
    for (size_t n = 0; n < T.terms.size(); ++n) {
        const TermRef& tr = T.terms[n];
        const MaskRec& m = T.masks[tr.mask];
        const uint64_t off = T.bin_off[tr.mask];
        const uint32_t type = m.type_tab >> 28;
        const C ph = iphase(tr.ph) * 0.25;
        C s = 0.0;
        if (type == MASK_QUAD) {
            // the term's own 16-entry table with J = 1 (same construction as build_tables)
            for (int idx = 0; idx < 16; ++idx) {
                uint32_t s_loc = 0;
                for (int j = 0; j < 4; ++j)
                    if (!((idx >> j) & 1)) s_loc |= 1u << mask_q(m.qpack, j);
                const double sg = (__builtin_popcount(s_loc & tr.z) & 1) ? -1.0 : 1.0;
                s += sg * ph * bin(off + idx);
            }
        } else if (type == MASK_PAIR) {
            const uint32_t qa = mask_q(m.qpack, 0), qb = mask_q(m.qpack, 1);
            const int e0 = (int)((tr.z >> qa) & 1u), e1 = (int)((tr.z >> qb) & 1u);
            for (int idx = 0; idx < 4; ++idx) {
                const int sa = !(idx & 1), sb = !((idx >> 1) & 1);
                const double sg = (((sa & e0) ^ (sb & e1)) & 1) ? -1.0 : 1.0;
                s += sg * ph * (bin(off + idx) - 2.0 * bin(off + 4 + 4 * (uint64_t)tr.slot + idx));
            }
        } else {
            s = ph * bin(off + tr.slot);
        }
        out[n] = s.real();
        (void)M;
    }
}

}  // namespace syk

namespace syk {

// Tables of H restricted to one fermion-parity sector (SI, section
// "Jordan-Wigner transformation": H conserves the parity of the qubit string,
// so it is block-diagonal in the two sectors).  A sector-s state keeps the
// rows r with popcount(r) = s (mod 2), indexed by u = r without its top qubit
// t = M-1, whose bit is then parity(u) ^ s.  Every flip mask has even weight,
// so x acts on u as x & low.  A dependence on the implied bit b = parity(u)^s
// becomes a Z string over all of u: (-1)^b = (-1)^s (-1)^{|u & low|}.
//  - QUAD masks without t: unchanged.  With q3 = t the table index bit 3 is b:
//    T[i | b<<3] = A[i] + (-1)^b B[i] gives two masks flipping q0..q2 with
//    tables A and (-1)^s (-1)^{|i|} B (bit 3 of the index unused, qubit 31 as
//    a never-set placeholder), Z strings zbase and (zbase ^ low) minus x.
//  - PAIR masks with q1 = t: the terms with e1 = 0 do not see b, those with
//    e1 = 1 carry (-1)^{1 + b}: two masks flipping q0 (placeholder 31 for q1,
//    which the kernel reads as bit 0, flipping e1 = 1 terms once), Z strings
//    zbase and zbase ^ low.  Otherwise the linear forms' term w_{e,t} r_t =
//    w/2 - (w/2)(-1)^s (-1)^{|u & low|} moves w/2 into W_e and leaves a second
//    mask with constant forms -(-1)^s w_{e,t}/2 and Z string zbase ^ low.
//  - DIAG terms with Z on t: Z string (dz & low) ^ low, coefficient times (-1)^s.
void build_sector_tables(const TermTables& F, int s, TermTables& out)
{
    const int M = F.M, R = F.n_real;
    if (M < 3) throw Error(SYK_EINVAL, "parity sectors need N >= 6");
    const int tq = M - 1;
    const uint32_t low = (1u << tq) - 1u;
    const double ss = (s & 1) ? -1.0 : 1.0;
    out = TermTables{};
    out.N = F.N;
    out.M = tq;
    out.n_real = R;
    out.n_terms = F.n_terms;
    std::vector<MaskRec> masks;
    auto add_quad = [&](uint32_t x, uint32_t zb, uint32_t qpack, const std::function<c128(int, int)>& tab) {
        MaskRec m{x, zb, qpack, (uint32_t)MASK_QUAD << 28 | (uint32_t)out.n_quad};
        masks.push_back(m);
        for (int r = 0; r < R; ++r)
            for (int i = 0; i < 16; ++i) out.tab4.push_back(tab(r, i));
        out.qinfo.push_back(qpack);
        out.qinfo.push_back(zb);
        ++out.n_quad;
    };
    const int Wn = M + 1;   // weights per linear form in the full tables
    auto add_pair = [&](uint32_t x, uint32_t zb, uint32_t qpack, const std::function<c128(int)>& phi,
                        const std::function<double(int, int, int)>& w /* (r, e, c <= tq; c == tq is W) */) {
        MaskRec m{x, zb, qpack, (uint32_t)MASK_PAIR << 28 | (uint32_t)out.n_pair};
        masks.push_back(m);
        for (int i = 0; i < 16; ++i) out.phi2.push_back(phi(i));
        for (int r = 0; r < R; ++r)
            for (int e = 0; e < 4; ++e)
                for (int c = 0; c <= tq; ++c) out.w2.push_back(w(r, e, c));
        ++out.n_pair;
    };
    for (const MaskRec& m : F.masks) {
        const uint32_t type = m.type_tab >> 28, tab = m.type_tab & 0x0fffffffu;
        if (type == MASK_QUAD) {
            const c128* T = &F.tab4[(size_t)tab * R * 16];
            if (!((m.x >> tq) & 1u)) {
                add_quad(m.x, m.zbase, m.qpack, [&](int r, int i) { return T[r * 16 + i]; });
            } else {
                if (mask_q(m.qpack, 3) != (uint32_t)tq || (m.zbase >> tq)) throw Error(SYK_EINVAL, "sector: QUAD layout");
                const uint32_t x = m.x & low;
                const uint32_t qp = (m.qpack & 0x00ffffffu) | (31u << 24);
                add_quad(x, m.zbase, qp, [&](int r, int i) {
                    const c128 a = T[r * 16 + (i & 7)], b = T[r * 16 + ((i & 7) | 8)];
                    return c128{0.5 * (a.re + b.re), 0.5 * (a.im + b.im)};
                });
                add_quad(x, (m.zbase ^ low) & ~x, qp, [&](int r, int i) {
                    const c128 a = T[r * 16 + (i & 7)], b = T[r * 16 + ((i & 7) | 8)];
                    const double sg = ss * ((__builtin_popcount((unsigned)(i & 7)) & 1) ? -1.0 : 1.0);
                    return c128{0.5 * sg * (a.re - b.re), 0.5 * sg * (a.im - b.im)};
                });
            }
        } else if (type == MASK_PAIR) {
            const c128* P = &F.phi2[(size_t)tab * 16];
            const double* Wt = &F.w2[(size_t)tab * R * 4 * Wn];
            auto wf = [&](int r, int e, int c) { return Wt[((size_t)r * 4 + e) * Wn + c]; };
            if (mask_q(m.qpack, 1) == (uint32_t)tq) {
                for (int r = 0; r < R; ++r)
                    for (int e = 0; e < 4; ++e)
                        if (wf(r, e, tq) != 0.0) throw Error(SYK_EINVAL, "sector: pair on the top qubit");
                const uint32_t x = m.x & low;
                const uint32_t qp = (m.qpack & 0xffu) | (31u << 8);
                auto wsec = [&](int r, int e, int c) { return c == tq ? wf(r, e, M) : wf(r, e, c); };
                add_pair(x, m.zbase, qp, [&](int i) { return (i & 2) ? c128{0.0, 0.0} : P[i]; }, wsec);
                add_pair(x, m.zbase ^ low, qp,
                         [&](int i) { return (i & 2) ? c128{ss * P[i].re, ss * P[i].im} : c128{0.0, 0.0}; }, wsec);
            } else {
                add_pair(m.x, m.zbase, m.qpack, [&](int i) { return P[i]; }, [&](int r, int e, int c) {
                    return c == tq ? wf(r, e, M) + 0.5 * wf(r, e, tq) : wf(r, e, c);
                });
                add_pair(m.x, m.zbase ^ low, m.qpack, [&](int i) { return P[i]; }, [&](int r, int e, int c) {
                    return c == tq ? -0.5 * ss * wf(r, e, tq) : 0.0;
                });
            }
        } else {
            masks.push_back({0u, 0u, 0u, (uint32_t)MASK_DIAG << 28});
            out.n_diag = F.n_diag;
            out.dz.resize(F.n_diag);
            out.dw.resize((size_t)R * F.n_diag);
            for (int n = 0; n < F.n_diag; ++n) {
                const bool top = (F.dz[n] >> tq) & 1u;
                out.dz[n] = top ? ((F.dz[n] & low) ^ low) : F.dz[n];
                for (int r = 0; r < R; ++r)
                    out.dw[(size_t)r * F.n_diag + n] = (top ? ss : 1.0) * F.dw[(size_t)r * F.n_diag + n];
            }
        }
    }
    std::stable_sort(masks.begin(), masks.end(), [](const MaskRec& a, const MaskRec& b) { return a.x < b.x; });
    out.masks = std::move(masks);
}

}  // namespace syk
