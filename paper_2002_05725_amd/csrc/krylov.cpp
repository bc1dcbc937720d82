// Lanczos propagation (SI "Krylov subspace methods"): e^{zH} psi is replaced by
// ||psi|| V e^{zT} e_1, with V an orthonormal basis of span{psi, H psi, ...}
// (m vectors) and T = V^dag H V the m x m tridiagonal projection.  The basis
// is orthogonalised against all previous vectors with two passes of classical
// Gram-Schmidt; inner products are FP64 on the device, T and its exponential
// are FP64 on the host.
#include "krylov.hpp"

#include <algorithm>

#include <cmath>

namespace syk {

BlockCtx::BlockCtx(syk_terms_s& h_, syk_dtype dt, int nvec_, const int32_t* real, hipStream_t s, int sector)
    : h(h_), dtype(dt), nvec(nvec_), real_of_col(real), stream(s), sector0(sector),
      Hact(sector < 0 ? &h_.H : &sector_ham(h_, sector)), plan(plan_for(h_, Hact->M, nvec_, dt)),
      ops(h_, dt, (int64_t)1 << Hact->M, nvec_, s)
{
}

void BlockCtx::apply_H(const void* in, void* out) { launch_apply_h(*Hact, dtype, nvec, real_of_col, in, out, plan, stream); }

void BlockCtx::at(int s)
{
    if (sector0 >= 0) Hact = &sector_ham(h, s);
}

void BlockCtx::majorana(int a, int s_in, const void* in, void* out)
{
    if (s_in < 0) ops.majorana(a, in, out);
    else ops.majorana_sector(a, Hact->M, s_in, in, out);
}

// Cyclic Jacobi rotations on the dense n x n matrix (O(n^3) per sweep, a few
// sweeps).  Converges to full FP64 accuracy.
void symmetric_eig(int n, std::vector<double>& a, std::vector<double>& w, std::vector<double>& v)
{
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double x = a[(size_t)i * n + j] * a[(size_t)i * n + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-34 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {   // columns p, q
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = cs * akp - sn * akq;
                    a[(size_t)k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {   // rows p, q
                    const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = cs * apk - sn * aqk;
                    a[(size_t)q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = cs * vkp - sn * vkq;
                    v[(size_t)k * n + q] = sn * vkp + cs * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
}

// Builds the Krylov basis of psi (V, m vectors in the workspace) and the
// tridiagonal projection per column.
LanczosBasis lanczos_build(BlockCtx& c, const void* psi, int m)
{
    const int B = c.nvec;
    VecOps& ops = c.ops;
    const size_t vb = ops.vec_bytes();
    LanczosBasis L;
    L.m = m;
    L.V = (char*)c.h.ws.get("krylov_V", vb * (size_t)m);
    void* w = c.h.ws.get("krylov_w", vb);
    char* V = L.V;

    std::vector<double> nrm2 = ops.norm2(psi);
    L.nrm.assign(B, 0.0);
    std::vector<double> inv(B);
    for (int b = 0; b < B; ++b) {
        if (!std::isfinite(nrm2[b])) throw Error(SYK_EBREAKDOWN, "non-finite norm in Krylov step");
        L.nrm[b] = std::sqrt(nrm2[b]);
        inv[b] = L.nrm[b] > 0 ? 1.0 / L.nrm[b] : 0.0;
    }
    ops.scale(V, psi, inv);

    L.alpha.assign((size_t)m * B, 0.0);
    L.beta.assign((size_t)m * B, 0.0);
    L.kdim.assign(B, m);
    std::vector<double>& alpha = L.alpha;
    std::vector<double>& beta = L.beta;
    std::vector<int>& kdim = L.kdim;
    std::vector<double> scale(B, 0.0);
    for (int j = 0; j < m; ++j) {
        c.apply_H(V + (size_t)j * vb, w);
        std::vector<zd> c1 = ops.multidot(V, j + 1, w);
        ops.update(w, V, j + 1, c1, false);
        std::vector<zd> c2 = ops.multidot(V, j + 1, w);
        std::vector<double> b2 = ops.update(w, V, j + 1, c2, true);
        std::vector<double> f(B, 0.0);
        for (int b = 0; b < B; ++b) {
            const double a = (c1[(size_t)j * B + b] + c2[(size_t)j * B + b]).real();
            const double bt = std::sqrt(b2[b]);
            if (!std::isfinite(a) || !std::isfinite(bt)) throw Error(SYK_EBREAKDOWN, "non-finite Lanczos coefficient");
            alpha[(size_t)j * B + b] = a;
            beta[(size_t)j * B + b] = bt;
            if (j >= kdim[b]) continue;   // column already invariant: its basis stays zero
            scale[b] = std::max(scale[b], std::fabs(a) + (j > 0 ? beta[(size_t)(j - 1) * B + b] : 0.0));
            if (j < m - 1) {
                if (bt <= 1e-13 * scale[b] || L.nrm[b] == 0.0) {
                    kdim[b] = j + 1;          // invariant subspace: T is exact
                } else {
                    f[b] = 1.0 / bt;
                }
            }
        }
        if (j < m - 1) ops.scale(V + (size_t)(j + 1) * vb, w, f);
    }
    return L;
}

void ritz_values(const LanczosBasis& L, int col, int nvec, std::vector<double>& ev, std::vector<double>& S)
{
    const int k = L.kdim[col];
    std::vector<double> T((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) {
        T[(size_t)i * k + i] = L.alpha[(size_t)i * nvec + col];
        if (i + 1 < k) T[(size_t)i * k + i + 1] = T[(size_t)(i + 1) * k + i] = L.beta[(size_t)i * nvec + col];
    }
    symmetric_eig(k, T, ev, S);
}

void krylov_step(BlockCtx& c, void* psi, std::complex<double> z, int m, KrylovStats& st)
{
    const int B = c.nvec;
    LanczosBasis L = lanczos_build(c, psi, m);
    const std::vector<double>& beta = L.beta;
    const std::vector<int>& kdim = L.kdim;
    const std::vector<double>& nrm = L.nrm;
    char* V = L.V;
    VecOps& ops = c.ops;

    // Per column: y = ||psi|| V S e^{z Lambda} S^T e_1.
    std::vector<zd> coef((size_t)m * B, zd(0.0, 0.0));
    if (st.err.size() != (size_t)B) st.err.assign(B, 0.0);
    for (int b = 0; b < B; ++b) {
        const int k = kdim[b];
        std::vector<double> ev, S;
        ritz_values(L, b, B, ev, S);
        std::vector<zd> g(k);
        for (int l = 0; l < k; ++l) g[l] = std::exp(z * ev[l]) * S[(size_t)0 * k + l];
        for (int i = 0; i < k; ++i) {
            zd s(0.0, 0.0);
            for (int l = 0; l < k; ++l) s += S[(size_t)i * k + l] * g[l];
            coef[(size_t)i * B + b] = nrm[b] * s;
        }
        if (k == m) {
            const double e = beta[(size_t)(m - 1) * B + b] * std::abs(coef[(size_t)(m - 1) * B + b]);
            st.err[b] = std::max(st.err[b], e);
        }
    }
    ops.combine(psi, V, m, coef);
    ++st.steps;
}

void lanczos_extremes(BlockCtx& c, const void* psi, int m, double* emin, double* emax)
{
    require(c.nvec == 1, "spectrum bounds: one column");
    LanczosBasis L = lanczos_build(c, psi, m);
    std::vector<double> ev, S;
    ritz_values(L, 0, 1, ev, S);
    *emin = ev[0];
    *emax = ev[0];
    for (double e : ev) {
        *emin = std::min(*emin, e);
        *emax = std::max(*emax, e);
    }
}

int lowest_eigenvalues(BlockCtx& c, const void* psi, int m, int k, double* ev_out, double* res_out)
{
    require(c.nvec == 1, "eigenvalues: one column");
    LanczosBasis L = lanczos_build(c, psi, m);
    std::vector<double> ev, S;
    ritz_values(L, 0, 1, ev, S);
    const int kd = L.kdim[0];
    std::vector<int> ord(kd);
    for (int i = 0; i < kd; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return ev[a] < ev[b]; });
    // beta of the step that would extend the basis; 0 when the space is invariant
    const double bl = (kd == m) ? L.beta[(size_t)(m - 1)] : 0.0;
    const int n = std::min(k, kd);
    for (int i = 0; i < n; ++i) {
        ev_out[i] = ev[ord[i]];
        if (res_out) res_out[i] = bl * std::fabs(S[(size_t)(kd - 1) * kd + ord[i]]);
    }
    return n;
}

void krylov_propagate(BlockCtx& c, void* psi, std::complex<double> z, double total, double step, int m,
                      KrylovStats& st)
{
    if (total == 0.0) return;
    require(total > 0 && step > 0, "propagation length and step must be positive");
    const int n = std::max(1, (int)std::ceil(total / step - 1e-9));
    const double h = total / n;
    for (int i = 0; i < n; ++i) krylov_step(c, psi, z * h, m, st);
}

}  // namespace syk
