// Lanczos propagation (SI "Krylov subspace methods"): e^{zH} psi is replaced by
// ||psi|| V e^{zT} e_1, with V an orthonormal basis of span{psi, H psi, ...}
// (m vectors) and T = V^dag H V the m x m tridiagonal projection.  The basis
// is orthogonalised against all previous vectors with two passes of classical
// Gram-Schmidt; inner products are FP64 on the device, T (tridiagonal QR for
// its eigen-decomposition) and its exponential are FP64 on the host.  Up to 16 basis vectors the first pass's update and
// the second pass's projection share one sweep over the basis.  The
// projections, alpha, beta and the invariant-subspace test stay on the device
// for the whole build (no host round trip per iteration); the host reads them
// once at the end.
#include "krylov.hpp"
#include "tridiag_eig.hpp"

#include <algorithm>

#include <cmath>
#include <cstdio>
#include <cstdlib>

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
    // Device scalars: alpha, beta [m][B], then scale, nrm, f [B]; kdim [B] and
    // the error flag.  A column whose subspace became invariant keeps f = 0,
    // so its later basis vectors are zero.
    const size_t nB = (size_t)B;
    double* dd = (double*)c.h.ws.get("lz_dbl", (2 * (size_t)m + 3) * nB * sizeof(double));
    int* di = (int*)c.h.ws.get("lz_int", (nB + 1) * sizeof(int));
    {
        std::vector<double> h((2 * (size_t)m + 3) * nB, 0.0);
        std::copy(L.nrm.begin(), L.nrm.end(), h.begin() + (2 * (size_t)m + 1) * nB);
        ops.to_device(dd, h.data(), h.size() * sizeof(double));
        std::vector<int> hi(nB + 1, m);
        hi[nB] = 0;
        ops.to_device(di, hi.data(), hi.size() * sizeof(int));
    }
    LanczosScalars z{dd, dd + (size_t)m * nB, di, dd + 2 * (size_t)m * nB, dd + (2 * (size_t)m + 1) * nB,
                     dd + (2 * (size_t)m + 2) * nB, di + nB};
    // projections of up to m basis vectors (sized once: no reallocation inside the loop)
    const size_t proj_bytes = (size_t)std::max(m, VecOps::kFusedMax) * nB * 2 * sizeof(double);
    c.h.ws.get("gs_c1", proj_bytes);
    c.h.ws.get("gs_c2", proj_bytes);
    for (int j = 0; j < m; ++j) {
        c.apply_H(V + (size_t)j * vb, w);
        const double* d1 = ops.multidot_dev(V, j + 1, w, "gs_c1");
        const double* d2;
        if (j + 1 <= VecOps::kFusedMax) {
            d2 = ops.update_dot(w, V, j + 1, d1, "gs_c2");
        } else {
            ops.update_dev_norm(w, V, j + 1, d1, false);
            d2 = ops.multidot_dev(V, j + 1, w, "gs_c2");
        }
        const double* wn = ops.update_dev_norm(w, V, j + 1, d2, true);
        ops.lanczos_coef(d1, d2, wn, j, m, z);
        if (j < m - 1) ops.scale_dev(V + (size_t)(j + 1) * vb, w, z.f);
    }
    ops.to_host(L.alpha.data(), z.alpha, L.alpha.size() * sizeof(double));
    ops.to_host(L.beta.data(), z.beta, L.beta.size() * sizeof(double));
    std::vector<int> hi(nB + 1);
    ops.to_host(hi.data(), di, hi.size() * sizeof(int));
    if (hi[nB] != 0) throw Error(SYK_EBREAKDOWN, "non-finite Lanczos coefficient");
    std::copy(hi.begin(), hi.begin() + nB, L.kdim.begin());
    return L;
}

void ritz_values(const LanczosBasis& L, int col, int nvec, std::vector<double>& ev, std::vector<double>& S)
{
    const int k = L.kdim[col];
    std::vector<double> d(k), e(k > 1 ? k - 1 : 0);
    for (int i = 0; i < k; ++i) {
        d[i] = L.alpha[(size_t)i * nvec + col];
        if (i + 1 < k) e[i] = L.beta[(size_t)i * nvec + col];
    }
    try {
        tridiag_eig(k, d, e, ev, S);
    } catch (const std::runtime_error& x) {
        throw Error(SYK_EBREAKDOWN, x.what());
    }
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
    // With SYK_PROGRESS set in the environment, every finished step is reported
    // on stderr (each step has already read its Lanczos scalars back).
    static const bool report = std::getenv("SYK_PROGRESS") != nullptr;
    for (int i = 0; i < n; ++i) {
        krylov_step(c, psi, z * h, m, st);
        if (report) {
            std::fprintf(stderr, "[syk] Krylov step %d/%d of exp((%g%+gi) H), %d column(s)\n", i + 1, n, h * z.real(),
                         h * z.imag(), c.nvec);
            std::fflush(stderr);
        }
    }
}

}  // namespace syk
