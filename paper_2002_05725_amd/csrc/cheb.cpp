// Chebyshev propagation and the reverse sweep for dF/dJ.
//
// Every propagator of the OTOC estimator (the same symmetric cut as the
// Krylov path) is a fixed polynomial: with H~ = (H - e_c)/e_h and
// v_0 = v, v_1 = H~ v, v_{n+1} = 2 H~ v_n - v_{n-1},
//   e^{-i h H} v ~ sum_n c_n v_n,  c_n = (2 - delta_n0) (-i)^n J_n(e_h h) e^{-i e_c h}
//   e^{-tau H} v ~ sum_n c_n v_n,  c_n = (2 - delta_n0) (-1)^n I_n(e_h tau) e^{-e_c tau}
// (Jacobi-Anger expansion; generating function of I_n).  F is then a fixed
// polynomial in the couplings and its derivative is exact.
//
// Reverse sweep of one step y = sum_n c_n v_n against a cotangent lambda
// (d Re<lambda|y>): Clenshaw's recurrence G_K = conj(c_K) lambda,
// G_n = conj(c_n) lambda + 2 H~ G_{n+1} - G_{n+2}, and
// G_0 = conj(c_0) lambda + H~ G_1 - G_2 is the cotangent of the step input;
// the couplings receive sum_n w_n / e_h Re <G_{n+1}| Q v_n> with w_0 = 1,
// w_n = 2, Q = dH/dJ.  States of a chain are stored every checkpoint_every
// operations and recomputed segment by segment.
#include "cheb.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace syk {

namespace {

typedef std::complex<double> C;

// With SYK_PROGRESS set in the environment, long gradient calls report each
// finished checkpoint segment of the reverse sweep on stderr (after waiting for
// the segment's device work).
void progress(const char* what, const std::string& chain, int done, int total, hipStream_t s)
{
    static const bool on = std::getenv("SYK_PROGRESS") != nullptr;
    if (!on) return;
    (void)hipStreamSynchronize(s);
    std::fprintf(stderr, "[syk] %s %s: %d/%d\n", what, chain.c_str(), done, total);
    std::fflush(stderr);
}

struct Pool {
    syk_terms_s& h;
    size_t bytes;
    void* get(const std::string& name) { return h.ws.get("cheb_" + name, bytes); }
    void* get(const std::string& name, int i) { return get(name + std::to_string(i)); }
};

// H~-products through apply_H followed by the fused recurrence kernel.
struct Stepper {
    BlockCtx& c;
    const ChebSettings& s;
    Pool& pool;
    int64_t n;   // elements per vector

    void rec(void* out, const void* w, const void* y, const void* z, const void* x, void* acc, double b, double sz,
             C cx, C ca)
    {
        cheb_rec(c.dtype, n, out, w, y, z, x, acc, b, s.e_c, sz, cx, ca, c.stream);
    }

    // out = sum_n coef_n v_n with v_n = T_n(H~) in.  With `store`, v_n is left
    // in store[n] (out may then be null); else three rotating buffers are used.
    void forward(const ChebOp& op, const void* in, void* out, const std::vector<void*>* store)
    {
        const int K = (int)op.c.size() - 1;
        void* w = pool.get("w");
        void* b[3] = {nullptr, nullptr, nullptr};
        auto vec = [&](int k) -> void* {
            if (store) return (*store)[k];
            if (!b[k % 3]) b[k % 3] = pool.get("rot", k % 3);
            return b[k % 3];
        };
        const void* v0 = in;
        if (store) {
            c.ops.copy((*store)[0], in);
            v0 = (*store)[0];
        }
        if (out) c.ops.combine(out, v0, 1, std::vector<C>{op.c[0]});
        c.apply_H(v0, w);
        void* v1 = vec(1);
        rec(v1, w, v0, nullptr, nullptr, out, 1.0 / s.e_h, 0.0, 0.0, op.c[1]);
        const void* pm = v0;   // v_{n-2}
        const void* pc = v1;   // v_{n-1}
        for (int k = 2; k <= K; ++k) {
            c.apply_H(pc, w);
            void* nv = vec(k);
            rec(nv, w, pc, pm, nullptr, out, 2.0 / s.e_h, -1.0, 0.0, op.c[k]);
            pm = pc;
            pc = nv;
        }
    }

    // lam_out = cotangent of the step input; bins += the step's coupling terms.
    // kept: the step's vectors v_0..v_K from the segment's recomputation, or
    // NULL to compute them here.
    void backward(const ChebOp& op, const void* in, const void* lam, void* lam_out, double* bins,
                  const std::vector<void*>* kept)
    {
        const int K = (int)op.c.size() - 1;
        std::vector<void*> V(K + 1), G(K + 1);
        for (int k = 1; k <= K; ++k) G[k] = pool.get("G", k);
        if (kept) {
            V = *kept;
        } else {
            for (int k = 0; k <= K; ++k) V[k] = pool.get("V", k);
            forward(op, in, nullptr, &V);
        }
        void* w = pool.get("w");
        c.ops.combine(G[K], lam, 1, std::vector<C>{std::conj(op.c[K])});
        for (int k = K - 1; k >= 0; --k) {
            c.apply_H(G[k + 1], w);
            void* out = (k == 0) ? lam_out : G[k];
            const void* z = (k + 2 <= K) ? G[k + 2] : nullptr;
            rec(out, w, G[k + 1], z, lam, nullptr, (k == 0 ? 1.0 : 2.0) / s.e_h, -1.0, std::conj(op.c[k]), 0.0);
        }
        // the bins add linearly over pairs: at most kGradMaxPairs pairs per call
        for (int k0 = 0; k0 < K; k0 += kGradMaxPairs) {
            std::vector<const void*> gp, vp;
            std::vector<double> wp;
            for (int k = k0; k < std::min(K, k0 + kGradMaxPairs); ++k) {
                gp.push_back(G[k + 1]);
                vp.push_back(V[k]);
                wp.push_back((k == 0 ? 1.0 : 2.0) / s.e_h);
            }
            grad_bins(c.h, gp, vp, wp, bins, c.stream);
        }
    }
};

void apply_op(Stepper& st, const ChebOp& op, const void* in, void* out)
{
    if (op.maj >= 0) st.c.ops.majorana(op.maj, in, out);
    else st.forward(op, in, out, nullptr);
}

// Runs `ops` on psi into out.  With ckpt_name, stores the input of every
// checkpoint_every-th operation as pool vectors ckpt_name<k>.
void chain_forward(Stepper& st, const std::vector<ChebOp>& ops, const void* psi, void* out,
                   const std::string& ckpt_name)
{
    void* x = st.pool.get("cx0");
    void* y = st.pool.get("cx1");
    st.c.ops.copy(x, psi);
    const int Ck = st.s.checkpoint_every;
    for (size_t l = 0; l < ops.size(); ++l) {
        if (!ckpt_name.empty() && l % Ck == 0) st.c.ops.copy(st.pool.get(ckpt_name, (int)(l / Ck)), x);
        apply_op(st, ops[l], x, y);
        std::swap(x, y);
    }
    st.c.ops.copy(out, x);
}

// Propagates the cotangent seed back through `ops` (checkpoints from
// chain_forward) and adds every step's coupling terms into bins.  Each segment
// between checkpoints is recomputed forward once; with keep_segment (and the
// memory for it) the Chebyshev vectors of its steps are kept from that pass,
// else every step computes them again in its reverse sweep.
void chain_backward(Stepper& st, const std::vector<ChebOp>& ops, const std::string& ckpt_name, const void* seed,
                    double* bins)
{
    const int Ck = st.s.checkpoint_every;
    const int L = (int)ops.size();
    const int K = st.s.degree;
    auto kept_name = [](int j, int k) { return "SV" + std::to_string(j) + "_" + std::to_string(k); };
    bool keep = st.s.keep_segment != 0;
    if (keep) {
        size_t need = 0;
        for (int j = 0; j < Ck; ++j)
            for (int k = 0; k <= K; ++k) {
                const size_t h = st.c.h.ws.held("cheb_" + kept_name(j, k));
                need += h >= st.pool.bytes ? 0 : st.pool.bytes;
            }
        size_t free_b = 0, total_b = 0;
        SYK_HIP(hipMemGetInfo(&free_b, &total_b));
        keep = need <= free_b / 2;
    }
    std::vector<std::vector<void*>> SV;
    if (keep) {
        SV.assign(Ck, std::vector<void*>(K + 1));
        for (int j = 0; j < Ck; ++j)
            for (int k = 0; k <= K; ++k) SV[j][k] = st.pool.get(kept_name(j, k));
    }
    void* lam = st.pool.get("lam0");
    void* lam2 = st.pool.get("lam1");
    st.c.ops.copy(lam, seed);
    const int nseg = (L + Ck - 1) / Ck;
    for (int sg = nseg - 1; sg >= 0; --sg) {
        progress("reverse sweep", ckpt_name, nseg - 1 - sg, nseg, st.c.stream);
        const int l0 = sg * Ck, l1 = std::min(L, l0 + Ck);
        // inputs of operations l0 .. l1-1 (and, kept, every step's vectors)
        st.c.ops.copy(st.pool.get("in", 0), st.pool.get(ckpt_name, sg));
        for (int l = l0; l < l1; ++l) {
            const bool last = l + 1 == l1;
            if (!keep || ops[l].maj >= 0) {
                if (!last) apply_op(st, ops[l], st.pool.get("in", l - l0), st.pool.get("in", l - l0 + 1));
            } else {
                st.forward(ops[l], st.pool.get("in", l - l0), last ? nullptr : st.pool.get("in", l - l0 + 1),
                           &SV[l - l0]);
            }
        }
        for (int l = l1 - 1; l >= l0; --l) {
            const void* in = st.pool.get("in", l - l0);
            if (ops[l].maj >= 0) st.c.ops.majorana(ops[l].maj, lam, lam2);   // chi is Hermitian
            else st.backward(ops[l], in, lam, lam2, bins, keep ? &SV[l - l0] : nullptr);
            std::swap(lam, lam2);
        }
    }
}

}  // namespace

std::vector<C> cheb_coeffs_real(double h, const ChebSettings& s)
{
    std::vector<C> c(s.degree + 1);
    const double x = s.e_h * std::fabs(h);
    const C ph = std::exp(C(0.0, -s.e_c * h));
    const C unit = (h >= 0) ? C(0.0, -1.0) : C(0.0, 1.0);   // (-i)^n, or i^n going backwards
    C p = 1.0;
    for (int n = 0; n <= s.degree; ++n) {
        c[n] = (n == 0 ? 1.0 : 2.0) * p * std::cyl_bessel_j((double)n, x) * ph;
        p *= unit;
    }
    return c;
}

std::vector<C> cheb_coeffs_imag(double tau, const ChebSettings& s)
{
    std::vector<C> c(s.degree + 1);
    const double x = s.e_h * tau;
    const double ph = std::exp(-s.e_c * tau);
    for (int n = 0; n <= s.degree; ++n)
        c[n] = (n == 0 ? 1.0 : 2.0) * ((n & 1) ? -1.0 : 1.0) * std::cyl_bessel_i((double)n, x) * ph;
    return c;
}

// Chains (W = chi_i, V = chi_j, P(s) = rho^s, U = e^{-iHt}):
//   A psi = P(1/8) U^dag W U P(1/4) V P(1/8) psi
//   B psi = P(1/8) V P(1/4) U^dag W U P(1/8) psi   (= A^dag psi)
//   u     = P(1/2) psi
OtocChains otoc_chains(int i, int j, double beta, double t, const ChebSettings& s)
{
    const int nt = (int)std::llround(t / s.dt);
    require(std::fabs(nt * s.dt - t) <= 1e-9 * std::max(1.0, t), "t_star must be a multiple of dt");
    auto imag = [&](std::vector<ChebOp>& ch, double frac) {
        if (beta == 0.0) return;
        for (int k = 0; k < s.tau_steps; ++k) ch.push_back({-1, cheb_coeffs_imag(beta * frac / s.tau_steps, s)});
    };
    auto real = [&](std::vector<ChebOp>& ch, double sign) {
        for (int k = 0; k < nt; ++k) ch.push_back({-1, cheb_coeffs_real(sign * s.dt, s)});
    };
    OtocChains o;
    imag(o.A, 1.0 / 8);
    o.A.push_back({j, {}});
    imag(o.A, 1.0 / 4);
    real(o.A, +1.0);
    o.A.push_back({i, {}});
    real(o.A, -1.0);
    imag(o.A, 1.0 / 8);

    imag(o.B, 1.0 / 8);
    real(o.B, +1.0);
    o.B.push_back({i, {}});
    real(o.B, -1.0);
    imag(o.B, 1.0 / 4);
    o.B.push_back({j, {}});
    imag(o.B, 1.0 / 8);

    imag(o.U, 1.0 / 2);
    return o;
}

void cheb_otoc(BlockCtx& c, int i, int j, double beta, double t, const ChebSettings& s, const void* psi0, double* F,
               double* grad)
{
    require(c.nvec == 1 && c.dtype == SYK_C128, "Chebyshev OTOC: one complex128 column");
    require(s.degree >= 2 && s.degree <= 256, "Chebyshev degree must be in [2, 256]");
    require(s.e_h > 0 && std::isfinite(s.e_h) && std::isfinite(s.e_c), "Chebyshev interval must be finite, e_h > 0");
    require(s.dt > 0 && s.tau_steps >= 1 && s.checkpoint_every >= 1, "bad Chebyshev step settings");
    const OtocChains ch = otoc_chains(i, j, beta, t, s);
    Pool pool{c.h, c.ops.vec_bytes()};
    Stepper st{c, s, pool, c.dim()};
    const bool g = grad != nullptr;
    void* A = pool.get("A");
    void* B = pool.get("B");
    void* u = pool.get("u");
    chain_forward(st, ch.A, psi0, A, g ? "ckA" : "");
    progress("forward", "A", 1, 1, c.stream);
    chain_forward(st, ch.B, psi0, B, g ? "ckB" : "");
    progress("forward", "B", 1, 1, c.stream);
    chain_forward(st, ch.U, psi0, u, g ? "ckU" : "");
    const double Z = c.ops.norm2(u)[0];
    const double num = c.ops.multidot(B, 1, A)[0].real();
    require(std::isfinite(Z) && Z > 0, "Chebyshev OTOC: non-positive <psi|rho|psi>");
    const double f = num / Z;
    *F = f;
    if (!g) return;

    const TermTables& T = c.h.host;
    double* bins = (double*)c.h.ws.get("cheb_bins", T.n_bins * 2 * sizeof(double));
    SYK_HIP(hipMemsetAsync(bins, 0, T.n_bins * 2 * sizeof(double), c.stream));
    void* seed = pool.get("seed");
    // d(num)/dA = B, d(num)/dB = A (Re <B|A> is symmetric), dZ/du = 2u; F = num/Z.
    c.ops.combine(seed, B, 1, std::vector<C>{1.0 / Z});
    chain_backward(st, ch.A, "ckA", seed, bins);
    c.ops.combine(seed, A, 1, std::vector<C>{1.0 / Z});
    chain_backward(st, ch.B, "ckB", seed, bins);
    if (!ch.U.empty()) {
        c.ops.combine(seed, u, 1, std::vector<C>{-2.0 * f / Z});
        chain_backward(st, ch.U, "ckU", seed, bins);
    }
    std::vector<double> hb(T.n_bins * 2);
    SYK_HIP(hipMemcpyAsync(hb.data(), bins, hb.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    SYK_HIP(hipStreamSynchronize(c.stream));
    couplings_from_bins(T, hb.data(), grad);
}

}  // namespace syk
