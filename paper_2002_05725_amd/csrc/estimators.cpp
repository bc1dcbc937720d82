// Typical-state estimators of the two-point functions (main text Eq. 2-3), the
// regularized OTOC (main text Eq. 4) and the unregularized OTOC (SI section
// "Unregularized OTOCs"), with the trace replaced by a Gaussian random state
// as in the SI section "Disorder averaging".
#include "estimators.hpp"

#include <cmath>

namespace syk {

namespace {

const std::complex<double> kReal(0.0, -1.0);   // e^{-iHt}: z = -i
const std::complex<double> kImag(-1.0, 0.0);   // e^{-tau H}: z = -1

void check_times(const double* t, int nt)
{
    require(t != nullptr && nt >= 1, "need at least one time");
    for (int k = 0; k < nt; ++k) {
        require(std::isfinite(t[k]) && t[k] >= 0.0, "times must be finite and >= 0");
        require(k == 0 || t[k] >= t[k - 1], "times must be ascending");
    }
}

}  // namespace

void two_point(BlockCtx& c, int i, double beta, const double* t, int nt, const void* psi0,
               const syk_krylov_opts& o, double* G, double* Z)
{
    check_times(t, nt);
    const int B = c.nvec;
    const int s0 = c.sector0, s1 = BlockCtx::other(s0);   // sectors of psi and of chi psi
    const size_t vb = c.ops.vec_bytes();
    void* a = c.h.ws.get("est_a", vb);
    void* b = c.h.ws.get("est_b", vb);
    void* tmp = c.h.ws.get("est_tmp", vb);
    KrylovStats st;
    c.ops.copy(a, psi0);
    c.at(s0);
    krylov_propagate(c, a, kImag, beta / 2, o.tau_step, o.m, st);           // rho^{1/2} psi
    std::vector<double> z = c.ops.norm2(a);
    c.majorana(i, s0, a, b);                                                   // chi_i rho^{1/2} psi
    double tcur = 0.0;
    for (int k = 0; k < nt; ++k) {
        c.at(s0);
        krylov_propagate(c, a, kReal, t[k] - tcur, o.dt, o.m, st);
        c.at(s1);
        krylov_propagate(c, b, kReal, t[k] - tcur, o.dt, o.m, st);
        tcur = t[k];
        c.majorana(i, s1, b, tmp);
        std::vector<zd> d = c.ops.multidot(a, 1, tmp);                          // <U a | chi U b>
        for (int col = 0; col < B; ++col) {
            G[((size_t)k * B + col) * 2] = d[col].real() / z[col];
            G[((size_t)k * B + col) * 2 + 1] = d[col].imag() / z[col];
        }
    }
    if (Z)
        for (int col = 0; col < B; ++col) Z[col] = z[col];
    if (o.tol > 0)
        for (double e : st.err)
            if (e > o.tol) throw Error(SYK_ENOTCONVERGED, "Krylov error estimate above tolerance");
}

void otoc(BlockCtx& c, int i, int j, double beta, const double* t, int nt, const void* psi0,
          const syk_krylov_opts& o, double* F, double* F_im, double* Z)
{
    check_times(t, nt);
    const int B = c.nvec;
    const int s0 = c.sector0, s1 = BlockCtx::other(s0);   // sectors of psi and of chi psi
    const size_t vb = c.ops.vec_bytes();
    void* fa = c.h.ws.get("est_a", vb);     // U(t) rho^{1/8} psi                     (s0)
    void* fb = c.h.ws.get("est_b", vb);     // U(t) rho^{1/4} chi_j rho^{1/8} psi     (s1)
    void* x = c.h.ws.get("est_x", vb);
    void* y = c.h.ws.get("est_y", vb);
    KrylovStats st;

    c.at(s0);
    c.ops.copy(x, psi0);
    krylov_propagate(c, x, kImag, beta / 2, o.tau_step, o.m, st);
    const std::vector<double> z = c.ops.norm2(x);                              // <psi|rho|psi>

    c.ops.copy(fa, psi0);
    krylov_propagate(c, fa, kImag, beta / 8, o.tau_step, o.m, st);
    c.majorana(j, s0, fa, fb);
    c.at(s1);
    krylov_propagate(c, fb, kImag, beta / 4, o.tau_step, o.m, st);

    double tcur = 0.0;
    for (int k = 0; k < nt; ++k) {
        c.at(s0);
        krylov_propagate(c, fa, kReal, t[k] - tcur, o.dt, o.m, st);
        c.at(s1);
        krylov_propagate(c, fb, kReal, t[k] - tcur, o.dt, o.m, st);
        tcur = t[k];
        // A psi = rho^{1/8} U^dag chi_i U [rho^{1/4} chi_j rho^{1/8} psi]
        c.majorana(i, s1, fb, x);
        c.at(s0);
        krylov_propagate(c, x, std::conj(kReal), t[k], o.dt, o.m, st);
        krylov_propagate(c, x, kImag, beta / 8, o.tau_step, o.m, st);
        // A^dag psi = rho^{1/8} chi_j rho^{1/4} U^dag chi_i U [rho^{1/8} psi]
        c.majorana(i, s0, fa, y);
        c.at(s1);
        krylov_propagate(c, y, std::conj(kReal), t[k], o.dt, o.m, st);
        krylov_propagate(c, y, kImag, beta / 4, o.tau_step, o.m, st);
        void* y2 = c.h.ws.get("est_tmp", vb);
        c.majorana(j, s1, y, y2);
        c.at(s0);
        krylov_propagate(c, y2, kImag, beta / 8, o.tau_step, o.m, st);
        std::vector<zd> d = c.ops.multidot(y2, 1, x);                           // <A^dag psi | A psi>
        for (int col = 0; col < B; ++col) {
            F[(size_t)k * B + col] = d[col].real() / z[col];
            if (F_im) F_im[(size_t)k * B + col] = d[col].imag() / z[col];
        }
    }
    if (Z)
        for (int col = 0; col < B; ++col) Z[col] = z[col];
    if (o.tol > 0)
        for (double e : st.err)
            if (e > o.tol) throw Error(SYK_ENOTCONVERGED, "Krylov error estimate above tolerance");
}

void otoc_unregularized(BlockCtx& c, int i, int j, double beta, const double* t, int nt, const void* psi0,
                        const syk_krylov_opts& o, double* F, double* F_im, double* Z)
{
    check_times(t, nt);
    const int B = c.nvec;
    const int s0 = c.sector0, s1 = BlockCtx::other(s0);   // sectors of psi and of chi psi
    const size_t vb = c.ops.vec_bytes();
    void* uphi = c.h.ws.get("est_a", vb);   // U(t) phi, phi = rho^{1/2} psi  (s0)
    void* uvp = c.h.ws.get("est_b", vb);    // U(t) V phi                     (s1)
    void* x = c.h.ws.get("est_x", vb);
    void* y = c.h.ws.get("est_y", vb);
    void* y2 = c.h.ws.get("est_tmp", vb);
    KrylovStats st;

    c.at(s0);
    c.ops.copy(uphi, psi0);
    krylov_propagate(c, uphi, kImag, beta / 2, o.tau_step, o.m, st);
    const std::vector<double> z = c.ops.norm2(uphi);                           // <psi|rho|psi>
    c.majorana(j, s0, uphi, uvp);

    double tcur = 0.0;
    for (int k = 0; k < nt; ++k) {
        c.at(s0);
        krylov_propagate(c, uphi, kReal, t[k] - tcur, o.dt, o.m, st);
        c.at(s1);
        krylov_propagate(c, uvp, kReal, t[k] - tcur, o.dt, o.m, st);
        tcur = t[k];
        // W V phi = U^dag chi_i U [V phi]
        c.majorana(i, s1, uvp, x);
        c.at(s0);
        krylov_propagate(c, x, std::conj(kReal), t[k], o.dt, o.m, st);
        // V W phi = chi_j U^dag chi_i U [phi]
        c.majorana(i, s0, uphi, y);
        c.at(s1);
        krylov_propagate(c, y, std::conj(kReal), t[k], o.dt, o.m, st);
        c.majorana(j, s1, y, y2);
        std::vector<zd> d = c.ops.multidot(y2, 1, x);                           // <V W phi | W V phi>
        for (int col = 0; col < B; ++col) {
            F[(size_t)k * B + col] = d[col].real() / z[col];
            if (F_im) F_im[(size_t)k * B + col] = d[col].imag() / z[col];
        }
    }
    if (Z)
        for (int col = 0; col < B; ++col) Z[col] = z[col];
    if (o.tol > 0)
        for (double e : st.err)
            if (e > o.tol) throw Error(SYK_ENOTCONVERGED, "Krylov error estimate above tolerance");
}

void imag_two_point(BlockCtx& c, int i, double beta, const double* tau, int ntau, const void* psi0,
                    const syk_krylov_opts& o, double* G, double* Z)
{
    check_times(tau, ntau);
    require(tau[ntau - 1] <= beta, "imaginary times must lie in [0, beta]");
    const int B = c.nvec;
    const int s0 = c.sector0, s1 = BlockCtx::other(s0);   // sectors of psi and of chi psi
    const size_t vb = c.ops.vec_bytes();
    void* u = c.h.ws.get("est_a", vb);      // e^{-(beta - tau) H / 2} psi, tau descending  (s0)
    void* w = c.h.ws.get("est_b", vb);
    KrylovStats st;

    c.at(s0);
    c.ops.copy(w, psi0);
    krylov_propagate(c, w, kImag, beta / 2, o.tau_step, o.m, st);
    const std::vector<double> z = c.ops.norm2(w);                              // <psi|rho|psi>

    c.ops.copy(u, psi0);
    double done = 0.0;   // imaginary time already applied to u
    for (int k = ntau - 1; k >= 0; --k) {
        const double need = (beta - tau[k]) / 2;
        c.at(s0);
        krylov_propagate(c, u, kImag, need - done, o.tau_step, o.m, st);
        done = need;
        c.majorana(i, s0, u, w);
        c.at(s1);
        krylov_propagate(c, w, kImag, tau[k] / 2, o.tau_step, o.m, st);
        const std::vector<double> n2 = c.ops.norm2(w);
        for (int col = 0; col < B; ++col) G[(size_t)k * B + col] = n2[col] / z[col];
    }
    if (Z)
        for (int col = 0; col < B; ++col) Z[col] = z[col];
    if (o.tol > 0)
        for (double e : st.err)
            if (e > o.tol) throw Error(SYK_ENOTCONVERGED, "Krylov error estimate above tolerance");
}

}  // namespace syk
