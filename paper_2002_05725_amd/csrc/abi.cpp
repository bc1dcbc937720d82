// C-ABI entry points: argument validation, error capture, dispatch.
#include <cmath>
#include <cstring>
#include <string>

#include "cheb.hpp"
#include "estimators.hpp"
#include "timing.hpp"

using namespace syk;

namespace {

thread_local std::string g_last_error;

template <typename F>
syk_status guard(F&& f)
{
    try {
        f();
        g_last_error.clear();
        return SYK_OK;
    } catch (const Error& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return SYK_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SYK_EINVAL;
    } catch (...) {
        g_last_error = "unknown error";
        return SYK_EINVAL;
    }
}

void check_handle(syk_terms t) { require(t != nullptr && t->H.masks != nullptr, "invalid syk_terms handle"); }

void check_dtype(syk_dtype d) { require(d == SYK_C128 || d == SYK_C64, "dtype must be SYK_C128 or SYK_C64"); }

void check_block(syk_terms t, int nvec, const int32_t* real)
{
    require(nvec >= 1, "nvec must be >= 1");
    if (real)
        for (int c = 0; c < nvec; ++c)
            require(real[c] >= 0 && real[c] < t->host.n_real, "real_of_col entry out of range");
}

void check_sector(syk_terms t, int sector)
{
    if (!t) throw Error(SYK_EINVAL, "handle is NULL");
    require(sector == 0 || sector == 1, "sector must be 0 or 1");
    require(t->H.N >= 6, "parity sectors need N >= 6");
}

void check_ptr(const void* p, const char* what)
{
    require(p != nullptr, std::string(what) + " is NULL");
    require(((uintptr_t)p & 15u) == 0, std::string(what) + " is not 16-byte aligned");
}

void check_no_overlap(const void* a, const void* b, size_t bytes)
{
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    require(x + bytes <= y || y + bytes <= x, "input and output buffers overlap");
}

syk_krylov_opts check_opts(const syk_krylov_opts* o)
{
    require(o != nullptr, "Krylov options are NULL");
    require(o->m >= 2 && o->m <= 64, "Krylov m must be in [2, 64]");
    require(std::isfinite(o->dt) && o->dt > 0, "Krylov dt must be > 0");
    require(std::isfinite(o->tau_step) && o->tau_step > 0, "Krylov tau_step must be > 0");
    return *o;
}

template <typename T>
void upload(DevBuf& b, const std::vector<T>& v)
{
    b.ensure(std::max<size_t>(v.size() * sizeof(T), 16));
    if (!v.empty()) SYK_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

template <typename T>
std::vector<T> narrow(const std::vector<T>& v) { return v; }

std::vector<c64> to_c64(const std::vector<c128>& v)
{
    std::vector<c64> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = {(float)v[i].re, (float)v[i].im};
    return o;
}

std::vector<float> to_f32(const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); }

}  // namespace

namespace syk {

// Device copies of a table set and the kernels' view of them.
void make_device(const TermTables& T, DeviceTerms& d, HamiltonianDev& H)
{
    upload(d.masks, T.masks);
    upload(d.tab4_d, T.tab4);
    upload(d.tab4_f, to_c64(T.tab4));
    upload(d.qinfo, T.qinfo);
    upload(d.phi2_d, T.phi2);
    upload(d.phi2_f, to_c64(T.phi2));
    upload(d.w2_d, T.w2);
    upload(d.w2_f, to_f32(T.w2));
    upload(d.dz, T.dz);
    upload(d.dw_d, T.dw);
    upload(d.dw_f, to_f32(T.dw));
    H.N = T.N;
    H.M = T.M;
    H.n_real = T.n_real;
    H.n_diag = T.n_diag;
    H.masks = d.masks.as<MaskRec>();
    H.tab4_d = d.tab4_d.as<c128>();
    H.tab4_f = d.tab4_f.as<c64>();
    H.qinfo = d.qinfo.as<uint32_t>();
    H.phi2_d = d.phi2_d.as<c128>();
    H.phi2_f = d.phi2_f.as<c64>();
    H.w2_d = d.w2_d.as<double>();
    H.w2_f = d.w2_f.as<float>();
    H.dz = d.dz.as<uint32_t>();
    H.dw_d = d.dw_d.as<double>();
    H.dw_f = d.dw_f.as<float>();
    H.host_masks = &T.masks;
    H.bin_off = &T.bin_off;
}

const HamiltonianDev& sector_ham(syk_terms_s& h, int s)
{
    require(s == 0 || s == 1, "sector must be 0 or 1");
    auto& p = h.sectors[s];
    if (!p) {
        std::unique_ptr<syk_terms_s::Sector> n(new syk_terms_s::Sector());
        build_sector_tables(h.host, s, n->host);
        make_device(n->host, n->dev, n->H);
        p = std::move(n);
    }
    return p->H;
}

}  // namespace syk

extern "C" {

const char* syk_last_error(void) { return g_last_error.c_str(); }

int syk_version(void) { return 100; }


syk_status syk_build_terms(int N, int n_real, const double* J, syk_terms* out)
{
    return guard([&] {
        require(out != nullptr, "out is NULL");
        *out = nullptr;
        require(N >= 4 && N <= 60 && N % 2 == 0, "N must be even with 4 <= N <= 60");
        require(n_real >= 1, "n_real must be >= 1");
        require(J != nullptr, "J is NULL");
        const int64_t nq = (int64_t)N * (N - 1) * (N - 2) * (N - 3) / 24;
        for (int64_t k = 0; k < nq * n_real; ++k) require(std::isfinite(J[k]), "J holds a non-finite value");
        std::unique_ptr<syk_terms_s> h(new syk_terms_s());
        SYK_HIP(hipGetDevice(&h->device));
        build_tables(N, n_real, J, h->host);
        make_device(h->host, h->dev, h->H);
        *out = h.release();
    });
}

syk_status syk_destroy_terms(syk_terms t)
{
    return guard([&] { delete t; });
}

syk_status syk_terms_info(syk_terms t, int* N, int* n_real, int64_t* dim, int64_t* n_terms, int64_t* n_masks)
{
    return guard([&] {
        check_handle(t);
        if (N) *N = t->H.N;
        if (n_real) *n_real = t->H.n_real;
        if (dim) *dim = (int64_t)1 << t->H.M;
        if (n_terms) *n_terms = t->host.n_terms;
        if (n_masks) *n_masks = (int64_t)t->host.masks.size();
    });
}

static void apply_impl(syk_terms t, syk_dtype dtype, int sector, int nvec, const int32_t* real_of_col,
                       const void* psi, void* out, hipStream_t stream)
{
    check_handle(t);
    check_dtype(dtype);
    check_block(t, nvec, real_of_col);
    check_ptr(psi, "psi");
    check_ptr(out, "out");
    const HamiltonianDev& H = sector < 0 ? t->H : sector_ham(*t, sector);
    const size_t bytes = ((size_t)1 << H.M) * nvec * elem_bytes(dtype);
    check_no_overlap(psi, out, bytes);
    ApplyPlan P = plan_for(*t, H.M, nvec, dtype);
    launch_apply_h(H, dtype, nvec, real_of_col, psi, out, P, stream);
}

syk_status syk_apply_H(syk_terms t, syk_dtype dtype, int nvec, const int32_t* real_of_col, const void* psi,
                       void* out, hipStream_t stream)
{
    return guard([&] { apply_impl(t, dtype, -1, nvec, real_of_col, psi, out, stream); });
}

syk_status syk_apply_H_noalloc(syk_terms t, syk_dtype dtype, int nvec, const int32_t* real_of_col, const void* psi,
                               void* out, hipStream_t stream)
{
    return guard([&] {
        check_handle(t);
        check_dtype(dtype);
        check_block(t, nvec, real_of_col);
        check_ptr(psi, "psi");
        check_ptr(out, "out");
        const size_t bytes = ((size_t)1 << t->H.M) * nvec * elem_bytes(dtype);
        check_no_overlap(psi, out, bytes);
        const ApplyPlan P = plan_for(*t, t->H.M, nvec, dtype);
        launch_apply_h_noalloc(t->H, t->device, dtype, nvec, real_of_col, psi, out, P, stream);
    });
}

syk_status syk_apply_H_sector(syk_terms t, syk_dtype dtype, int sector, int nvec, const int32_t* real_of_col,
                              const void* psi, void* out, hipStream_t stream)
{
    return guard([&] {
        check_sector(t, sector);
        apply_impl(t, dtype, sector, nvec, real_of_col, psi, out, stream);
    });
}

syk_status syk_set_apply_tuning(syk_terms t, int tile_bits, int xcd_remap, int cols_per_group)
{
    return guard([&] {
        check_handle(t);
        require(tile_bits >= 0 && tile_bits <= 11, "tile_bits must be in [0, 11]");
        require(xcd_remap == 0 || xcd_remap == 1, "xcd_remap must be 0 or 1");
        require(cols_per_group >= 0 && cols_per_group <= 2, "cols_per_group must be 0, 1 or 2");
        const bool o_tuned = t->tuned;
        const int o_tb = t->tune_tile_bits, o_x = t->tune_xcd, o_c = t->tune_cols;
        t->tuned = true;
        t->tune_tile_bits = tile_bits;
        t->tune_xcd = xcd_remap;
        t->tune_cols = cols_per_group;
        try {
            (void)plan_for(*t, 1, SYK_C128);   // reject shapes that cannot launch
            (void)plan_for(*t, 1, SYK_C64);
        } catch (...) {
            t->tuned = o_tuned;
            t->tune_tile_bits = o_tb;
            t->tune_xcd = o_x;
            t->tune_cols = o_c;
            throw;
        }
    });
}

syk_status syk_set_workspace_limit(syk_terms t, uint64_t bytes)
{
    return guard([&] {
        check_handle(t);
        t->ws.limit = (size_t)bytes;
    });
}

syk_status syk_timing_enable(int on)
{
    return guard([&] { timing_enable(on != 0); });
}

syk_status syk_timing_read(int64_t* launches, double* total_ms)
{
    return guard([&] { timing_read(launches, total_ms); });
}

syk_status syk_timing_reset(void)
{
    return guard([&] { timing_reset(); });
}

static void majorana_impl(syk_terms t, syk_dtype dtype, int a, int sector, int nvec, const void* psi, void* out,
                          hipStream_t stream)
{
    check_handle(t);
    check_dtype(dtype);
    require(a >= 0 && a < t->H.N, "Majorana index out of range");
    require(nvec >= 1, "nvec must be >= 1");
    check_ptr(psi, "psi");
    check_ptr(out, "out");
    const int M = sector < 0 ? t->H.M : t->H.M - 1;
    VecOps ops(*t, dtype, (int64_t)1 << M, nvec, stream);
    check_no_overlap(psi, out, ops.vec_bytes());
    if (sector < 0) ops.majorana(a, psi, out);
    else ops.majorana_sector(a, M, sector, psi, out);
}

syk_status syk_apply_majorana(syk_terms t, syk_dtype dtype, int a, int nvec, const void* psi, void* out,
                              hipStream_t stream)
{
    return guard([&] { majorana_impl(t, dtype, a, -1, nvec, psi, out, stream); });
}

syk_status syk_apply_majorana_sector(syk_terms t, syk_dtype dtype, int a, int sector_in, int nvec, const void* psi,
                                     void* out, hipStream_t stream)
{
    return guard([&] {
        check_sector(t, sector_in);
        majorana_impl(t, dtype, a, sector_in, nvec, psi, out, stream);
    });
}

syk_status syk_dot(syk_dtype dtype, int64_t dim, int nvec, const void* a, const void* b, double* out,
                   hipStream_t stream)
{
    return guard([&] {
        check_dtype(dtype);
        require(dim >= 1 && nvec >= 1, "dim and nvec must be >= 1");
        check_ptr(a, "a");
        check_ptr(b, "b");
        require(out != nullptr, "out is NULL");
        // Workspace owner for handle-free reductions; kept until the process
        // ends so no device memory is freed during thread teardown.
        static thread_local syk_terms_s* scratch = new syk_terms_s();
        VecOps ops(*scratch, dtype, dim, nvec, stream);
        std::vector<zd> d = ops.multidot(a, 1, b);
        for (int c = 0; c < nvec; ++c) {
            out[2 * c] = d[c].real();
            out[2 * c + 1] = d[c].imag();
        }
    });
}

static void expmv_impl(syk_terms t, syk_dtype dtype, int sector, int nvec, const int32_t* real_of_col, double z_re,
                       double z_im, double total, const syk_krylov_opts* opts, void* psi_inout, double* err_est,
                       hipStream_t stream)
{
    {
        check_handle(t);
        check_dtype(dtype);
        check_block(t, nvec, real_of_col);
        syk_krylov_opts o = check_opts(opts);
        check_ptr(psi_inout, "psi");
        require(std::isfinite(z_re) && std::isfinite(z_im) && std::isfinite(total) && total >= 0,
                "z and total must be finite, total >= 0");
        BlockCtx c(*t, dtype, nvec, real_of_col, stream, sector);
        KrylovStats st;
        st.err.assign(nvec, 0.0);
        const double step = (z_re == 0.0) ? o.dt : o.tau_step;
        krylov_propagate(c, psi_inout, std::complex<double>(z_re, z_im), total, step, o.m, st);
        SYK_HIP(hipStreamSynchronize(stream));
        if (err_est)
            for (int k = 0; k < nvec; ++k) err_est[k] = st.err[k];
        if (o.tol > 0)
            for (double e : st.err)
                if (e > o.tol) throw Error(SYK_ENOTCONVERGED, "Krylov error estimate above tolerance");
    }
}

syk_status syk_krylov_expmv(syk_terms t, syk_dtype dtype, int nvec, const int32_t* real_of_col, double z_re,
                            double z_im, double total, const syk_krylov_opts* opts, void* psi_inout,
                            double* err_est, hipStream_t stream)
{
    return guard([&] { expmv_impl(t, dtype, -1, nvec, real_of_col, z_re, z_im, total, opts, psi_inout, err_est, stream); });
}

syk_status syk_krylov_expmv_sector(syk_terms t, syk_dtype dtype, int sector, int nvec, const int32_t* real_of_col,
                                   double z_re, double z_im, double total, const syk_krylov_opts* opts,
                                   void* psi_inout, double* err_est, hipStream_t stream)
{
    return guard([&] {
        check_sector(t, sector);
        expmv_impl(t, dtype, sector, nvec, real_of_col, z_re, z_im, total, opts, psi_inout, err_est, stream);
    });
}

static void two_point_impl(int sector, syk_terms t, syk_dtype dtype, int i, double beta, const double* times, int nt, int nvec,
                         const int32_t* real_of_col, const void* psi0, const syk_krylov_opts* opts, double* G,
                         double* Z, hipStream_t stream)
{
    {
        check_handle(t);
        check_dtype(dtype);
        check_block(t, nvec, real_of_col);
        syk_krylov_opts o = check_opts(opts);
        require(i >= 0 && i < t->H.N, "Majorana index out of range");
        require(std::isfinite(beta) && beta >= 0, "beta must be finite and >= 0");
        check_ptr(psi0, "psi0");
        require(G != nullptr, "G is NULL");
        BlockCtx c(*t, dtype, nvec, real_of_col, stream, sector);
        two_point(c, i, beta, times, nt, psi0, o, G, Z);
    }
}

static void otoc_impl(int sector, syk_terms t, syk_dtype dtype, int i, int j, double beta, const double* times, int nt, int nvec,
                    const int32_t* real_of_col, const void* psi0, const syk_krylov_opts* opts, double* F,
                    double* F_im, double* Z, hipStream_t stream)
{
    {
        check_handle(t);
        check_dtype(dtype);
        check_block(t, nvec, real_of_col);
        syk_krylov_opts o = check_opts(opts);
        require(i >= 0 && i < t->H.N && j >= 0 && j < t->H.N, "Majorana index out of range");
        require(i != j, "the OTOC needs i != j");
        require(std::isfinite(beta) && beta >= 0, "beta must be finite and >= 0");
        check_ptr(psi0, "psi0");
        require(F != nullptr, "F is NULL");
        BlockCtx c(*t, dtype, nvec, real_of_col, stream, sector);
        otoc(c, i, j, beta, times, nt, psi0, o, F, F_im, Z);
    }
}

static void otoc_unregularized_impl(int sector, syk_terms t, syk_dtype dtype, int i, int j, double beta, const double* times,
                                  int nt, int nvec, const int32_t* real_of_col, const void* psi0,
                                  const syk_krylov_opts* opts, double* F, double* F_im, double* Z,
                                  hipStream_t stream)
{
    {
        check_handle(t);
        check_dtype(dtype);
        check_block(t, nvec, real_of_col);
        syk_krylov_opts o = check_opts(opts);
        require(i >= 0 && i < t->H.N && j >= 0 && j < t->H.N, "Majorana index out of range");
        require(i != j, "the OTOC needs i != j");
        require(std::isfinite(beta) && beta >= 0, "beta must be finite and >= 0");
        check_ptr(psi0, "psi0");
        require(F != nullptr, "F is NULL");
        BlockCtx c(*t, dtype, nvec, real_of_col, stream, sector);
        otoc_unregularized(c, i, j, beta, times, nt, psi0, o, F, F_im, Z);
    }
}

static void imag_two_point_impl(int sector, syk_terms t, syk_dtype dtype, int i, double beta, const double* taus, int ntau,
                              int nvec, const int32_t* real_of_col, const void* psi0, const syk_krylov_opts* opts,
                              double* G, double* Z, hipStream_t stream)
{
    {
        check_handle(t);
        check_dtype(dtype);
        check_block(t, nvec, real_of_col);
        syk_krylov_opts o = check_opts(opts);
        require(i >= 0 && i < t->H.N, "Majorana index out of range");
        require(std::isfinite(beta) && beta >= 0, "beta must be finite and >= 0");
        check_ptr(psi0, "psi0");
        require(G != nullptr, "G is NULL");
        BlockCtx c(*t, dtype, nvec, real_of_col, stream, sector);
        imag_two_point(c, i, beta, taus, ntau, psi0, o, G, Z);
    }
}

syk_status syk_two_point(syk_terms t, syk_dtype dtype, int i, double beta, const double* times, int nt, int nvec,
                         const int32_t* real_of_col, const void* psi0, const syk_krylov_opts* opts, double* G,
                         double* Z, hipStream_t stream)
{
    return guard([&] { two_point_impl(-1, t, dtype, i, beta, times, nt, nvec, real_of_col, psi0, opts, G, Z, stream); });
}

syk_status syk_two_point_sector(syk_terms t, syk_dtype dtype, int sector, int i, double beta, const double* times,
                                int nt, int nvec, const int32_t* real_of_col, const void* psi0,
                                const syk_krylov_opts* opts, double* G, double* Z, hipStream_t stream)
{
    return guard([&] {
        check_sector(t, sector);
        two_point_impl(sector, t, dtype, i, beta, times, nt, nvec, real_of_col, psi0, opts, G, Z, stream);
    });
}

syk_status syk_otoc(syk_terms t, syk_dtype dtype, int i, int j, double beta, const double* times, int nt, int nvec,
                    const int32_t* real_of_col, const void* psi0, const syk_krylov_opts* opts, double* F,
                    double* F_im, double* Z, hipStream_t stream)
{
    return guard([&] { otoc_impl(-1, t, dtype, i, j, beta, times, nt, nvec, real_of_col, psi0, opts, F, F_im, Z, stream); });
}

syk_status syk_otoc_sector(syk_terms t, syk_dtype dtype, int sector, int i, int j, double beta, const double* times,
                           int nt, int nvec, const int32_t* real_of_col, const void* psi0, const syk_krylov_opts* opts,
                           double* F, double* F_im, double* Z, hipStream_t stream)
{
    return guard([&] {
        check_sector(t, sector);
        otoc_impl(sector, t, dtype, i, j, beta, times, nt, nvec, real_of_col, psi0, opts, F, F_im, Z, stream);
    });
}

syk_status syk_otoc_unregularized(syk_terms t, syk_dtype dtype, int i, int j, double beta, const double* times,
                                  int nt, int nvec, const int32_t* real_of_col, const void* psi0,
                                  const syk_krylov_opts* opts, double* F, double* F_im, double* Z,
                                  hipStream_t stream)
{
    return guard([&] {
        otoc_unregularized_impl(-1, t, dtype, i, j, beta, times, nt, nvec, real_of_col, psi0, opts, F, F_im, Z, stream);
    });
}

syk_status syk_otoc_unregularized_sector(syk_terms t, syk_dtype dtype, int sector, int i, int j, double beta,
                                         const double* times, int nt, int nvec, const int32_t* real_of_col,
                                         const void* psi0, const syk_krylov_opts* opts, double* F, double* F_im,
                                         double* Z, hipStream_t stream)
{
    return guard([&] {
        check_sector(t, sector);
        otoc_unregularized_impl(sector, t, dtype, i, j, beta, times, nt, nvec, real_of_col, psi0, opts, F, F_im, Z,
                                stream);
    });
}

syk_status syk_imag_two_point(syk_terms t, syk_dtype dtype, int i, double beta, const double* taus, int ntau,
                              int nvec, const int32_t* real_of_col, const void* psi0, const syk_krylov_opts* opts,
                              double* G, double* Z, hipStream_t stream)
{
    return guard([&] { imag_two_point_impl(-1, t, dtype, i, beta, taus, ntau, nvec, real_of_col, psi0, opts, G, Z, stream); });
}

syk_status syk_imag_two_point_sector(syk_terms t, syk_dtype dtype, int sector, int i, double beta, const double* taus,
                                     int ntau, int nvec, const int32_t* real_of_col, const void* psi0,
                                     const syk_krylov_opts* opts, double* G, double* Z, hipStream_t stream)
{
    return guard([&] {
        check_sector(t, sector);
        imag_two_point_impl(sector, t, dtype, i, beta, taus, ntau, nvec, real_of_col, psi0, opts, G, Z, stream);
    });
}

syk_status syk_spectrum_bounds(syk_terms t, syk_dtype dtype, int m, const void* psi0, double* e_min, double* e_max,
                               hipStream_t stream)
{
    return guard([&] {
        check_handle(t);
        check_dtype(dtype);
        require(m >= 2 && m <= 64, "m must be in [2, 64]");
        check_ptr(psi0, "psi0");
        require(e_min && e_max, "outputs are NULL");
        BlockCtx c(*t, dtype, 1, nullptr, stream);
        lanczos_extremes(c, psi0, m, e_min, e_max);
    });
}

syk_status syk_lowest_eigenvalues(syk_terms t, syk_dtype dtype, int m, int k, const void* psi0, double* evals,
                                  double* resid, int* n_found, hipStream_t stream)
{
    return guard([&] {
        check_handle(t);
        check_dtype(dtype);
        require(m >= 2 && m <= 512, "m must be in [2, 512]");
        require(k >= 1 && k <= m, "k must be in [1, m]");
        check_ptr(psi0, "psi0");
        require(evals != nullptr && n_found != nullptr, "outputs are NULL");
        BlockCtx c(*t, dtype, 1, nullptr, stream);
        *n_found = lowest_eigenvalues(c, psi0, m, k, evals, resid);
    });
}

static ChebSettings check_cheb(syk_terms t, int i, int j, double beta, double t_star, const syk_cheb_opts* o)
{
    check_handle(t);
    require(o != nullptr, "Chebyshev options are NULL");
    require(i >= 0 && i < t->H.N && j >= 0 && j < t->H.N && i != j, "need 0 <= i, j < N with i != j");
    require(std::isfinite(beta) && beta >= 0, "beta must be finite and >= 0");
    require(std::isfinite(t_star) && t_star >= 0, "t_star must be finite and >= 0");
    require(o->keep_segment == 0 || o->keep_segment == 1, "keep_segment must be 0 or 1");
    ChebSettings s{o->degree, o->dt, o->tau_steps, o->checkpoint_every, o->e_center, o->e_halfwidth,
                   o->keep_segment};
    return s;
}

syk_status syk_cheb_otoc(syk_terms t, int i, int j, double beta, double t_star, const syk_cheb_opts* opts,
                         const void* psi0, double* F, hipStream_t stream)
{
    return guard([&] {
        ChebSettings s = check_cheb(t, i, j, beta, t_star, opts);
        check_ptr(psi0, "psi0");
        require(F != nullptr, "F is NULL");
        BlockCtx c(*t, SYK_C128, 1, nullptr, stream);
        cheb_otoc(c, i, j, beta, t_star, s, psi0, F, nullptr);
    });
}

syk_status syk_grad_couplings(syk_terms t, int i, int j, double beta, double t_star, const syk_cheb_opts* opts,
                              const void* psi0, double* F, double* dF_dJ, hipStream_t stream)
{
    return guard([&] {
        ChebSettings s = check_cheb(t, i, j, beta, t_star, opts);
        check_ptr(psi0, "psi0");
        require(F != nullptr && dF_dJ != nullptr, "F or dF_dJ is NULL");
        BlockCtx c(*t, SYK_C128, 1, nullptr, stream);
        cheb_otoc(c, i, j, beta, t_star, s, psi0, F, dF_dJ);
    });
}

syk_status syk_coupling_overlaps(syk_terms t, int npairs, const void* const* g, const void* const* v,
                                 const double* w, double* out, hipStream_t stream)
{
    return guard([&] {
        check_handle(t);
        require(npairs >= 1 && npairs <= 64, "npairs must be in [1, 64]");
        require(g != nullptr && v != nullptr && w != nullptr && out != nullptr, "g, v, w or out is NULL");
        std::vector<const void*> gv(npairs), vv(npairs);
        std::vector<double> wv(npairs);
        for (int p = 0; p < npairs; ++p) {
            check_ptr(g[p], "g[p]");
            check_ptr(v[p], "v[p]");
            require(std::isfinite(w[p]), "weights must be finite");
            gv[p] = g[p];
            vv[p] = v[p];
            wv[p] = w[p];
        }
        BlockCtx c(*t, SYK_C128, 1, nullptr, stream);
        const TermTables& T = t->host;
        double* bins = (double*)t->ws.get("overlap_bins", T.n_bins * 2 * sizeof(double));
        SYK_HIP(hipMemsetAsync(bins, 0, T.n_bins * 2 * sizeof(double), c.stream));
        grad_bins(*t, gv, vv, wv, bins, c.stream);
        std::vector<double> hb(T.n_bins * 2);
        SYK_HIP(hipMemcpyAsync(hb.data(), bins, hb.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        SYK_HIP(hipStreamSynchronize(c.stream));
        couplings_from_bins(T, hb.data(), out);
    });
}

}  // extern "C"
