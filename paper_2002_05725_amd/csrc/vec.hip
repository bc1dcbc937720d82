// Vector kernels on blocks of nvec states of dimension dim, stored one after
// another (entry (r, c) at c*dim + r).
//
// Grid (gx, nvec): workgroup (bx, c) strides over the rows of column c, so
// loads are coalesced and every column reduces on its own.  Reductions
// accumulate in FP64 per thread, reduce over the workgroup with a fixed-shape
// tree in LDS, then over the fixed number of workgroups in index order: the
// result does not depend on timing.
#include <cmath>
#include <cstring>

#include "vec.hpp"

namespace syk {

namespace {

constexpr int RB = 256;    // threads per workgroup
constexpr int KC = 8;      // vectors per pass of a multi-vector kernel

struct Shape {
    int64_t D;   // rows per column
    int B;       // columns
};

// Workgroups per column: about 2048 over the whole block (a few per CU, enough
// loads in flight to stream at HBM speed), at most 1024 per column.  For
// reductions this count is a function of the shape only, so the summation
// order, and the result, do not depend on timing.
inline dim3 grid_of(const Shape& S, bool reduction)
{
    const int64_t want = (S.D + RB - 1) / RB;
    int gx = reduction ? std::max(32, std::min(1024, 2048 / std::max(1, S.B)))
                       : (int)std::max<int64_t>(1, 4096 / std::max(1, S.B));
    if (want < gx) gx = (int)want;
    if (gx < 1) gx = 1;
    return dim3(gx, S.B);
}

// Sum red[i][*] over the workgroup (fixed tree); thread 0 holds the totals.
__device__ __forceinline__ void tree_reduce(double* red, int n)
{
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int i = 0; i < n; ++i) red[i * RB + threadIdx.x] += red[i * RB + threadIdx.x + s];
        __syncthreads();
    }
}

template <typename R>
__global__ void __launch_bounds__(RB) k_majorana(const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                 Shape S, int a)
{
    const int64_t col = (int64_t)blockIdx.y * S.D;
    const int k = a >> 1;
    const uint64_t bit = (uint64_t)1 << k;
    const uint64_t below = bit - 1;
    const R amp = (R)0.70710678118654752440;
    const int64_t step = (int64_t)gridDim.x * RB;
    for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < S.D; r += step) {
        const uint64_t s = (uint64_t)r ^ bit;   // source row
        const cplx<R> v = in[col + (int64_t)s];
        int neg = __popcll(s & below) & 1;
        cplx<R> o;
        if (a & 1) {             // i (-1)^{s_k} times the Z string
            neg ^= (int)((s >> k) & 1);
            o.re = -amp * v.im;
            o.im = amp * v.re;
        } else {
            o.re = amp * v.re;
            o.im = amp * v.im;
        }
        if (neg) { o.re = -o.re; o.im = -o.im; }
        out[col + r] = o;
    }
}

// chi_a on a parity-sector state (rows u: full row u + 2^top (parity(u) ^ s_in)).
// For k = a/2 < top the map is the full-space one on u; for k = top the flipped
// qubit is the implied one, so u maps to itself and the Z string below it covers
// every bit of u.
template <typename R>
__global__ void __launch_bounds__(RB) k_majorana_sector(const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                        Shape S, int a, int top, int s_in)
{
    const int64_t col = (int64_t)blockIdx.y * S.D;
    const int k = a >> 1;
    const bool implied = (k == top);
    const uint64_t bit = implied ? 0u : (uint64_t)1 << k;
    const uint64_t below = implied ? (uint64_t)S.D - 1u : bit - 1u;
    const R amp = (R)0.70710678118654752440;
    const int64_t step = (int64_t)gridDim.x * RB;
    for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < S.D; r += step) {
        const uint64_t s = (uint64_t)r ^ bit;   // source row
        const cplx<R> v = in[col + (int64_t)s];
        int neg = __popcll(s & below) & 1;
        cplx<R> o;
        if (a & 1) {             // i (-1)^{s_k} times the Z string
            neg ^= implied ? ((__popcll(s) & 1) ^ s_in) : (int)((s >> k) & 1);
            o.re = -amp * v.im;
            o.im = amp * v.re;
        } else {
            o.re = amp * v.re;
            o.im = amp * v.im;
        }
        if (neg) { o.re = -o.re; o.im = -o.im; }
        out[col + r] = o;
    }
}

// partial[bx][k][c] = sum over this workgroup's rows of conj(V_k[r,c]) w[r,c]
template <typename R>
__global__ void __launch_bounds__(RB) k_multidot(const cplx<R>* __restrict__ V, int64_t vstride, int K,
                                                 const cplx<R>* __restrict__ w, Shape S,
                                                 double* __restrict__ partial)
{
    __shared__ double red[2 * KC * RB];
    const int64_t col = (int64_t)blockIdx.y * S.D;
    double ar[KC], ai[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) ar[k] = ai[k] = 0.0;
    const int64_t step = (int64_t)gridDim.x * RB;
    for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < S.D; r += step) {
        const int64_t e = col + r;
        const cplx<R> b = w[e];
        const double br = b.re, bi = b.im;
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (k < K) {
                const cplx<R> v = V[k * vstride + e];
                const double vr = v.re, vi = v.im;
                ar[k] += vr * br + vi * bi;
                ai[k] += vr * bi - vi * br;
            }
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        red[(2 * k) * RB + threadIdx.x] = ar[k];
        red[(2 * k + 1) * RB + threadIdx.x] = ai[k];
    }
    tree_reduce(red, 2 * K);
    if (threadIdx.x == 0)
        for (int k = 0; k < K; ++k) {
            double* p = partial + (((int64_t)blockIdx.x * K + k) * S.B + blockIdx.y) * 2;
            p[0] = red[(2 * k) * RB];
            p[1] = red[(2 * k + 1) * RB];
        }
}

// w -= sum_k coef[k][c] V_k; optionally partial[bx][c] = sum |w_new|^2
template <typename R>
__global__ void __launch_bounds__(RB) k_update(cplx<R>* __restrict__ w, const cplx<R>* __restrict__ V,
                                               int64_t vstride, int K, const double* __restrict__ coef,
                                               Shape S, double* __restrict__ partial)
{
    __shared__ double red[RB];
    const int c = blockIdx.y;
    const int64_t col = (int64_t)c * S.D;
    double cr[KC], ci[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        cr[k] = (k < K) ? coef[(k * S.B + c) * 2] : 0.0;
        ci[k] = (k < K) ? coef[(k * S.B + c) * 2 + 1] : 0.0;
    }
    double nrm = 0.0;
    const int64_t step = (int64_t)gridDim.x * RB;
    for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < S.D; r += step) {
        const int64_t e = col + r;
        const cplx<R> b = w[e];
        double xr = b.re, xi = b.im;
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (k < K) {
                const cplx<R> v = V[k * vstride + e];
                xr -= cr[k] * v.re - ci[k] * v.im;
                xi -= cr[k] * v.im + ci[k] * v.re;
            }
        cplx<R> o;
        o.re = (R)xr;
        o.im = (R)xi;
        w[e] = o;
        const double orr = o.re, oi = o.im;
        nrm += orr * orr + oi * oi;
    }
    if (!partial) return;
    red[threadIdx.x] = nrm;
    tree_reduce(red, 1);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * S.B + c] = red[0];
}

// Sum partial[g][i] over g < G in index order, for i < n doubles.
__global__ void k_finish(const double* __restrict__ partial, int G, int n, double* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += partial[(int64_t)g * n + i];
    out[i] = s;
}

template <typename R>
__global__ void __launch_bounds__(RB) k_scale(cplx<R>* out, const cplx<R>* in, const double* __restrict__ f, Shape S)
{
    const int64_t col = (int64_t)blockIdx.y * S.D;
    const double fc = f[blockIdx.y];
    const int64_t step = (int64_t)gridDim.x * RB;
    for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < S.D; r += step) {
        const int64_t e = col + r;
        const cplx<R> v = in[e];
        cplx<R> o;
        o.re = (R)(fc * (double)v.re);
        o.im = (R)(fc * (double)v.im);
        out[e] = o;
    }
}

// y = sum_k coef[k][c] V_k for all K vectors
template <typename R>
__global__ void __launch_bounds__(RB) k_combine(cplx<R>* __restrict__ y, const cplx<R>* __restrict__ V,
                                                int64_t vstride, int K, const double* __restrict__ coef, Shape S)
{
    const int c = blockIdx.y;
    const int64_t col = (int64_t)c * S.D;
    const int64_t step = (int64_t)gridDim.x * RB;
    for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < S.D; r += step) {
        const int64_t e = col + r;
        double xr = 0.0, xi = 0.0;
        for (int k = 0; k < K; ++k) {
            const double cr = coef[(k * S.B + c) * 2], ci = coef[(k * S.B + c) * 2 + 1];
            const cplx<R> v = V[k * vstride + e];
            xr += cr * v.re - ci * v.im;
            xi += cr * v.im + ci * v.re;
        }
        cplx<R> o;
        o.re = (R)xr;
        o.im = (R)xi;
        y[e] = o;
    }
}

}  // namespace

VecOps::VecOps(syk_terms_s& h, syk_dtype dt, int64_t dim, int nvec, hipStream_t s)
    : h_(h), dt_(dt), dim_(dim), nvec_(nvec), s_(s)
{
    require(nvec >= 1 && nvec <= 65535, "nvec must be in [1, 65535]");
}

void* VecOps::upload(const std::vector<zd>& c)
{
    std::vector<double> flat(2 * c.size());
    std::memcpy(flat.data(), c.data(), flat.size() * sizeof(double));
    return upload(flat);
}

void* VecOps::upload(const std::vector<double>& c)
{
    // A synchronous copy from the caller's host vector (a few hundred bytes):
    // when it returns, all earlier work on the stream has finished, so the
    // device slot can be reused freely.
    void* d = h_.ws.get("upload" + std::to_string(h_.upload_slot++ % 8), c.size() * sizeof(double));
    SYK_HIP(hipMemcpyAsync(d, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, s_));
    SYK_HIP(hipStreamSynchronize(s_));
    return d;
}

template <typename T>
std::vector<T> VecOps::download(const void* dev, size_t n)
{
    std::vector<T> out(n);
    SYK_HIP(hipMemcpyAsync(out.data(), dev, n * sizeof(T), hipMemcpyDeviceToHost, s_));
    SYK_HIP(hipStreamSynchronize(s_));
    return out;
}

void VecOps::majorana(int a, const void* in, void* out)
{
    Shape S{dim_, nvec_};
    dim3 g = grid_of(S, false);
    if (dt_ == SYK_C128)
        hipLaunchKernelGGL(k_majorana<double>, g, dim3(RB), 0, s_, (const c128*)in, (c128*)out, S, a);
    else
        hipLaunchKernelGGL(k_majorana<float>, g, dim3(RB), 0, s_, (const c64*)in, (c64*)out, S, a);
    SYK_HIP(hipGetLastError());
}

void VecOps::majorana_sector(int a, int top, int s_in, const void* in, void* out)
{
    if ((a >> 1) > top || top >= 63 || (s_in != 0 && s_in != 1)) throw Error(SYK_EINVAL, "majorana: bad sector arguments");
    Shape S{dim_, nvec_};
    dim3 g = grid_of(S, false);
    if (dt_ == SYK_C128)
        hipLaunchKernelGGL(k_majorana_sector<double>, g, dim3(RB), 0, s_, (const c128*)in, (c128*)out, S, a, top, s_in);
    else
        hipLaunchKernelGGL(k_majorana_sector<float>, g, dim3(RB), 0, s_, (const c64*)in, (c64*)out, S, a, top, s_in);
    SYK_HIP(hipGetLastError());
}

std::vector<zd> VecOps::multidot(const void* V, int K, const void* w)
{
    Shape S{dim_, nvec_};
    dim3 g = grid_of(S, true);
    const int B = nvec_;
    std::vector<zd> res((size_t)K * B);
    double* out = (double*)h_.ws.get("md_out", (size_t)K * B * 2 * sizeof(double));
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kk = std::min(KC, K - k0);
        double* part = (double*)h_.ws.get("md_part", (size_t)g.x * kk * B * 2 * sizeof(double));
        const size_t off = (size_t)k0 * vec_bytes();
        if (dt_ == SYK_C128)
            hipLaunchKernelGGL(k_multidot<double>, g, dim3(RB), 0, s_,
                               (const c128*)((const char*)V + off), dim_ * B, kk, (const c128*)w, S, part);
        else
            hipLaunchKernelGGL(k_multidot<float>, g, dim3(RB), 0, s_,
                               (const c64*)((const char*)V + off), dim_ * B, kk, (const c64*)w, S, part);
        SYK_HIP(hipGetLastError());
        const int n = kk * B * 2;
        hipLaunchKernelGGL(k_finish, dim3((n + 255) / 256), dim3(256), 0, s_, part, (int)g.x, n,
                           out + (size_t)k0 * B * 2);
        SYK_HIP(hipGetLastError());
    }
    std::vector<double> flat = download<double>(out, (size_t)K * B * 2);
    for (size_t i = 0; i < res.size(); ++i) res[i] = zd(flat[2 * i], flat[2 * i + 1]);
    return res;
}

std::vector<double> VecOps::norm2(const void* a)
{
    std::vector<zd> d = multidot(a, 1, a);
    std::vector<double> out(d.size());
    for (size_t i = 0; i < d.size(); ++i) out[i] = d[i].real();
    return out;
}

std::vector<double> VecOps::update(void* w, const void* V, int K, const std::vector<zd>& coef, bool want_norm)
{
    Shape S{dim_, nvec_};
    const int B = nvec_;
    dim3 g = grid_of(S, true);
    std::vector<double> norms;
    double* dcoef = (double*)upload(coef);
    double* part = want_norm ? (double*)h_.ws.get("up_part", (size_t)g.x * B * sizeof(double)) : nullptr;
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kk = std::min(KC, K - k0);
        const bool last = k0 + KC >= K;
        const size_t off = (size_t)k0 * vec_bytes();
        double* p = (last && want_norm) ? part : nullptr;
        if (dt_ == SYK_C128)
            hipLaunchKernelGGL(k_update<double>, g, dim3(RB), 0, s_, (c128*)w,
                               (const c128*)((const char*)V + off), dim_ * B, kk, dcoef + (size_t)k0 * B * 2, S, p);
        else
            hipLaunchKernelGGL(k_update<float>, g, dim3(RB), 0, s_, (c64*)w,
                               (const c64*)((const char*)V + off), dim_ * B, kk, dcoef + (size_t)k0 * B * 2, S, p);
        SYK_HIP(hipGetLastError());
    }
    if (!want_norm) return norms;
    double* out = (double*)h_.ws.get("up_out", (size_t)B * sizeof(double));
    hipLaunchKernelGGL(k_finish, dim3((B + 255) / 256), dim3(256), 0, s_, part, (int)g.x, B, out);
    SYK_HIP(hipGetLastError());
    return download<double>(out, B);
}

void VecOps::scale(void* out, const void* in, const std::vector<double>& f)
{
    Shape S{dim_, nvec_};
    dim3 g = grid_of(S, false);
    double* df = (double*)upload(f);
    if (dt_ == SYK_C128)
        hipLaunchKernelGGL(k_scale<double>, g, dim3(RB), 0, s_, (c128*)out, (const c128*)in, df, S);
    else
        hipLaunchKernelGGL(k_scale<float>, g, dim3(RB), 0, s_, (c64*)out, (const c64*)in, df, S);
    SYK_HIP(hipGetLastError());
}

void VecOps::combine(void* y, const void* V, int K, const std::vector<zd>& coef)
{
    Shape S{dim_, nvec_};
    dim3 g = grid_of(S, false);
    double* dcoef = (double*)upload(coef);
    if (dt_ == SYK_C128)
        hipLaunchKernelGGL(k_combine<double>, g, dim3(RB), 0, s_, (c128*)y, (const c128*)V, dim_ * nvec_, K, dcoef, S);
    else
        hipLaunchKernelGGL(k_combine<float>, g, dim3(RB), 0, s_, (c64*)y, (const c64*)V, dim_ * nvec_, K, dcoef, S);
    SYK_HIP(hipGetLastError());
}

void VecOps::copy(void* dst, const void* src)
{
    if (dst != src) SYK_HIP(hipMemcpyAsync(dst, src, vec_bytes(), hipMemcpyDeviceToDevice, s_));
}

}  // namespace syk
