// Vector kernels on blocks of nvec states of dimension dim, stored one after
// another (entry (r, c) at c*dim + r).
//
// Grid (gx, nvec): workgroup (bx, c) strides over the rows of column c, so
// loads are coalesced and every column reduces on its own.  Reductions
// accumulate in FP64 per thread, reduce over each wave with a fixed butterfly
// of lane exchanges, over the four waves of the workgroup in wave order, then
// over the fixed number of workgroups in index order: the result does not
// depend on timing.
#include <cmath>
#include <cstring>
#include <type_traits>

#include "vec.hpp"

namespace syk {

namespace {

constexpr int RB = 256;    // threads per workgroup
constexpr int KC = 8;      // vectors per pass of a multi-vector kernel
constexpr int kWaves = RB / 64;

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

// Workgroup sums of a[0..n) (n <= N, the same n on every thread): each wave
// adds its 64 lanes with a butterfly of lane exchanges, lane 0 of every wave
// stores its sums in red[wave][i], and after one barrier thread i < n returns
// red[0][i] + red[1][i] + red[2][i] + red[3][i] (others return 0).  red holds
// kWaves * N doubles.
template <int N>
__device__ __forceinline__ double block_sum(double (&a)[N], int n, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (i >= n) break;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a[i] += __shfl_xor(a[i], off, 64);
        if (lane == 0) red[wave * N + i] = a[i];
    }
    __syncthreads();
    double s = 0.0;
    if ((int)threadIdx.x < n)
        for (int w = 0; w < kWaves; ++w) s += red[w * N + threadIdx.x];
    return s;
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

// The multi-vector kernels take the number of basis vectors K as a template
// argument: every load of a row is then unconditional and issued before the
// first is used, instead of one branch and one wait per vector.
template <int N, typename F>
void with_count(int k, F&& f)
{
    if constexpr (N > 0) {
        if (k == N) f(std::integral_constant<int, N>{});
        else with_count<N - 1>(k, f);
    } else {
        throw Error(SYK_EINVAL, "vector kernels: unsupported number of basis vectors");
    }
}

// partial[bx][k][c] = sum over this workgroup's rows of conj(V_k[r,c]) w[r,c]
template <typename R, int K>
__global__ void __launch_bounds__(RB) k_multidot(const cplx<R>* __restrict__ V, int64_t vstride,
                                                 const cplx<R>* __restrict__ w, Shape S,
                                                 double* __restrict__ partial)
{
    __shared__ double red[kWaves * 2 * K];
    const int64_t col = (int64_t)blockIdx.y * S.D;
    double a[2 * K];
#pragma unroll
    for (int k = 0; k < 2 * K; ++k) a[k] = 0.0;
    const int64_t step = (int64_t)gridDim.x * RB;
    for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < S.D; r += step) {
        const int64_t e = col + r;
        const cplx<R> b = w[e];
        cplx<R> v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = V[k * vstride + e];
        const double br = b.re, bi = b.im;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double vr = v[k].re, vi = v[k].im;
            a[2 * k] += vr * br + vi * bi;
            a[2 * k + 1] += vr * bi - vi * br;
        }
    }
    const double t = block_sum(a, 2 * K, red);
    // thread i < 2K holds (k, re/im) = (i / 2, i % 2)
    if ((int)threadIdx.x < 2 * K)
        partial[(((int64_t)blockIdx.x * K + (threadIdx.x >> 1)) * S.B + blockIdx.y) * 2 + (threadIdx.x & 1)] = t;
}

// w -= sum_k coef[k][c] V_k; optionally partial[bx][c] = sum |w_new|^2
template <typename R, int K>
__global__ void __launch_bounds__(RB) k_update(cplx<R>* __restrict__ w, const cplx<R>* __restrict__ V,
                                               int64_t vstride, const double* __restrict__ coef,
                                               Shape S, double* __restrict__ partial)
{
    __shared__ double red[kWaves];
    const int c = blockIdx.y;
    const int64_t col = (int64_t)c * S.D;
    double cr[K], ci[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        cr[k] = coef[(k * S.B + c) * 2];
        ci[k] = coef[(k * S.B + c) * 2 + 1];
    }
    double nrm = 0.0;
    const int64_t step = (int64_t)gridDim.x * RB;
    for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < S.D; r += step) {
        const int64_t e = col + r;
        const cplx<R> b = w[e];
        cplx<R> v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = V[k * vstride + e];
        double xr = b.re, xi = b.im;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            xr -= cr[k] * v[k].re - ci[k] * v[k].im;
            xi -= cr[k] * v[k].im + ci[k] * v[k].re;
        }
        cplx<R> o;
        o.re = (R)xr;
        o.im = (R)xi;
        w[e] = o;
        const double orr = o.re, oi = o.im;
        nrm += orr * orr + oi * oi;
    }
    if (!partial) return;
    double a[1] = {nrm};
    const double t = block_sum(a, 1, red);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * S.B + c] = t;
}

// The first Gram-Schmidt update fused with the second projection, for K
// basis vectors: w' = w - sum_k coef[k][c] V_k (rounded to the state's
// precision, as stored), and partial[bx][k][c] = sum over this workgroup's rows
// of conj(V_k[r,c]) w'[r,c].  Each V_k[r] is read once for both uses.
template <typename R, int K>
__global__ void __launch_bounds__(RB) k_update_dot(cplx<R>* __restrict__ w, const cplx<R>* __restrict__ V,
                                                   int64_t vstride, const double* __restrict__ coef,
                                                   Shape S, double* __restrict__ partial)
{
    __shared__ double red[kWaves * 2 * K];
    const int c = blockIdx.y;
    const int64_t col = (int64_t)c * S.D;
    double cr[K], ci[K], a[2 * K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        cr[k] = coef[(k * S.B + c) * 2];
        ci[k] = coef[(k * S.B + c) * 2 + 1];
        a[2 * k] = a[2 * k + 1] = 0.0;
    }
    const int64_t step = (int64_t)gridDim.x * RB;
    for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < S.D; r += step) {
        const int64_t e = col + r;
        const cplx<R> b = w[e];
        cplx<R> v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = V[k * vstride + e];
        double xr = b.re, xi = b.im;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            xr -= cr[k] * v[k].re - ci[k] * v[k].im;
            xi -= cr[k] * v[k].im + ci[k] * v[k].re;
        }
        cplx<R> o;
        o.re = (R)xr;
        o.im = (R)xi;
        w[e] = o;
        const double orr = o.re, oi = o.im;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double vr = v[k].re, vi = v[k].im;
            a[2 * k] += vr * orr + vi * oi;
            a[2 * k + 1] += vr * oi - vi * orr;
        }
    }
    const double t = block_sum(a, 2 * K, red);
    if ((int)threadIdx.x < 2 * K)
        partial[(((int64_t)blockIdx.x * K + (threadIdx.x >> 1)) * S.B + c) * 2 + (threadIdx.x & 1)] = t;
}

// The scalars of Lanczos iteration j for column b = thread: alpha_j =
// Re(c1[j] + c2[j]) (the two projections on the newest basis vector), beta_j =
// ||w||.  While the column is still growing its basis, its scale estimate
// max_i (|alpha_i| + beta_{i-1}) is updated, and unless j is the last
// iteration, beta_j at or below 1e-13 times that scale (or a zero start
// vector) marks the subspace invariant (kdim = j + 1, f = 0); otherwise
// f = 1 / beta_j scales w into the next basis vector.  A non-finite alpha or
// beta sets flag[0].
__global__ void k_lanczos_coef(const double* __restrict__ c1, const double* __restrict__ c2,
                               const double* __restrict__ wnorm2, int j, int m, int B, double* __restrict__ alpha,
                               double* __restrict__ beta, int* __restrict__ kdim, double* __restrict__ scale,
                               const double* __restrict__ nrm, double* __restrict__ f, int* __restrict__ flag)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double a = c1[((size_t)j * B + b) * 2] + c2[((size_t)j * B + b) * 2];
    const double bt = sqrt(wnorm2[b]);
    if (!isfinite(a) || !isfinite(bt)) flag[0] = 1;
    alpha[(size_t)j * B + b] = a;
    beta[(size_t)j * B + b] = bt;
    double fb = 0.0;
    if (j < kdim[b]) {
        scale[b] = fmax(scale[b], fabs(a) + (j > 0 ? beta[(size_t)(j - 1) * B + b] : 0.0));
        if (j < m - 1) {
            if (bt <= 1e-13 * scale[b] || nrm[b] == 0.0) kdim[b] = j + 1;
            else fb = 1.0 / bt;
        }
    }
    f[b] = fb;
}

// out[i] = sum of partial[g][i] over g < G, for i < n doubles: one wave per
// output, lane l adding g = l, l + 64, ... in order, then a fixed butterfly
// over the lanes (the same order on every run).
__global__ void __launch_bounds__(64) k_finish(const double* __restrict__ partial, int G, int n,
                                               double* __restrict__ out)
{
    const int i = blockIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int g = (int)threadIdx.x; g < G; g += 64) s += partial[(int64_t)g * n + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) out[i] = s;
}

void launch_finish(const double* partial, int G, int n, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_finish, dim3(n), dim3(64), 0, st, partial, G, n, out);
    SYK_HIP(hipGetLastError());
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
        int k = 0;
        for (; k + KC <= K; k += KC) {   // KC loads in flight, then their FMAs
            cplx<R> v[KC];
#pragma unroll
            for (int u = 0; u < KC; ++u) v[u] = V[(k + u) * vstride + e];
#pragma unroll
            for (int u = 0; u < KC; ++u) {
                const double cr = coef[((k + u) * S.B + c) * 2], ci = coef[((k + u) * S.B + c) * 2 + 1];
                xr += cr * v[u].re - ci * v[u].im;
                xi += cr * v[u].im + ci * v[u].re;
            }
        }
        for (; k < K; ++k) {
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

const double* VecOps::multidot_dev(const void* V, int K, const void* w, const char* slot)
{
    Shape S{dim_, nvec_};
    dim3 g = grid_of(S, true);
    const int B = nvec_;
    double* out = (double*)h_.ws.get(slot, (size_t)std::max(K, kFusedMax) * B * 2 * sizeof(double));
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kk = std::min(KC, K - k0);
        double* part = (double*)h_.ws.get("md_part", (size_t)g.x * kk * B * 2 * sizeof(double));
        const size_t off = (size_t)k0 * vec_bytes();
        with_count<KC>(kk, [&](auto kc) {
            constexpr int K_ = decltype(kc)::value;
            if (dt_ == SYK_C128)
                hipLaunchKernelGGL((k_multidot<double, K_>), g, dim3(RB), 0, s_,
                                   (const c128*)((const char*)V + off), dim_ * B, (const c128*)w, S, part);
            else
                hipLaunchKernelGGL((k_multidot<float, K_>), g, dim3(RB), 0, s_,
                                   (const c64*)((const char*)V + off), dim_ * B, (const c64*)w, S, part);
        });
        SYK_HIP(hipGetLastError());
        const int n = kk * B * 2;
        launch_finish(part, (int)g.x, n, out + (size_t)k0 * B * 2, s_);
        SYK_HIP(hipGetLastError());
    }
    return out;
}

std::vector<zd> VecOps::fetch(const double* dev, int K)
{
    const size_t n = (size_t)K * nvec_;
    std::vector<double> flat = download<double>(dev, 2 * n);
    std::vector<zd> res(n);
    for (size_t i = 0; i < n; ++i) res[i] = zd(flat[2 * i], flat[2 * i + 1]);
    return res;
}

std::vector<zd> VecOps::multidot(const void* V, int K, const void* w)
{
    return fetch(multidot_dev(V, K, w, "md_out"), K);
}

const double* VecOps::update_dot(void* w, const void* V, int K, const double* c1, const char* slot)
{
    if (K < 1 || K > kFusedMax) throw Error(SYK_EINVAL, "update_dot: unsupported basis size");
    Shape S{dim_, nvec_};
    dim3 g = grid_of(S, true);
    const int B = nvec_;
    double* part = (double*)h_.ws.get("ud_part", (size_t)g.x * kFusedMax * B * 2 * sizeof(double));
    double* out = (double*)h_.ws.get(slot, (size_t)kFusedMax * B * 2 * sizeof(double));
    const int64_t vs = dim_ * B;
    with_count<kFusedMax>(K, [&](auto kc) {
        constexpr int K_ = decltype(kc)::value;
        if (dt_ == SYK_C128)
            hipLaunchKernelGGL((k_update_dot<double, K_>), g, dim3(RB), 0, s_, (c128*)w, (const c128*)V, vs, c1, S,
                               part);
        else
            hipLaunchKernelGGL((k_update_dot<float, K_>), g, dim3(RB), 0, s_, (c64*)w, (const c64*)V, vs, c1, S, part);
    });
    SYK_HIP(hipGetLastError());
    const int n = K * B * 2;
    launch_finish(part, (int)g.x, n, out, s_);
    SYK_HIP(hipGetLastError());
    return out;
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
    return update_dev(w, V, K, (const double*)upload(coef), want_norm);
}

std::vector<double> VecOps::update_dev(void* w, const void* V, int K, const double* dcoef, bool want_norm)
{
    const double* n = update_dev_norm(w, V, K, dcoef, want_norm);
    if (!want_norm) return {};
    return download<double>(n, nvec_);
}

const double* VecOps::update_dev_norm(void* w, const void* V, int K, const double* dcoef, bool want_norm)
{
    Shape S{dim_, nvec_};
    const int B = nvec_;
    dim3 g = grid_of(S, true);
    double* part = want_norm ? (double*)h_.ws.get("up_part", (size_t)g.x * B * sizeof(double)) : nullptr;
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kk = std::min(KC, K - k0);
        const bool last = k0 + KC >= K;
        const size_t off = (size_t)k0 * vec_bytes();
        double* p = (last && want_norm) ? part : nullptr;
        with_count<KC>(kk, [&](auto kc) {
            constexpr int K_ = decltype(kc)::value;
            if (dt_ == SYK_C128)
                hipLaunchKernelGGL((k_update<double, K_>), g, dim3(RB), 0, s_, (c128*)w,
                                   (const c128*)((const char*)V + off), dim_ * B, dcoef + (size_t)k0 * B * 2, S, p);
            else
                hipLaunchKernelGGL((k_update<float, K_>), g, dim3(RB), 0, s_, (c64*)w,
                                   (const c64*)((const char*)V + off), dim_ * B, dcoef + (size_t)k0 * B * 2, S, p);
        });
        SYK_HIP(hipGetLastError());
    }
    if (!want_norm) return nullptr;
    double* out = (double*)h_.ws.get("up_out", (size_t)B * sizeof(double));
    launch_finish(part, (int)g.x, B, out, s_);
    SYK_HIP(hipGetLastError());
    return out;
}

void VecOps::lanczos_coef(const double* c1, const double* c2, const double* wnorm2, int j, int m, LanczosScalars& z)
{
    const int B = nvec_;
    hipLaunchKernelGGL(k_lanczos_coef, dim3((B + 255) / 256), dim3(256), 0, s_, c1, c2, wnorm2, j, m, B, z.alpha,
                       z.beta, z.kdim, z.scale, z.nrm, z.f, z.flag);
    SYK_HIP(hipGetLastError());
}

void VecOps::scale_dev(void* out, const void* in, const double* df)
{
    Shape S{dim_, nvec_};
    dim3 g = grid_of(S, false);
    if (dt_ == SYK_C128)
        hipLaunchKernelGGL(k_scale<double>, g, dim3(RB), 0, s_, (c128*)out, (const c128*)in, df, S);
    else
        hipLaunchKernelGGL(k_scale<float>, g, dim3(RB), 0, s_, (c64*)out, (const c64*)in, df, S);
    SYK_HIP(hipGetLastError());
}

void VecOps::to_device(void* dev, const void* host, size_t bytes)
{
    SYK_HIP(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, s_));
    SYK_HIP(hipStreamSynchronize(s_));
}

void VecOps::to_host(void* host, const void* dev, size_t bytes)
{
    SYK_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s_));
    SYK_HIP(hipStreamSynchronize(s_));
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
