// Kernels of the Chebyshev propagator and of the coupling derivatives.
//
// k_cheb_rec: one step of the three-term recurrence T_{n+1} = 2 H~ T_n - T_{n-1}
// (and of its transpose, Clenshaw's recurrence), fused with the running sum.
//
// k_grad_bins: for pairs (g_p, v_p) with weights w_p, accumulates for every flip
// mask the bins of sum_p w_p conj(g_p[r]) (-1)^{|r & zbase|} v_p[r ^ x] that
// determine Re <g_p| Q_n v_p> for each coupling n of the mask (terms.hpp).  A
// workgroup sweeps a fixed set of tiles for one chunk of masks at a time with
// the chunk's bins in LDS, then writes them to its own slice of a partial
// buffer; k_bins_reduce adds the slices in a fixed order.
#include "grad.hpp"

#include <cstring>

namespace syk {

namespace {

__device__ __forceinline__ uint32_t parity(uint32_t v) { return __popc(v) & 1u; }
__device__ __forceinline__ uint32_t bit(uint32_t r, uint32_t q) { return (r >> q) & 1u; }
__device__ __forceinline__ double flip(double x, uint32_t s)
{
    return __hiloint2double(__double2hiint(x) ^ (int)(s << 31), __double2loint(x));
}
__device__ __forceinline__ uint32_t quad_index(uint32_t r, uint32_t qpack)
{
    return bit(r, mask_q(qpack, 0)) | (bit(r, mask_q(qpack, 1)) << 1) | (bit(r, mask_q(qpack, 2)) << 2) |
           (bit(r, mask_q(qpack, 3)) << 3);
}

// out = b (w - gamma y) + s z + c x ; acc += ca out (acc optional).  Null
// pointers drop their term.  out may alias z or x.
template <typename R>
__global__ void __launch_bounds__(256) k_cheb_rec(cplx<R>* out, const cplx<R>* __restrict__ w,
                                                  const cplx<R>* __restrict__ y, const cplx<R>* z,
                                                  const cplx<R>* x, cplx<R>* acc, double b, double gamma, double s,
                                                  double c_re, double c_im, double ca_re, double ca_im, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double re = 0.0, im = 0.0;
        if (w) {
            const cplx<R> wv = w[e];
            const cplx<R> yv = y[e];
            re = b * ((double)wv.re - gamma * (double)yv.re);
            im = b * ((double)wv.im - gamma * (double)yv.im);
        }
        if (z) {
            const cplx<R> zv = z[e];
            re += s * (double)zv.re;
            im += s * (double)zv.im;
        }
        if (x) {
            const cplx<R> xv = x[e];
            re += c_re * (double)xv.re - c_im * (double)xv.im;
            im += c_re * (double)xv.im + c_im * (double)xv.re;
        }
        cplx<R> o;
        o.re = (R)re;
        o.im = (R)im;
        out[e] = o;
        if (acc) {
            const cplx<R> a = acc[e];
            cplx<R> r;
            r.re = (R)((double)a.re + ca_re * re - ca_im * im);
            r.im = (R)((double)a.im + ca_re * im + ca_im * re);
            acc[e] = r;
        }
    }
}

struct GLayout {
    int tile_bits;
    uint32_t n_tiles;
    int n_chunks;
    int npairs;
    int M;
    int n_diag;
    uint64_t n_bins;
};

template <int RPT>
__global__ void __launch_bounds__(256) k_grad_bins(const KRec* __restrict__ krec, const GChunk* __restrict__ chunks,
                                                    const uint32_t* __restrict__ dz, GLayout L,
                                                    const c128* const* __restrict__ gs,
                                                    const c128* const* __restrict__ vs,
                                                    const double* __restrict__ wts, double* __restrict__ partial)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const uint32_t nt = blockDim.x;
    const uint32_t tile_elems = nt * RPT;
    c128* src = reinterpret_cast<c128*>(smem_raw);
    double* bins = reinterpret_cast<double*>(src + tile_elems);     // [kGradBinCap][2]
    const uint32_t tid = threadIdx.x;
    const uint32_t row_mask = (1u << L.tile_bits) - 1u;
    const uint32_t kmask = row_mask & ~(nt - 1u);
    double* mine = partial + (uint64_t)blockIdx.x * L.n_bins * 2;

    for (int ch = 0; ch < L.n_chunks; ++ch) {
        const GChunk C = chunks[ch];
        for (uint32_t e = tid; e < 2 * C.bin_count; e += nt) bins[e] = 0.0;
        for (uint32_t tile = blockIdx.x; tile < L.n_tiles; tile += gridDim.x) {
            const uint32_t base = tile << L.tile_bits;
            for (int p = 0; p < L.npairs; ++p) {
                const c128* __restrict__ g = gs[p];
                const c128* __restrict__ v = vs[p];
                const double wt = wts[p];
                c128 gk[RPT];
#pragma unroll
                for (int k = 0; k < RPT; ++k) gk[k] = g[base + tid + k * nt];
                __syncthreads();   // previous users of src are done
                const uint64_t sbase = (uint64_t)(tile ^ C.x_high) << L.tile_bits;
#pragma unroll
                for (int k = 0; k < RPT; ++k) src[tid + k * nt] = v[sbase + tid + k * nt];
                __syncthreads();

                for (uint32_t mi = C.first; mi < C.first + C.count; ++mi) {
                    const KRec m = krec[mi];
                    const uint32_t type = m.meta >> 28;
                    double* mb = bins + 2 * (m.pad[0] - C.bin_begin);
                    if (type == MASK_QUAD) {
                        const uint32_t path = (m.meta >> 26) & 3u;
                        const uint32_t il = quad_index(tid, m.qpack) | quad_index(base, m.qpack);
                        const uint32_t sl = parity(tid & m.zbase) ^ parity(base & m.zbase);
                        if (path != PATH_FULL) {
                            double ar = 0.0, ai = 0.0;
#pragma unroll
                            for (int k = 0; k < RPT; ++k) {
                                const uint32_t sk = (m.kinfo[k / 6] >> (5 * (k % 6) + 4)) & 1u;
                                const c128 x = src[(tid + k * nt) ^ m.xl];
                                // conj(g) x with the row's sign
                                const double pr = gk[k].re * x.re + gk[k].im * x.im;
                                const double pi = gk[k].re * x.im - gk[k].im * x.re;
                                ar += flip(pr, sk);
                                ai += flip(pi, sk);
                            }
                            const uint32_t idx = il | (m.kinfo[0] & 15u);
                            atomicAdd(&mb[2 * idx], wt * flip(ar, sl));
                            atomicAdd(&mb[2 * idx + 1], wt * flip(ai, sl));
                        } else {
#pragma unroll
                            for (int k = 0; k < RPT; ++k) {
                                const uint32_t ki = (m.kinfo[k / 6] >> (5 * (k % 6))) & 31u;
                                const c128 x = src[(tid + k * nt) ^ m.xl];
                                const uint32_t s = sl ^ (ki >> 4);
                                const double pr = gk[k].re * x.re + gk[k].im * x.im;
                                const double pi = gk[k].re * x.im - gk[k].im * x.re;
                                const uint32_t idx = il | (ki & 15u);
                                atomicAdd(&mb[2 * idx], wt * flip(pr, s));
                                atomicAdd(&mb[2 * idx + 1], wt * flip(pi, s));
                            }
                        }
                    } else if (type == MASK_PAIR) {
                        const uint32_t q0 = mask_q(m.qpack, 0), q1 = mask_q(m.qpack, 1);
#pragma unroll
                        for (int k = 0; k < RPT; ++k) {
                            const uint32_t r = base | tid | (k * nt);
                            const c128 x = src[(tid + k * nt) ^ m.xl];
                            const uint32_t s = parity(r & m.zbase);
                            const double pr = wt * flip(gk[k].re * x.re + gk[k].im * x.im, s);
                            const double pi = wt * flip(gk[k].re * x.im - gk[k].im * x.re, s);
                            const uint32_t idx = bit(r, q0) | (bit(r, q1) << 1);
                            atomicAdd(&mb[2 * idx], pr);
                            atomicAdd(&mb[2 * idx + 1], pi);
                            for (uint32_t rb = r & ((1u << L.M) - 1u); rb; rb &= rb - 1) {
                                const uint32_t c = __ffs(rb) - 1;
                                atomicAdd(&mb[2 * (4 + 4 * c + idx)], pr);
                                atomicAdd(&mb[2 * (4 + 4 * c + idx) + 1], pi);
                            }
                        }
                    } else {  // MASK_DIAG
#pragma unroll
                        for (int k = 0; k < RPT; ++k) {
                            const uint32_t r = base | tid | (k * nt);
                            const c128 x = src[tid + k * nt];
                            const double pr = wt * (gk[k].re * x.re + gk[k].im * x.im);
                            const double pi = wt * (gk[k].re * x.im - gk[k].im * x.re);
                            for (int n = 0; n < L.n_diag; ++n) {
                                const uint32_t s = parity(r & dz[n]);
                                atomicAdd(&mb[2 * n], flip(pr, s));
                                atomicAdd(&mb[2 * n + 1], flip(pi, s));
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        for (uint32_t e = tid; e < 2 * C.bin_count; e += nt) mine[2 * (uint64_t)C.bin_begin + e] = bins[e];
        __syncthreads();
    }
    (void)kmask;
}

// out[i] += sum_b partial[b][i] for i < n (in block order b = 0, 1, ...).
__global__ void k_bins_reduce(const double* __restrict__ partial, int nblk, uint64_t n, double* __restrict__ out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(uint64_t)b * n + i];
    out[i] += s;
}

}  // namespace

std::vector<GChunk> make_grad_chunks(const std::vector<MaskRec>& masks, const std::vector<uint64_t>& bin_off,
                                     uint64_t n_bins, int tile_bits)
{
    std::vector<GChunk> out;
    for (uint32_t i = 0; i < (uint32_t)masks.size(); ++i) {
        const uint32_t xh = masks[i].x >> tile_bits;
        const uint64_t nb = ((i + 1 < masks.size()) ? bin_off[i + 1] : n_bins) - bin_off[i];
        if (nb > (uint64_t)kGradBinCap) throw Error(SYK_EUNSUPPORTED, "gradient: mask with too many bins");
        const bool same = !out.empty() && out.back().x_high == xh;
        if (!same || out.back().count == (uint32_t)kChunkMasks || out.back().bin_count + nb > (uint64_t)kGradBinCap) {
            GChunk c{};
            c.x_high = xh;
            c.first = i;
            c.bin_begin = (uint32_t)bin_off[i];
            out.push_back(c);
        }
        ++out.back().count;
        out.back().bin_count += (uint32_t)nb;
    }
    return out;
}

void cheb_rec(syk_dtype dtype, int64_t n, void* out, const void* w, const void* y, const void* z, const void* x,
              void* acc, double b, double gamma, double s, std::complex<double> c, std::complex<double> ca,
              hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    if (dtype == SYK_C128)
        hipLaunchKernelGGL(k_cheb_rec<double>, dim3((unsigned)blocks), dim3(256), 0, st, (c128*)out, (const c128*)w,
                           (const c128*)y, (const c128*)z, (const c128*)x, (c128*)acc, b, gamma, s, c.real(), c.imag(),
                           ca.real(), ca.imag(), n);
    else
        hipLaunchKernelGGL(k_cheb_rec<float>, dim3((unsigned)blocks), dim3(256), 0, st, (c64*)out, (const c64*)w,
                           (const c64*)y, (const c64*)z, (const c64*)x, (c64*)acc, b, gamma, s, c.real(), c.imag(),
                           ca.real(), ca.imag(), n);
    SYK_HIP(hipGetLastError());
}

void grad_bins(syk_terms_s& h, const std::vector<const void*>& g, const std::vector<const void*>& v,
               const std::vector<double>& w, double* bins_dev, hipStream_t st)
{
    const HamiltonianDev& H = h.H;
    const TermTables& T = h.host;
    const int npairs = (int)g.size();
    if (npairs == 0) return;
    require(npairs <= 64 && (int)v.size() == npairs && (int)w.size() == npairs, "gradient: bad pair list");
    // 1024-row tiles, 256 threads (the kernel's launch bound)
    const ApplyTuning tune{10, 256, 1};
    const ApplyPlan P = plan_apply(H.M, 1, SYK_C128, &tune);
    require(P.nt <= 256, "gradient: launch shape");
    const KRec* krec = krecs_for(H, P);
    auto it = h.grad_chunks.find(P.tile_bits);
    if (it == h.grad_chunks.end()) {
        std::vector<GChunk> c = make_grad_chunks(T.masks, T.bin_off, T.n_bins, P.tile_bits);
        std::unique_ptr<DevBuf> b(new DevBuf());
        b->ensure(c.size() * sizeof(GChunk));
        SYK_HIP(hipMemcpy(b->p, c.data(), c.size() * sizeof(GChunk), hipMemcpyHostToDevice));
        h.grad_nchunks[P.tile_bits] = (int)c.size();
        it = h.grad_chunks.emplace(P.tile_bits, std::move(b)).first;
    }
    GLayout L{};
    L.tile_bits = P.tile_bits;
    L.n_tiles = (uint32_t)(((uint64_t)1 << H.M) >> P.tile_bits);
    L.n_chunks = h.grad_nchunks[P.tile_bits];
    L.npairs = npairs;
    L.M = H.M;
    L.n_diag = H.n_diag;
    L.n_bins = T.n_bins;
    const int nblk = (int)std::min<uint32_t>(L.n_tiles, 512u);

    // pointer lists and weights: one small synchronous upload
    std::vector<uint64_t> host(3 * (size_t)npairs);
    for (int p = 0; p < npairs; ++p) {
        host[p] = (uint64_t)(uintptr_t)g[p];
        host[npairs + p] = (uint64_t)(uintptr_t)v[p];
        double wp = w[p];
        std::memcpy(&host[2 * npairs + p], &wp, sizeof(double));
    }
    void* dlist = h.ws.get("grad_lists", host.size() * sizeof(uint64_t));
    SYK_HIP(hipMemcpyAsync(dlist, host.data(), host.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    SYK_HIP(hipStreamSynchronize(st));
    const c128* const* gl = (const c128* const*)dlist;
    const c128* const* vl = gl + npairs;
    const double* wl = (const double*)(gl + 2 * npairs);

    double* partial = (double*)h.ws.get("grad_partial", (size_t)nblk * T.n_bins * 2 * sizeof(double));
    const size_t lds = ((size_t)1 << P.tile_bits) * sizeof(c128) + (size_t)kGradBinCap * 2 * sizeof(double);
    const GChunk* chunks = it->second->as<GChunk>();
    switch (P.rpt) {
    case 1: hipLaunchKernelGGL(k_grad_bins<1>, dim3(nblk), dim3(P.nt), lds, st, krec, chunks, H.dz, L, gl, vl, wl, partial); break;
    case 2: hipLaunchKernelGGL(k_grad_bins<2>, dim3(nblk), dim3(P.nt), lds, st, krec, chunks, H.dz, L, gl, vl, wl, partial); break;
    case 4: hipLaunchKernelGGL(k_grad_bins<4>, dim3(nblk), dim3(P.nt), lds, st, krec, chunks, H.dz, L, gl, vl, wl, partial); break;
    case 8: hipLaunchKernelGGL(k_grad_bins<8>, dim3(nblk), dim3(P.nt), lds, st, krec, chunks, H.dz, L, gl, vl, wl, partial); break;
    default: throw Error(SYK_EUNSUPPORTED, "gradient: launch shape");
    }
    SYK_HIP(hipGetLastError());
    const uint64_t n = 2 * T.n_bins;
    hipLaunchKernelGGL(k_bins_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, partial, nblk, n, bins_dev);
    SYK_HIP(hipGetLastError());
}

}  // namespace syk
