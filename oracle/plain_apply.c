/*
 * CPU checker for the SYK hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct evaluation of H|psi> for the q=4 SYK
 * Hamiltonian (main text, Eq. 1):
 *     H = sum_{i<j<k<l} J_ijkl chi_i chi_j chi_k chi_l,
 * with the Majoranas realised on N/2 qubits by the Jordan-Wigner map of the
 * SI (section "Jordan-Wigner transformation"):
 *     chi_i = 2^{-1/2} (prod_{q<k} Z_q) X_k   (i even),
 *     chi_i = 2^{-1/2} (prod_{q<k} Z_q) Y_k   (i odd),   k = floor(i/2).
 * The 2^{-1/2} makes {chi_i, chi_j} = delta_ij hold as the main text states;
 * the SI formula itself lists bare Pauli strings.  Qubit k is bit k of the
 * basis index and Y = [[0,-i],[i,0]].
 *
 * Each term is evaluated by composing its four Majorana maps on a basis
 * state, one map at a time; there are no mask tables, no grouping of terms
 * and nothing shared with the HIP library.  Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg load this file's library.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* chi_a acting on |s>: returns the new basis state and multiplies *amp. */
static inline uint64_t majorana_on_basis(int a, uint64_t s, cplx *amp)
{
    int k = a >> 1;
    uint64_t below = s & ((UINT64_C(1) << k) - 1);
    int neg = __builtin_popcountll(below) & 1;       /* Z string below qubit k */
    cplx f = M_SQRT1_2;
    if (a & 1) {                                      /* Y_k = i X_k Z_k */
        f *= I;
        neg ^= (int)((s >> k) & 1);
    }
    *amp *= neg ? -f : f;
    return s ^ (UINT64_C(1) << k);
}

/* Quartets in lexicographic order i<j<k<l over 0..N-1. */
static int64_t fill_quartets(int N, int32_t *q)
{
    int64_t n = 0;
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j)
            for (int k = j + 1; k < N; ++k)
                for (int l = k + 1; l < N; ++l) {
                    q[4 * n + 0] = i; q[4 * n + 1] = j;
                    q[4 * n + 2] = k; q[4 * n + 3] = l;
                    ++n;
                }
    return n;
}

static int64_t n_quartets(int N)
{
    return (int64_t)N * (N - 1) * (N - 2) * (N - 3) / 24;
}

/* <r| chi_i chi_j chi_k chi_l |s> with s = r ^ (flip of the quartet):
 * apply chi_l first, then chi_k, chi_j, chi_i. */
static inline cplx quartet_element(const int32_t *q, uint64_t r, uint64_t *src)
{
    uint64_t flip = (UINT64_C(1) << (q[0] >> 1)) ^ (UINT64_C(1) << (q[1] >> 1)) ^
                    (UINT64_C(1) << (q[2] >> 1)) ^ (UINT64_C(1) << (q[3] >> 1));
    uint64_t s = r ^ flip;
    cplx amp = 1.0;
    uint64_t t = s;
    t = majorana_on_basis(q[3], t, &amp);
    t = majorana_on_basis(q[2], t, &amp);
    t = majorana_on_basis(q[1], t, &amp);
    t = majorana_on_basis(q[0], t, &amp);
    if (t != r) amp = NAN;            /* cannot happen; poisons the result if it does */
    *src = s;
    return amp;
}

/* out[i] = (H psi)[rows[i]] for i < nrows.  psi has 2^(N/2) entries. */
int oracle_apply_rows(int N, const double *J, const cplx *psi,
                      const int64_t *rows, int64_t nrows, cplx *out)
{
    if (N < 4 || N > 62 || (N & 1)) return 1;
    int64_t nq = n_quartets(N);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)nq);
    if (!q) return 2;
    fill_quartets(N, q);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nrows; ++i) {
        uint64_t r = (uint64_t)rows[i];
        cplx acc = 0.0;
        for (int64_t n = 0; n < nq; ++n) {
            uint64_t s;
            cplx e = quartet_element(q + 4 * n, r, &s);
            acc += J[n] * e * psi[s];
        }
        out[i] = acc;
    }
    free(q);
    return 0;
}

/* out = H psi over all rows in [row_begin, row_end). */
int oracle_apply_range(int N, const double *J, const cplx *psi,
                       int64_t row_begin, int64_t row_end, cplx *out)
{
    if (row_end < row_begin) return 1;
    int64_t n = row_end - row_begin;
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!rows) return 2;
    for (int64_t i = 0; i < n; ++i) rows[i] = row_begin + i;
    int rc = oracle_apply_rows(N, J, psi, rows, n, out);
    free(rows);
    return rc;
}

/* out = chi_a psi (one Majorana, SI Jordan-Wigner map). */
int oracle_majorana(int N, int a, const cplx *psi, cplx *out)
{
    if (a < 0 || a >= N) return 1;
    int64_t D = INT64_C(1) << (N / 2);
#pragma omp parallel for
    for (int64_t s = 0; s < D; ++s) {
        cplx amp = 1.0;
        uint64_t r = majorana_on_basis(a, (uint64_t)s, &amp);
        out[r] = amp * psi[s];
    }
    return 0;
}

/*
 * Sparse form of H for repeated products at moderate N.  The matrix element
 * <r|H|s> is the sum of J_n <r|Q_n|s> over the quartets Q_n whose qubit flip
 * equals r^s.  The set of distinct flips does not depend on the row, so row r
 * holds exactly one entry per distinct flip f, at column r^f.
 * row_ptr has D+1 entries; cols/vals have D * n_flips entries, where n_flips
 * is returned by oracle_sparse_nflips.
 */
static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

static uint64_t quartet_flip(const int32_t *q)
{
    return (UINT64_C(1) << (q[0] >> 1)) ^ (UINT64_C(1) << (q[1] >> 1)) ^
           (UINT64_C(1) << (q[2] >> 1)) ^ (UINT64_C(1) << (q[3] >> 1));
}

static int64_t distinct_flips(int N, const int32_t *q, int64_t nq, uint64_t **out)
{
    uint64_t *f = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nq);
    if (!f) return -1;
    for (int64_t n = 0; n < nq; ++n) f[n] = quartet_flip(q + 4 * n);
    qsort(f, (size_t)nq, sizeof(uint64_t), cmp_u64);
    int64_t nu = 0;
    for (int64_t n = 0; n < nq; ++n)
        if (n == 0 || f[n] != f[n - 1]) f[nu++] = f[n];
    *out = f;
    (void)N;
    return nu;
}

int64_t oracle_sparse_nflips(int N)
{
    if (N < 4 || N > 62 || (N & 1)) return -1;
    int64_t nq = n_quartets(N);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)nq);
    if (!q) return -1;
    fill_quartets(N, q);
    uint64_t *f = NULL;
    int64_t nu = distinct_flips(N, q, nq, &f);
    free(q);
    free(f);
    return nu;
}

int oracle_sparse_H(int N, const double *J, int64_t *row_ptr, int64_t *cols, cplx *vals)
{
    if (N < 4 || N > 40 || (N & 1)) return 1;
    int64_t D = INT64_C(1) << (N / 2);
    int64_t nq = n_quartets(N);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)nq);
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)nq);
    if (!q || !slot) { free(q); free(slot); return 2; }
    fill_quartets(N, q);
    uint64_t *uf = NULL;
    int64_t nu = distinct_flips(N, q, nq, &uf);
    if (nu < 0) { free(q); free(slot); return 2; }
    for (int64_t n = 0; n < nq; ++n) {          /* slot of each quartet's flip */
        uint64_t f = quartet_flip(q + 4 * n);
        int64_t lo = 0, hi = nu - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (uf[mid] < f) lo = mid + 1; else hi = mid;
        }
        slot[n] = lo;
    }
    for (int64_t r = 0; r <= D; ++r) row_ptr[r] = r * nu;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < D; ++r) {
        cplx *v = vals + r * nu;
        int64_t *c = cols + r * nu;
        for (int64_t u = 0; u < nu; ++u) { v[u] = 0.0; c[u] = (int64_t)((uint64_t)r ^ uf[u]); }
        for (int64_t n = 0; n < nq; ++n) {
            uint64_t s;
            cplx e = quartet_element(q + 4 * n, (uint64_t)r, &s);
            v[slot[n]] += J[n] * e;
        }
    }
    free(q); free(slot); free(uf);
    return 0;
}

/* y = A x for the sparse form above. */
int oracle_sparse_matvec(int64_t D, const int64_t *row_ptr, const int64_t *cols,
                         const cplx *vals, const cplx *x, cplx *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < D; ++r) {
        cplx acc = 0.0;
        for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) acc += vals[e] * x[cols[e]];
        y[r] = acc;
    }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
