/*
 * syk.h -- C interface of the MI355X (gfx950) SYK library.
 *
 * The library computes, on one GPU, the matrix-free product of the q=4 SYK
 * Hamiltonian with state vectors and the Krylov-propagated correlators built
 * on it, following arXiv:2002.05725:
 *   H = sum_{i<j<k<l} J_ijkl chi_i chi_j chi_k chi_l            (main text, Eq. 1)
 * with {chi_i, chi_j} = delta_ij and the Majoranas mapped to N/2 qubits by
 * the Jordan-Wigner transformation of the SI (section "Jordan-Wigner
 * transformation"): chi_i = 2^{-1/2} (prod_{q<k} Z_q) X_k for even i and
 * 2^{-1/2} (prod_{q<k} Z_q) Y_k for odd i, k = floor(i/2), 0 <= i < N.
 *
 * Conventions shared by every call:
 *  - States.  A state of N Majoranas has dim = 2^(N/2) complex entries.  Qubit
 *    k is bit k of the basis index; Y = [[0,-i],[i,0]].  Entries are
 *    interleaved (re, im) pairs: complex128 (SYK_C128) or complex64 (SYK_C64).
 *  - Blocks.  nvec >= 1 states (columns) are stored one after another:
 *    entry (r, c) is element c*dim + r.  nvec = 1 is a plain vector.
 *    real_of_col (host, nvec entries, or NULL meaning all zeros) names the
 *    coupling realisation used by each column.
 *  - Couplings.  J holds n_real realisations back to back, each C(N,4) FP64
 *    values for the quartets i<j<k<l in lexicographic order.
 *  - Memory.  State pointers are device pointers owned by the caller, aligned
 *    to 16 bytes; the library never frees them.  Scalar results go to host
 *    pointers.  The handle owns its device tables and workspaces.
 *  - Streams.  Device work is enqueued on `stream` (NULL = default stream).
 *    Calls with host outputs synchronize that stream before returning.  One
 *    handle serves one stream at a time: concurrent calls on one handle race
 *    on its workspaces.
 *  - Errors.  Nothing throws or aborts across this interface.  Any status
 *    other than SYK_OK leaves outputs unspecified and handles valid;
 *    syk_last_error() gives a message for the calling thread's last failure.
 */
#ifndef SYK_H
#define SYK_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SYK_OK = 0,
    SYK_EINVAL = 1,          /* invalid argument */
    SYK_ENOMEM = 2,          /* device allocation failed */
    SYK_EHIP = 3,            /* HIP runtime error */
    SYK_EBREAKDOWN = 4,      /* non-finite norm inside a propagation */
    SYK_ENOTCONVERGED = 5,   /* a-posteriori error estimate above the requested tolerance */
    SYK_EUNSUPPORTED = 6     /* valid request the library does not handle */
} syk_status;

typedef enum { SYK_C128 = 0, SYK_C64 = 1 } syk_dtype;

typedef struct syk_terms_s* syk_terms;

/* Message for the calling thread's last non-OK status ("" if none). */
const char* syk_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int syk_version(void);

/*
 * Builds the Hamiltonian handle for N Majoranas (N even, 4 <= N <= 60) and
 * n_real >= 1 coupling realisations (J: host, n_real * C(N,4) finite FP64,
 * Eq. 1 with quartets in lexicographic order).  Each quartet becomes a Pauli
 * string on N/2 qubits; strings are grouped by the set of qubits they flip,
 * and the coefficient tables are uploaded to the current device.  *out must
 * be released with syk_destroy_terms.
 */
syk_status syk_build_terms(int N, int n_real, const double* J, syk_terms* out);

/* Releases the handle and every device buffer it owns.  NULL is accepted. */
syk_status syk_destroy_terms(syk_terms t);

/* Sizes of a handle; any output pointer may be NULL.  n_masks is the number
 * of distinct qubit-flip patterns (C(M,4) + C(M,2) + 1 for M = N/2 qubits). */
syk_status syk_terms_info(syk_terms t, int* N, int* n_real, int64_t* dim, int64_t* n_terms,
                          int64_t* n_masks);

/*
 * out = H psi column by column (matrix-free product, SI "Krylov subspace
 * methods": the product is formed on the fly from the symbolic terms).
 * psi, out: device, nvec columns of dim entries of `dtype`; out must not
 * overlap psi.  Columns are served by one launch per 64 columns.
 * Column c uses realisation real_of_col[c].  complex64 stores and multiplies
 * in FP32 and sums each row in FP64 across flip groups.
 */
syk_status syk_apply_H(syk_terms t, syk_dtype dtype, int nvec, const int32_t* real_of_col,
                       const void* psi, void* out, hipStream_t stream);

/*
 * syk_apply_H for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results as syk_apply_H (full space), with no hipMalloc, hipFree
 * or other allocation.  The buffers of the second, bit-rotated row layout
 * (psi copied in that layout and its partial output: 2 * min(nvec, 64) * dim
 * elements) come from a device scratch array of 128 MiB built into the library,
 * which each device the library runs on holds until the process ends (e.g.
 * N <= 44 in complex128 or N <= 46 in complex64 for one column; N < 30 needs
 * none).  Larger requests return SYK_EINVAL.  The handle's per-dtype tables and
 * the diagonal of H are built by its first syk_apply_H call of that dtype and
 * block width: without one, SYK_EINVAL.  Every call on a device shares that
 * device's scratch, so calls that overlap in time on one device (other streams
 * or other threads) race and give wrong results; nothing in the scratch has to
 * start at zero.  The handle's device must be the current device.
 */
syk_status syk_apply_H_noalloc(syk_terms t, syk_dtype dtype, int nvec, const int32_t* real_of_col,
                               const void* psi, void* out, hipStream_t stream);

/* Launch shape of apply_H for this handle (used by the autotuner): each
 * workgroup owns 2^tile_bits rows (0 = automatic, else at most 11; capped at
 * the number of qubits) with min(256, 2^tile_bits) threads, each thread up to 8
 * rows.  xcd_remap = 1 hands each of the 8 XCDs a contiguous range of row
 * tiles, 0 keeps the hardware's round-robin order.  cols_per_group = 2 lets one
 * workgroup serve two consecutive columns of a block that share a realisation
 * (the two typical states of one disorder draw), decoding every mask once for
 * both; it needs tile_bits 10 or 11 (or automatic, where smaller tiles fall
 * back to one column), and a launch whose columns do not pair up by
 * realisation runs one column per workgroup.  1: one column per workgroup.
 * 0 (automatic): two for complex64, one for complex128.  The product is the
 * same in every shape up to the order of floating-point sums (and bit for bit
 * between one and two columns per workgroup on the same tiles).  Other values give SYK_EINVAL and leave the setting
 * unchanged. */
syk_status syk_set_apply_tuning(syk_terms t, int tile_bits, int xcd_remap, int cols_per_group);

/* Cap on the device workspace a handle may hold (Krylov basis, estimator
 * vectors, Chebyshev stacks, checkpoints, rotated-layout copies of the
 * gradient), in bytes; 0 removes the cap (the default).  A call that would
 * grow the workspace beyond the cap returns SYK_ENOMEM before allocating and
 * leaves the handle valid.  Lowering the cap does not free what is held. */
syk_status syk_set_workspace_limit(syk_terms t, uint64_t bytes);

/* Kernel timing: while enabled, every apply_H call records a HIP event before
 * and after its kernel launches on the call's stream.  syk_timing_read waits
 * for the recorded events and returns the number of timed apply_H calls and
 * their summed duration in milliseconds; syk_timing_reset discards them.
 * Process-wide; off by default. */
syk_status syk_timing_enable(int on);
syk_status syk_timing_read(int64_t* launches, double* total_ms);
syk_status syk_timing_reset(void);

/* out = chi_a psi for one Majorana 0 <= a < N (SI Jordan-Wigner map), every
 * column.  out must not overlap psi. */
syk_status syk_apply_majorana(syk_terms t, syk_dtype dtype, int a, int nvec, const void* psi,
                              void* out, hipStream_t stream);

/* Column-wise <a_c | b_c> accumulated in FP64 with a fixed reduction order
 * (bitwise reproducible run to run).  out: host, nvec (re, im) pairs. */
syk_status syk_dot(syk_dtype dtype, int64_t dim, int nvec, const void* a, const void* b,
                   double* out, hipStream_t stream);

/* Krylov options.  m: basis vectors per step (2..64).  dt: real-time step
 * length.  tau_step: imaginary-time step length.  tol: if > 0, a step whose
 * a-posteriori error estimate exceeds tol makes the call return
 * SYK_ENOTCONVERGED (the result is still written). */
typedef struct {
    int m;
    double dt;
    double tau_step;
    double tol;
} syk_krylov_opts;

/*
 * psi <- exp(total * (z_re + i z_im) * H) psi, column by column, by Lanczos
 * steps (SI "Krylov subspace methods"): each step builds an m-vector Krylov
 * basis with two passes of classical Gram-Schmidt (FP64 inner products),
 * exponentiates the m x m tridiagonal projection in FP64 on the host, and
 * combines the basis.  The step length is dt for z_re == 0 and tau_step
 * otherwise; total >= 0 is cut into equal steps no longer than that.  A
 * Krylov space that becomes invariant ends the step early with the exact
 * result.  err_est (host, nvec, may be NULL) receives the largest step error
 * estimate beta_m |e_m^T e^{zT} e_1| ||psi|| per column.  With the environment
 * variable SYK_PROGRESS set, every finished step is reported on stderr (here
 * and in the estimators built on these steps).
 */
syk_status syk_krylov_expmv(syk_terms t, syk_dtype dtype, int nvec, const int32_t* real_of_col,
                            double z_re, double z_im, double total, const syk_krylov_opts* opts,
                            void* psi_inout, double* err_est, hipStream_t stream);

/*
 * Two-point function from a typical state (main text Eq. 2-3 with the
 * typicality formula of SI "Disorder averaging"):
 *   G(t) = <psi| rho^{1/2} chi_i(t) chi_i rho^{1/2} |psi> / Z,
 *   Z = <psi|rho|psi>, rho = e^{-beta H}, chi(t) = e^{iHt} chi e^{-iHt}.
 * t: host, nt >= 1 ascending values >= 0.  psi0: device, nvec columns.
 * G: host [nt][nvec] (re, im) pairs; G_R(t) = 2 Re G.  Z: host [nvec] or NULL.
 */
syk_status syk_two_point(syk_terms t, syk_dtype dtype, int i, double beta, const double* times,
                         int nt, int nvec, const int32_t* real_of_col, const void* psi0,
                         const syk_krylov_opts* opts, double* G, double* Z, hipStream_t stream);

/*
 * Regularized OTOC (main text Eq. 4) from a typical state, i != j:
 *   F(t) = Re <A^dag psi | A psi> / <psi|rho|psi>,
 *   A = rho^{1/8} chi_i(t) rho^{1/4} chi_j rho^{1/8},  rho = e^{-beta H},
 * i.e. Tr[...] in Eq. 4 is replaced by <psi|...|psi> (SI "Disorder
 * averaging") with the trace cut symmetrically.  Forward legs e^{-iHt} are
 * advanced incrementally from one output time to the next; each output time
 * then propagates back by its full t.
 * t: host, nt >= 1 ascending values >= 0.  psi0: device, nvec columns.
 * F: host [nt][nvec]; F_im (may be NULL): the imaginary part, a typicality
 * diagnostic; Z: host [nvec] or NULL.
 */
syk_status syk_otoc(syk_terms t, syk_dtype dtype, int i, int j, double beta, const double* times,
                    int nt, int nvec, const int32_t* real_of_col, const void* psi0,
                    const syk_krylov_opts* opts, double* F, double* F_im, double* Z,
                    hipStream_t stream);

/*
 * Unregularized OTOC (SI section "Unregularized OTOCs") from a typical state,
 * i != j:
 *   F_u(t) = Tr[W V W V rho] / Tr rho,  W = chi_i(t), V = chi_j, rho = e^{-beta H},
 * with the trace cut symmetrically around psi: <V W phi | W V phi> / <phi|phi>,
 * phi = rho^{1/2} psi.  Forward legs advance incrementally between output times;
 * each output time propagates back by its full t.  Same arguments and layouts
 * as syk_otoc: F [nt][nvec] the real part, F_im (may be NULL) the imaginary
 * part (nonzero in general), Z [nvec] or NULL.
 */
syk_status syk_otoc_unregularized(syk_terms t, syk_dtype dtype, int i, int j, double beta, const double* times,
                                  int nt, int nvec, const int32_t* real_of_col, const void* psi0,
                                  const syk_krylov_opts* opts, double* F, double* F_im, double* Z,
                                  hipStream_t stream);

/*
 * Imaginary-time Green's function (main text Eq. 2) from a typical state:
 *   G(tau) = <chi_i(tau) chi_i>_beta,  chi(tau) = e^{tau H} chi e^{-tau H},
 * estimated as ||e^{-tau H/2} chi_i e^{-(beta - tau) H/2} psi||^2 / <psi|rho|psi>
 * (real, G(0) = 1/2).  taus: host, ntau >= 1 ascending values in [0, beta]
 * (processed from the largest down, so e^{-(beta - tau) H/2} psi advances
 * incrementally).  psi0: device, nvec columns.  G: host [ntau][nvec];
 * Z: host [nvec] or NULL.  Imaginary legs use opts->tau_step.
 */
syk_status syk_imag_two_point(syk_terms t, syk_dtype dtype, int i, double beta, const double* taus, int ntau,
                              int nvec, const int32_t* real_of_col, const void* psi0, const syk_krylov_opts* opts,
                              double* G, double* Z, hipStream_t stream);

/*
 * Smallest and largest Ritz values of m Lanczos steps started from psi0
 * (device, one column): inner bounds on the spectrum of realisation 0 that
 * converge quickly at the edges.  Used to choose the Chebyshev interval; e_min
 * also estimates the ground-state energy.
 */
syk_status syk_spectrum_bounds(syk_terms t, syk_dtype dtype, int m, const void* psi0, double* e_min,
                               double* e_max, hipStream_t stream);

/*
 * Low-lying spectrum by Lanczos (the eigenvalue use of the Krylov method of
 * the SI, section "Krylov subspace methods"; the paper's validity criterion
 * counts the eigenstates within 1/beta of the ground state): m Lanczos steps
 * with two passes of classical Gram-Schmidt against the whole basis, started
 * from psi0 (device, one column, realisation 0).  evals (host, k): the k
 * lowest Ritz values of the m x m tridiagonal projection, ascending; resid
 * (host, k, may be NULL): their residual norms ||H y - theta y|| = beta_m
 * |s_m| (each Ritz value lies within its residual of an eigenvalue);
 * *n_found: how many were written (fewer than k if the Krylov space became
 * invariant, in which case the residuals are 0).  A starting vector reaches
 * one copy of each distinct level in exact arithmetic; in floating point
 * copies of degenerate levels can appear late.  Holds m state vectors of
 * workspace (2 <= m <= 512, 1 <= k <= m); the host eigen-decomposition of the
 * m x m projection costs O(m^3).
 */
syk_status syk_lowest_eigenvalues(syk_terms t, syk_dtype dtype, int m, int k, const void* psi0, double* evals,
                                  double* resid, int* n_found, hipStream_t stream);

/*
 * Fermion-parity sectors.  H conserves the parity of the qubit string (each
 * term flips an even number of qubits; SI, section "Jordan-Wigner
 * transformation"), and the paper evolves one sector.  A sector-s state
 * (s = 0 or 1, N >= 6) holds the 2^(N/2 - 1) rows r with popcount(r) = s mod 2:
 * entry u stands for the full row r = u + 2^(M-1) (parity(u) ^ s), M = N/2,
 * i.e. the top qubit is implied.  Blocks, dtypes, memory, streams and errors
 * as above.  The calls below are the full-space calls restricted to a sector:
 * apply_H, krylov_expmv, two_point, otoc, otoc_unregularized and
 * imag_two_point keep the sector of psi (Majoranas inside the estimators move
 * between sectors as they must); syk_apply_majorana_sector maps a sector_in
 * state to the other sector.  The handle builds each sector's tables on first
 * use (QUAD masks on the top qubit become two three-qubit masks, PAIR masks a
 * main and a parity part).
 */
syk_status syk_apply_H_sector(syk_terms t, syk_dtype dtype, int sector, int nvec, const int32_t* real_of_col,
                              const void* psi, void* out, hipStream_t stream);
syk_status syk_apply_majorana_sector(syk_terms t, syk_dtype dtype, int a, int sector_in, int nvec, const void* psi,
                                     void* out, hipStream_t stream);
syk_status syk_krylov_expmv_sector(syk_terms t, syk_dtype dtype, int sector, int nvec, const int32_t* real_of_col,
                                   double z_re, double z_im, double total, const syk_krylov_opts* opts,
                                   void* psi_inout, double* err_est, hipStream_t stream);
syk_status syk_two_point_sector(syk_terms t, syk_dtype dtype, int sector, int i, double beta, const double* times,
                                int nt, int nvec, const int32_t* real_of_col, const void* psi0,
                                const syk_krylov_opts* opts, double* G, double* Z, hipStream_t stream);
syk_status syk_otoc_sector(syk_terms t, syk_dtype dtype, int sector, int i, int j, double beta, const double* times,
                           int nt, int nvec, const int32_t* real_of_col, const void* psi0, const syk_krylov_opts* opts,
                           double* F, double* F_im, double* Z, hipStream_t stream);
syk_status syk_otoc_unregularized_sector(syk_terms t, syk_dtype dtype, int sector, int i, int j, double beta,
                                         const double* times, int nt, int nvec, const int32_t* real_of_col,
                                         const void* psi0, const syk_krylov_opts* opts, double* F, double* F_im,
                                         double* Z, hipStream_t stream);
syk_status syk_imag_two_point_sector(syk_terms t, syk_dtype dtype, int sector, int i, double beta, const double* taus,
                                     int ntau, int nvec, const int32_t* real_of_col, const void* psi0,
                                     const syk_krylov_opts* opts, double* G, double* Z, hipStream_t stream);

/* Chebyshev options.  Every propagator of the OTOC becomes a fixed polynomial
 * of this degree (2..256) in H~ = (H - e_center) / e_halfwidth: real time in
 * steps of dt (t_star must be a multiple of dt), each imaginary-time leg in
 * tau_steps equal steps.  The interval must enclose the spectrum and is held
 * fixed (it does not move with J).  checkpoint_every: the reverse sweep stores
 * one state every this many operations and recomputes the others. */
typedef struct {
    int degree;
    double dt;
    int tau_steps;
    int checkpoint_every;
    double e_center;
    double e_halfwidth;
    int keep_segment;   /* 1: during the reverse sweep, keep the Chebyshev vectors
                           of every step of a checkpoint segment from its
                           recomputation when (checkpoint_every x (degree + 1))
                           state vectors fit in half of the free device memory
                           (held by the handle afterwards); 0: recompute each
                           step's vectors again.  Results are identical. */
} syk_cheb_opts;

/*
 * F(t_star) of the regularized OTOC (same estimator and symmetric cut as
 * syk_otoc) with every propagator a Chebyshev polynomial (Jacobi-Anger
 * expansion e^{-ihH} = sum (2-d_n0)(-i)^n J_n(e_h h) e^{-i e_c h} T_n(H~);
 * e^{-tau H} with (-1)^n I_n(e_h tau) e^{-e_c tau}).  complex128, one column,
 * realisation 0.  F: host scalar.
 */
syk_status syk_cheb_otoc(syk_terms t, int i, int j, double beta, double t_star, const syk_cheb_opts* opts,
                         const void* psi0, double* F, hipStream_t stream);

/*
 * F(t_star) as in syk_cheb_otoc and dF/dJ_ijkl for every coupling (host, C(N,4)
 * in lexicographic order), exact for that polynomial forward: a reverse sweep
 * through every Chebyshev step (Clenshaw's recurrence for the adjoint states)
 * with states recomputed from checkpoints, and per-coupling reductions
 * Re <g| dH/dJ v> accumulated on the device.  Includes the derivative of
 * <psi|rho|psi>.  With the environment variable SYK_PROGRESS set, each
 * finished checkpoint segment of the reverse sweep is reported on stderr (and
 * every Krylov propagation step of any call, as for syk_krylov_expmv).
 */
syk_status syk_grad_couplings(syk_terms t, int i, int j, double beta, double t_star, const syk_cheb_opts* opts,
                              const void* psi0, double* F, double* dF_dJ, hipStream_t stream);

/*
 * The per-coupling reductions of the adjoint gradient on their own:
 * out[n] = sum_p w[p] Re <g_p| dH/dJ_n |v_p> for every coupling n (host array of
 * C(N,4) doubles, lexicographic quartet order), where dH/dJ_n is the Majorana
 * quartet chi_a chi_b chi_c chi_d of coupling n (Eq. 1, Jordan-Wigner form as
 * in apply_H).  It does not depend on the couplings' values.  g, v: host arrays
 * of npairs device pointers, each a complex128 vector of the full space
 * (2^(N/2) elements, 16-byte aligned, not modified); w: host array of npairs
 * finite weights; 1 <= npairs <= 64.  Synchronises the stream before returning.
 */
syk_status syk_coupling_overlaps(syk_terms t, int npairs, const void* const* g, const void* const* v,
                                 const double* w, double* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SYK_H */
