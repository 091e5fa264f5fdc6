/*
 * dmd_stream.h -- C ABI of the MI355X (gfx950) streaming method-of-snapshots
 * dynamic mode decomposition library (libdmdstream.so).
 *
 * Method: Pendergrass, Kutz, Brunton, "Streaming GPU Singular Value and
 * Dynamic Mode Decompositions" (arXiv:1612.07875).
 *
 *   * A stream keeps a window of the last m+1 snapshots x_{t-m} .. x_t, each
 *     of length n.  X is the first m of them and X' the last m (Sec. 2,
 *     the data matrices X and X'; Algorithm 2 takes the (m+1)-column window).
 *   * Every push computes only the new snapshot's inner products with the
 *     window and reuses all others (Sec. 3.1, streaming method of snapshots;
 *     Algorithm 1).  One Gram of the whole (m+1)-column window serves both
 *     X^* X (Algorithm 1's xtx) and X^* X' (Algorithm 2's xty).
 *   * Once the window is full the small solves run in FP64 on the GPU:
 *     eig of X^* X -> sigma, V (Sec. 2.1); A~ = Sigma^-1 V^* X^* X' V Sigma^-1
 *     (Eq. Atilde with U = X V Sigma^-1 never formed, Sec. 3.4);
 *     A~ W = W Lambda (Sec. 2.2).
 *   * On request the tall-skinny projections run on the GPU:
 *     modes Phi = X' V Sigma^-1 W (Eq. Phi) and POD modes U = X V Sigma^-1
 *     (Sec. 2.1, step 2).
 *   * Complex snapshots given in compressed sparse form (sorted indices and
 *     complex64 values) use sparse inner products; SVD and DMD are invariant
 *     under the unitary Fourier transform, so Fourier coefficients can be
 *     processed directly (Sec. 3.5).
 *
 * Readings fixed by this library where the paper is silent:
 *   * Truncation to the r leading singular values (exact DMD of Tu et al.,
 *     cited in Sec. 2.2).  Singular values at or below rcond * sigma_1 are
 *     not resolvable by a Gram accumulated in FP64; only the leading
 *     r_eff <= r are then used and calls report DMD_W_RANK.
 *   * Conjugate transposes throughout (complex snapshots give a Hermitian Gram).
 *   * sigma is sorted descending and V's columns are permuted alike.
 *   * Eigenvalues are sorted by descending |lambda|, ties by ascending
 *     arg(lambda).  Columns of V and W have unit 2-norm and their entry of
 *     largest modulus (lowest index on ties) real and positive; Phi inherits W.
 *
 * Conventions of this ABI:
 *   * Every function returns an int status: DMD_OK (0), a positive warning,
 *     or a negative error.  No C++ exception crosses the ABI.  The message of
 *     the calling thread's last error is returned by dmd_last_error().
 *   * "stream" arguments are hipStream_t values passed as void* (NULL = the
 *     null stream).  Work on one handle is serialised in call order across
 *     all streams it is given, with two exceptions that read only what the
 *     next push leaves alone: dmd_stream_modes of a dense stream and
 *     dmd_stream_block_modes may run beside the push that follows them.
 *   * Device pointers are HIP device allocations of the current device of
 *     the handle; host pointers are ordinary host memory.
 *   * The library owns every device buffer it allocates (ring of snapshots,
 *     Gram, workspaces); the caller owns all input and output buffers and
 *     must keep inputs valid until the call's work completes
 *     (dmd_stream_sync, or any call that returns host results).
 *   * A handle is not thread-safe: calls on one handle must not overlap.
 *   * Matrices are column-major.  Complex values are interleaved (re, im)
 *     pairs: complex64 = 2 x float, complex128 = 2 x double.
 */
#ifndef DMD_STREAM_H
#define DMD_STREAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define DMD_OK              0
#define DMD_W_RANK          1   /* fewer than r singular values resolvable; r_eff < r */
#define DMD_E_INVAL        -1   /* bad argument (null pointer, size, alignment, index) */
#define DMD_E_NOMEM        -2   /* device or pinned-host allocation failed */
#define DMD_E_NOT_READY    -3   /* fewer than m+1 snapshots pushed, or no solve yet */
#define DMD_E_NONFINITE    -4   /* a pushed snapshot had a non-finite inner product; it
                                   was rejected and the window left unchanged */
#define DMD_E_CONVERGENCE  -5   /* an eigensolver hit its iteration limit */
#define DMD_E_DEVICE       -6   /* a HIP runtime call failed */
#define DMD_E_UNSUPPORTED  -7   /* valid request not supported for this dtype/precision */

/* ------------------------------------------------------------ options */
typedef enum {
    DMD_F32     = 0,  /* real float32 snapshots */
    DMD_F64     = 1,  /* real float64 snapshots */
    DMD_C64_CSR = 2   /* complex64 snapshots in sparse form (dmd_stream_push_csr) */
} dmd_dtype_t;

typedef enum {
    DMD_PREC_DEFAULT = 0, /* FP64 for F64 data, FP32 for F32 / C64 data          */
    DMD_PREC_FP32    = 1, /* dense contractions in FP32 (MFMA), FP32 accumulation */
    DMD_PREC_BF16X3  = 2, /* F32 data only: dense contractions as three BF16 MFMA
                             products (hi*hi + hi*lo + lo*hi), FP32 accumulation:
                             the projections (modes, POD modes, the modes of a
                             block push, grouped batch projections) and the
                             whole-window Gram (dmd_stream_load_window,
                             dmd_stream_resync)                                   */
    DMD_PREC_FP64    = 3  /* F32 data: coefficients, projections and the
                             whole-window Gram in FP64                            */
} dmd_precision_t;

typedef enum {
    DMD_EIG_DEFAULT = 0,  /* DMD_EIG_TRIDIAG, or DMD_EIG_JACOBI when warm_start is on   */
    DMD_EIG_JACOBI  = 1,  /* cyclic two-sided Jacobi, all m eigenvectors               */
    DMD_EIG_TRIDIAG = 2   /* Householder tridiagonalization, multisection for all
                             eigenvalues, twisted factorizations for the r leading
                             eigenvectors (O(m) dependent steps; no warm start)        */
} dmd_eig_solver_t;

typedef struct {
    int32_t dtype;       /* dmd_dtype_t (default DMD_F32)                           */
    int32_t precision;   /* dmd_precision_t for the dense contractions (the
                            tall-skinny projections and the whole-window Gram);
                            the per-frame inner products and the block Gram of a
                            block push always accumulate in FP64, and the small
                            solves always run in FP64                               */
    int32_t max_nnz;     /* DMD_C64_CSR: capacity per snapshot (0 = n)              */
    int32_t max_sweeps;  /* Jacobi sweep limit (0 = 40)                              */
    int32_t max_qr_iter; /* Hessenberg-QR iterations per eigenvalue (0 = 60)         */
    int32_t auto_solve;  /* 1 (default): a push into a full window also runs the
                            small solves; 0: only dmd_stream_solve runs them        */
    double  rcond;       /* rank cut-off relative to sigma_1 (< 0: default
                            10 * sqrt(2^-52) ~ 1.5e-7; 0: keep all nonzero)        */
    double  tol;         /* Jacobi stopping threshold: rotate while
                            |a_pq| > tol * sqrt(|a_pp a_qq|) (0 = 1e-15)            */
    int32_t warm_start;  /* 1: start each Jacobi solve from the previous solve's
                            eigenvectors, rows shifted by one window position
                            (consecutive solves then depend on each other); 0
                            (default): start from the identity                      */
    int32_t max_block;   /* largest k of dmd_stream_push_block, 1 .. 64 (0 = 1);
                            dense streams only.  For max_block > 1 the ring keeps
                            2 max_block spare slots, and there are max_block - 1
                            extra solve workspaces                               */
    int32_t eig_solver;  /* dmd_eig_solver_t for the symmetric eig of X^* X       */
    int32_t buildup;     /* 1: build-up start (Sec. 5): while the window fills, a
                            window of c >= 3 snapshots is solved as a window of
                            m' = c - 1 columns (X = its first c - 1 snapshots,
                            X' = its last c - 1, rank <= min(r, m')), so results
                            exist from the third push on; sigma and the rows of
                            V past m' read zero.  Dense streams with
                            max_block = 1 only.  0 (default): DMD_E_NOT_READY
                            until the window holds m + 1 snapshots              */
    int32_t reserved[4]; /* must be zero                                             */
} dmd_opts_t;

typedef struct dmd_stream dmd_stream_t;

/* Fill *opts with the defaults listed above.  DMD_E_INVAL if opts is NULL. */
int dmd_opts_init(dmd_opts_t* opts);

/* ------------------------------------------------------------ lifecycle */

/* Create a stream with snapshot length n, window m (X has m columns, the
 * window holds m+1 snapshots) and truncation rank r on the current HIP device.
 * Requires n >= 1, 2 <= m <= 256, 1 <= r <= min(m, 32); for DMD_C64_CSR also
 * 1 <= max_nnz <= n.  opts may be NULL (defaults).  Allocates the ring of
 * snapshots (m+2 slots of n elements, or m+1+2B slots for block streams,
 * B = opts->max_block: the window, the slots being filled and the columns of
 * the previous block's windows), the FP64 Gram over those slots and the solve
 * workspaces, all zeroed.
 * Errors: DMD_E_INVAL, DMD_E_NOMEM, DMD_E_DEVICE.  *out is NULL on error. */
int dmd_stream_create(int64_t n, int32_t m, int32_t r, const dmd_opts_t* opts,
                      dmd_stream_t** out);

/* Device memory in bytes that dmd_stream_create(n, m, r, opts) would allocate
 * (the device_bytes of dmd_stream_info right after creation), for admission
 * by HBM footprint before anything is allocated.  Host only: allocates
 * nothing and needs no device.  Same argument checks and errors as
 * dmd_stream_create (DMD_E_INVAL, DMD_E_UNSUPPORTED); *bytes is 0 on error. */
int dmd_stream_footprint(int64_t n, int32_t m, int32_t r, const dmd_opts_t* opts, int64_t* bytes);

/* Wait for all work of the handle, then free everything it owns.  NULL is a no-op. */
int dmd_stream_destroy(dmd_stream_t* h);

/* Wait for all work of the handle.  Returns DMD_E_NONFINITE once if pushes
 * were rejected since the last report, else DMD_OK. */
int dmd_stream_sync(dmd_stream_t* h);

/* Empty the window (the next push starts a new one).  Stream-ordered. */
int dmd_stream_reset(dmd_stream_t* h, void* stream);

/* ------------------------------------------------------------ ingest (Sec. 3.1) */

/* Append one dense snapshot (n elements of the stream's dtype, 4-byte aligned
 * for F32, 8-byte for F64) -- the new column that Sec. 3 appends on the right
 * of the window while the oldest leaves on the left.  x may be device memory
 * of the stream's device (read in place) or host memory, pageable or pinned
 * (copied on `stream` into a staging buffer of n elements that the first such
 * push allocates and the handle owns; device_bytes grows by it).  Either way
 * the caller keeps x valid until the stream reaches the push (a later
 * synchronising call).  Enqueues on `stream`:
 *   the copy of x into the ring, its n-length inner products with every
 *   snapshot that stays in the window and with itself (FP64 accumulation,
 *   fixed reduction order: bitwise reproducible), the Gram update (oldest
 *   snapshot dropped, new row and column written), and -- when the window is
 *   full and auto_solve is on -- the FP64 small solves.
 * A snapshot whose inner products are not finite is rejected on the device:
 * the window, Gram and results stay as they were and the next synchronising
 * call returns DMD_E_NONFINITE.  Asynchronous: returns before the work runs.
 * Errors: DMD_E_INVAL (NULL, wrong dtype, misaligned), DMD_E_DEVICE. */
int dmd_stream_push(dmd_stream_t* h, const void* x, void* stream);

/* Append one sparse complex snapshot: nnz entries, idx (int32) strictly
 * increasing in [0, n), val (complex64); device or host memory as for
 * dmd_stream_push (host data staged in buffers of max_nnz entries allocated
 * by the first such push).  Only for DMD_C64_CSR streams;
 * 0 <= nnz <= max_nnz.  Index validity is checked on the device: a snapshot
 * with unsorted or out-of-range indices is rejected like a non-finite one
 * (DMD_E_INVAL at the next synchronising call).  Otherwise as dmd_stream_push. */
int dmd_stream_push_csr(dmd_stream_t* h, int32_t nnz, const int32_t* idx,
                        const void* val, void* stream);

/* Spatial -> Fourier ingest for sparse streams (Sec. 3.5: SVD and DMD are
 * unchanged by a unitary change of basis, so dense frames may enter the
 * sparse path as Fourier coefficients).  Setup: h is a DMD_C64_CSR stream
 * with n = height x width; the support is the nkeep (1 <= nkeep <= max_nnz)
 * bins of the height x width 2-D DFT with the smallest ky^2 + kx^2, the
 * wavenumbers signed in FFT order (bin k of N is k for k < (N+1)/2, else
 * k - N), ties broken by the flattened index ky * width + kx; width <= 16384.
 * Computes the support and the tables on the host and allocates the
 * device buffers (a later call replaces them, after waiting for earlier
 * pushes).  Errors: DMD_E_INVAL (sizes), DMD_E_UNSUPPORTED (dense stream),
 * DMD_E_NOMEM, DMD_E_DEVICE. */
int dmd_stream_fourier_setup(dmd_stream_t* h, int32_t height, int32_t width, int32_t nkeep);

/* The support of the Fourier ingest: *nkeep receives its size and, when idx
 * is not NULL (host, cap >= nkeep entries), idx the flattened indices in
 * increasing order -- the index order of the coefficients the stream holds
 * and of the rows of its (dense, n-long) modes.  DMD_E_NOT_READY before
 * dmd_stream_fourier_setup. */
int dmd_stream_fourier_support(dmd_stream_t* h, int32_t* idx, int32_t cap, int32_t* nkeep);

/* Push one spatial frame: `frame` is height x width FP32 on the device,
 * row-major with row stride ld_row >= width elements (4-byte aligned).
 * Enqueues on `stream` the unitary 2-D DFT at the support points
 * ((height width)^-1/2 sum_y sum_x x[y][x] e^{-2 pi i (ky y / height + kx x / width)},
 * FP64 sums, stored as complex64) and then the sparse push of those
 * coefficients (dmd_stream_push_csr).  Asynchronous.  Errors: DMD_E_NOT_READY
 * (no setup), DMD_E_INVAL, DMD_E_DEVICE, and those of dmd_stream_push_csr. */
int dmd_stream_push_fourier(dmd_stream_t* h, const float* frame, int64_t ld_row, void* stream);

/* Append k dense snapshots at once (Sec. 5, updating with more than one new
 * column at a time): X_new is n x k in the stream's dtype (device,
 * column-major, leading dimension ldx >= n), 1 <= k <= opts.max_block.
 * Enqueues on `stream`: one pass over the window and X_new that computes the
 * (count+k) x k block of new inner products on the matrix cores (FP64
 * products and sums, fixed reduction order) and copies X_new into the ring,
 * the Gram update, and -- with auto_solve on -- the FP64 small solves of every
 * window the k single pushes would pass through, run side by side (one CU
 * each).  Afterwards the stream is in the state k dmd_stream_push calls in
 * column order would leave (up to the summation order of the inner
 * products); dmd_stream_eigs/svd/atilde/modes describe the last window and
 * dmd_stream_block_eigs returns every window's eigenvalues.
 * Unlike k single pushes, a non-finite inner product anywhere in the block
 * rejects the whole block (window, Gram and results unchanged; DMD_E_NONFINITE
 * at the next synchronising call).  With FP32 data and coefficients the
 * inputs of dmd_stream_block_modes (coefficients in the projection kernel's
 * fragment order, ring position, ranks) are packed right after the solves, in
 * one of two buffers used in turn.  Ordered after all earlier calls on the
 * handle except the dmd_stream_block_modes of the previous block push, which
 * reads nothing this push writes.  Asynchronous.
 * Errors: DMD_E_INVAL (NULL, k out of range, ldx < n, misaligned),
 * DMD_E_UNSUPPORTED (sparse stream), DMD_E_DEVICE. */
int dmd_stream_push_block(dmd_stream_t* h, const void* X_new, int64_t ldx,
                          int32_t k, void* stream);

/* Results of every window of the latest push when it was a block push with
 * auto_solve on (waits for its solves).  *k receives the block size k.  For
 * window w < k -- the window that ends at the block's snapshot w, so window
 * k-1 is the current one -- status[w] receives its status (DMD_OK,
 * DMD_W_RANK, DMD_E_NOT_READY if the window was not full yet,
 * DMD_E_CONVERGENCE, or DMD_E_NONFINITE for every window of a rejected block),
 * r_eff[w] its rank, and lam_re, lam_im and sigma (host, k x ld row-major,
 * ld >= r) its r_eff[w] leading eigenvalues and singular values at offset
 * w * ld.  Any pointer except k may be NULL.  Returns DMD_E_NOT_READY if the
 * latest push was not such a block push, otherwise the status of the current
 * window as dmd_stream_eigs does. */
int dmd_stream_block_eigs(dmd_stream_t* h, int32_t* k, double* lam_re, double* lam_im,
                          double* sigma, int64_t ld, int32_t* r_eff, int32_t* status);

/* DMD modes (Eq. Phi) of every window of the latest block push, each as
 * dmd_stream_modes writes it: window w's Phi (n x r_eff[w] complex, column j
 * at phi + w * ldw + j * ld complex elements; complex64, or complex128 for
 * DMD_F64 streams and DMD_PREC_FP64) into the device buffer phi, ld >= n,
 * ldw >= ld * r.  Windows that were not full, not solved, or belong to a
 * rejected block are left untouched.  For FP32 data and coefficients one pass
 * over the ring serves all k windows, reading only the ring columns of the
 * block's windows and the inputs packed by the push, so that on another
 * stream than the pushes it runs beside the next block push (whose Gram
 * update and solves then overlap it); the block push after that, and every
 * other later call, is ordered after it.  Stream-ordered; does not wait.
 * DMD_E_NOT_READY if the latest push was not a block push with auto_solve on. */
int dmd_stream_block_modes(dmd_stream_t* h, void* phi, int64_t ld, int64_t ldw, void* stream);

/* ------------------------------------------------------------ small solves (Alg. 1-2) */

/* Run the FP64 small solves for the current window on `stream` (not needed
 * when auto_solve is on). */
int dmd_stream_solve(dmd_stream_t* h, void* stream);

/* Host results of the latest solve (waits for it).  Each of lam_re, lam_im,
 * sigma may be NULL; otherwise it receives r_eff values (sigma: the r_eff
 * leading singular values of X).  *r_eff (may be NULL) receives the rank used.
 * Returns DMD_OK, DMD_W_RANK (r_eff < r), DMD_E_NOT_READY (window not full or
 * no solve yet), DMD_E_NONFINITE, DMD_E_CONVERGENCE. */
int dmd_stream_eigs(dmd_stream_t* h, double* lam_re, double* lam_im, double* sigma,
                    int32_t* r_eff);

/* Host copies of the latest solve's matrices (waits for it).  Any pointer may
 * be NULL.  sigma: all m singular values of X, descending.  V: m x r_eff
 * (leading dimension ldv >= m; complex128 for DMD_C64_CSR, else double).
 * Atilde: r_eff x r_eff (lda >= r_eff; complex128 for DMD_C64_CSR, else double).
 * W: r_eff x r_eff complex128 (ldw >= r_eff).  Status as dmd_stream_eigs. */
int dmd_stream_svd(dmd_stream_t* h, double* sigma, double* V, int64_t ldv, int32_t* r_eff);
int dmd_stream_atilde(dmd_stream_t* h, double* Atilde, int64_t lda, double* W, int64_t ldw,
                      int32_t* r_eff);

/* Host copy of the Gram of the current window in window order (oldest first):
 * G[i + j*ldg] = <x_i, x_j> = x_i^* x_j for 0 <= i, j < *ncols, where *ncols
 * (m+1 once full) is written first.  ldg >= m+1.  complex128 for DMD_C64_CSR,
 * else double.  Waits for the handle's work. */
int dmd_stream_gram(dmd_stream_t* h, double* G, int64_t ldg, int32_t* ncols);

/* ------------------------------------------------------------ checkpoint / resume (Sec. 5) */

/* A checkpoint holds what the streaming update keeps between pushes: the
 * window's snapshots (in window order), its Gram (FP64, window order) and the
 * stream's counters, in a versioned host-memory format; solve results are
 * recomputed on restore.  dmd_stream_checkpoint_bytes gives the size for the
 * current window (waits for the handle's state-changing work).  Errors:
 * DMD_E_INVAL (NULL), DMD_E_DEVICE. */
int dmd_stream_checkpoint_bytes(dmd_stream_t* h, int64_t* bytes);

/* Write a checkpoint of h into the host buffer buf (bytes >=
 * dmd_stream_checkpoint_bytes).  Waits for the handle's state-changing work;
 * blocks until written.  Errors: DMD_E_INVAL (NULL, buffer too small),
 * DMD_E_DEVICE. */
int dmd_stream_save(dmd_stream_t* h, void* buf, int64_t bytes);

/* Replace the window of h by the checkpoint in buf: h must have been created
 * with the same dtype, n, m and r (sparse streams: max_nnz at least the
 * checkpoint's largest snapshot); its options may differ.  Ordered after
 * h's earlier work on any stream; writes the window and Gram from host memory
 * (blocking), then, with auto_solve on, enqueues the solves on `stream`.
 * Pushes after a restore give the results the saved stream would give
 * (bitwise: same kernels on the same values), except that a warm-started
 * Jacobi solve starts cold once.  Errors: DMD_E_INVAL (NULL, not a
 * checkpoint, other shape, truncated or inconsistent), DMD_E_DEVICE. */
int dmd_stream_restore(dmd_stream_t* h, const void* buf, int64_t bytes, void* stream);

/* ------------------------------------------------------------ projections (Eq. Phi, Sec. 2.1) */

/* DMD modes Phi = X' V Sigma^-1 W of the latest solve into `phi` (device,
 * n x r_eff complex, leading dimension ld >= n, column order = eigenvalue
 * order).  complex128 for DMD_F64 streams or DMD_PREC_FP64, else complex64.
 * For DMD_C64_CSR streams rows outside the window's union support are zero.
 * Dense streams: every solve leaves a copy of its state and mode
 * coefficients, and the projection reads that copy and the solve's window
 * only, so that on another stream than the pushes it runs beside the next
 * push (its Gram update and solves overlap it); the push after that, and
 * every other later call, is ordered after it.  Stream-ordered; does not
 * wait.  DMD_E_NOT_READY if no solve was enqueued. */
int dmd_stream_modes(dmd_stream_t* h, void* phi, int64_t ld, void* stream);

/* POD modes U = X V Sigma^-1 (n x r_eff, leading dimension ld >= n; double for
 * DMD_F64 or DMD_PREC_FP64, complex64 for DMD_C64_CSR, else float). */
int dmd_stream_pod(dmd_stream_t* h, void* U, int64_t ld, void* stream);

/* ------------------------------------------------------------ amplitudes, background (Sec. 3.3, Alg. 3) */

/* Mode amplitudes of the latest solve (waits for it): b = (W Lambda)^-1
 * alpha_1, alpha_1 = Sigma_r V_r^* e_1 the POD coefficients of the window's
 * first snapshot x_1 (so that x_1 ~ Phi b, Sec. 3.3), and the background mode
 * index argmin_i |log lambda_i| (Algorithm 3; lowest index on ties), in
 * eigenvalue order.  b_re, b_im (host, r_eff values each) and bg_index may be
 * NULL; *bg_index is -1 when there is no solve.  Status as dmd_stream_eigs. */
int dmd_stream_amplitudes(dmd_stream_t* h, double* b_re, double* b_im, int32_t* bg_index,
                          int32_t* r_eff);

/* Background subtraction of the newest snapshot x_{m+1} (Algorithm 3, the
 * streaming branch): with i the background mode, the background is
 * l = b_i lambda_i^m phi_i and the foreground s = x_{m+1} - |l| (elementwise
 * modulus).  Writes s into fg and |l| into bg (device, n values each; either
 * may be NULL, not both): float for FP32 projections, double for DMD_F64
 * streams and DMD_PREC_FP64.  One pass over X' (m n elements).  Dense streams
 * only (DMD_E_UNSUPPORTED otherwise).  Stream-ordered; does not wait; leaves
 * the outputs untouched while no full window has been solved. */
int dmd_stream_background(dmd_stream_t* h, void* fg, void* bg, void* stream);

/* ------------------------------------------------------------ bulk Gram (Alg. 1 first step) */

/* Replace the window by the k = ncols snapshots in X (device, n x k
 * column-major, leading dimension ldx >= n, 1 <= k <= m+1, stream dtype;
 * dense dtypes only) and compute their whole Gram at once (Algorithm 1's
 * first step) with the MFMA Gram kernel in the stream's precision. */
int dmd_stream_load_window(dmd_stream_t* h, const void* X, int64_t ldx, int32_t ncols,
                           void* stream);

/* Recompute the whole Gram of the current window from the snapshots held in
 * the ring (MFMA Gram kernel, stream's precision), e.g. to compare precisions. */
int dmd_stream_resync(dmd_stream_t* h, void* stream);

/* Stateless whole Gram of a window (Algorithm 1's first step; Sec. 2.1
 * step 1): G = X^* X for the k = ncols columns of X, without a stream
 * handle.  X: device, n x k column-major FP32 (dtype DMD_F32) or FP64
 * (DMD_F64), leading dimension ldx >= n, 16-byte aligned with ldx * element
 * size a multiple of 16; 1 <= k <= 257.  G: device, k x k FP64 column-major,
 * leading dimension ldg >= k, both triangles written (rows/columns past k and
 * the padding untouched).  precision: the products of the MFMA Gram kernel
 * (DMD_PREC_FP64 or DMD_F64 data: FP64 products and sums; DMD_PREC_FP32 /
 * DEFAULT with FP32 data: FP32 products and in-tile sums; DMD_PREC_BF16X3:
 * split-BF16 products, FP32 in-tile sums); row-split tiles are always summed
 * in FP64 in a fixed order (bitwise reproducible).  Stream-ordered on
 * `stream`: the kernel's partial tiles (16.4 MB at most) are allocated with
 * hipMallocAsync and freed with hipFreeAsync on it; X and G belong to the
 * caller.  Errors: DMD_E_INVAL (NULL, sizes, alignment), DMD_E_UNSUPPORTED
 * (BF16X3 with FP64 data), DMD_E_NOMEM, DMD_E_DEVICE. */
int dmd_window_gram(const void* X, int64_t ldx, int64_t n, int32_t ncols, int32_t dtype,
                    int32_t precision, double* G, int64_t ldg, void* stream);

/* dmd_window_gram without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, checks, kernels and results as
 * dmd_window_gram (bitwise equal); the kernel's partial tiles go to a fixed
 * device array of the library (17,203,200 bytes, enough for the largest
 * window, ncols = 257), one per device, held until the process ends.  Its
 * address on a device is looked up on the first call there (on the device
 * that runs `stream`).  No hipMalloc, hipFree or allocating library call.
 * Every call on one device shares that array: calls that overlap on one
 * device (different streams, or different host threads) race and may return
 * wrong results; order them on one stream or synchronize between them.
 * Errors: as dmd_window_gram (DMD_E_INVAL also for a window whose partial
 * tiles would exceed the array), and DMD_E_DEVICE if the array's address
 * cannot be looked up. */
int dmd_window_gram_noalloc(const void* X, int64_t ldx, int64_t n, int32_t ncols, int32_t dtype,
                            int32_t precision, double* G, int64_t ldg, void* stream);

/* ------------------------------------------------------------ launch-shape tuning */

/* Launch shapes of a dense stream shape, chosen by measurement. */
typedef struct {
    int32_t gram_iter;   /* one-frame Gram pass: 16-byte loads per thread and column in a
                            workgroup's slab of rows (1, 2 or 4; fewer, larger slabs) */
    int32_t proj_form;   /* block projection (FP32 block streams): 0 built-in rule,
                            1 one product per window, 2 two windows per product,
                            3 one banded product of all windows */
    double gram_us;      /* measured one-frame Gram pass (push without solves) of the choice */
    double step_us;      /* measured pipelined block step of the chosen form, 0 if not timed */
    int32_t reserved[4];
} dmd_tuning_t;

/* Measure and record the launch shapes for streams of shape (n, m, r, opts)
 * (dense dtypes; no sparse tuning).  Runs on `stream` with streams and
 * buffers of its own, filled with uniform random numbers (up to a block's
 * modes, k r n complex64 values, for block streams):
 *   * the one-frame Gram pass in each slab form, as back-to-back pushes;
 *   * for FP32 block streams (max_block > 1): the block step (push_block
 *     with its solves on `stream`, block_modes on a second stream,
 *     overlapping the next push) with one product per window, with window
 *     pairs (where 2r = 8 (mod 16) lets two windows fill whole 16-column
 *     tiles) and with one banded product of all windows (where its staged
 *     rows, 128 x (m + max_block) FP32 values, fit the workgroup memory);
 * and keeps the fastest (the built-in rule's choice -- the banded product
 * where a fixed-step form of it applies (windows up to about m = 70), else
 * window pairs where they fill at most three tiles, else one product per
 * window -- unless another is more than 2 % faster) in the process-wide
 * table.  Streams created afterwards
 * with the same key -- dtype, precision, n to within 1/8 octave, m, r,
 * max_block -- use it; existing streams keep their shapes.  The table is
 * loaded once from the file named by the environment variable
 * DMD_TUNE_CACHE, if set.  Synchronous.  Errors: those of
 * dmd_stream_create, DMD_E_UNSUPPORTED (sparse), DMD_E_NOMEM, DMD_E_DEVICE. */
int dmd_tune(int64_t n, int32_t m, int32_t r, const dmd_opts_t* opts, dmd_tuning_t* out, void* stream);

/* The table's entry for this shape; DMD_E_NOT_READY if there is none (streams
 * then use the built-in rules). */
int dmd_tune_lookup(int64_t n, int32_t m, int32_t r, const dmd_opts_t* opts, dmd_tuning_t* out);

/* Write the table to a text file (one entry per line), or merge one into it.
 * A malformed file is refused whole (DMD_E_INVAL). */
int dmd_tune_save(const char* path);
int dmd_tune_load(const char* path);

/* Empty the table. */
int dmd_tune_clear(void);

/* ------------------------------------------------------------ introspection */

typedef struct {
    int64_t n;
    int32_t m, r, dtype, precision;
    int32_t count;          /* snapshots currently in the window */
    int32_t r_eff;          /* rank used by the latest solve (0 if none) */
    int32_t sweeps;         /* Jacobi sweeps of the latest solve */
    int32_t qr_iters;       /* Hessenberg-QR iterations of the latest solve */
    int64_t device_bytes;   /* device memory owned by the handle */
    int32_t gram_iter;      /* launch shapes fixed at creation (see dmd_tuning_t); 0 for sparse */
    int32_t proj_form;
} dmd_info_t;

/* Wait for the handle's work and describe it. */
int dmd_stream_info(dmd_stream_t* h, dmd_info_t* info);

/* ------------------------------------------------------------ batched tick */

/* A batch groups streams so that one tick processes a new snapshot for many
 * of them with one launch per phase: one Gram pass over all their windows,
 * one finalize, the Jacobi solves of all streams side by side (one workgroup,
 * i.e. one CU, per stream), one eig launch and one projection launch.  Only
 * dense FP32 streams with auto_solve on can join (any m, n, r); their
 * projections run in FP32.  Results stay per stream: after a tick,
 * dmd_stream_eigs/svd/atilde/modes of each member return that member's latest
 * solve exactly as after dmd_stream_push.
 *
 * Admission: a batch has an HBM budget; dmd_batch_attach fails with
 * DMD_E_NOMEM when the stream's device footprint (ring, Gram, workspaces)
 * would exceed it, so a server admits a new stream only once others have
 * detached and freed their share. */
typedef struct dmd_batch dmd_batch_t;

typedef struct {
    int32_t max_streams;  /* capacity, 1 .. 1024 (0 = 256)                          */
    int32_t graphs;       /* 0 (default): a tick enqueues its launches one by one;
                             1 .. 256: a tick runs as one HIP graph launch, captured
                             the first time a tick of its shape occurs (number of
                             streams of each solver kind, Gram and projection
                             workgroups, descriptor buffer) and replayed after that;
                             up to `graphs` graphs are kept (least recently used
                             evicted).  Results are identical to the eager form.    */
    int64_t hbm_budget;   /* bytes the attached streams may own together
                             (0 = 90 % of the device memory free at creation)       */
    int32_t reserved[8];  /* must be zero                                            */
} dmd_batch_opts_t;

int dmd_batch_opts_init(dmd_batch_opts_t* opts);

/* Create a batch on the current device.  opts may be NULL. */
int dmd_batch_create(const dmd_batch_opts_t* opts, dmd_batch_t** out);

/* Wait for the batch's ticks and free it (attached streams are not freed). */
int dmd_batch_destroy(dmd_batch_t* b);

/* Admit a stream (DMD_E_NOMEM over budget, DMD_E_INVAL if already attached or
 * full, DMD_E_UNSUPPORTED unless it solves every push (auto_solve) on the
 * batch's device; a sparse stream must use the tridiagonal solver, i.e. no
 * warm start).  Dense FP32 streams with FP32 or split-BF16 projections share
 * grouped Gram and projection launches; FP64 streams (FP64 data or FP64
 * projections) and sparse streams run their own Gram (or sparse ingest) and
 * projection kernels inside the tick; every member's small solves are
 * grouped.  Detach returns its footprint to the budget. */
int dmd_batch_attach(dmd_batch_t* b, dmd_stream_t* h);
int dmd_batch_detach(dmd_batch_t* b, dmd_stream_t* h);

/* One tick on `stream`: push snapshots[i] (n_i values of the stream's dtype,
 * FP32 or FP64, device) into streams[i] for i < count (attached, pairwise
 * distinct, dense), run every small solve and, where modes != NULL and
 * modes[i] != NULL, write that stream's Phi into modes[i] (complex64, or
 * complex128 for FP64 projections; leading dimension ld_modes[i] >= n_i).
 * Equivalent to dmd_stream_push + dmd_stream_modes per stream, with the same
 * results bit for bit; asynchronous.  Each member's later calls are ordered
 * after the tick.  Sparse members need dmd_batch_tick_frames (DMD_E_INVAL). */
int dmd_batch_tick(dmd_batch_t* b, int32_t count, dmd_stream_t* const* streams,
                   const void* const* snapshots, void* const* modes,
                   const int64_t* ld_modes, void* stream);

/* One member's frame of a tick: for a dense stream x (n values of its dtype,
 * device; nnz, idx, val unused); for a sparse stream a snapshot as for
 * dmd_stream_push_csr (nnz in [0, max_nnz], idx and val on the device, idx
 * sorted, unique and in [0, n): a snapshot that breaks this is rejected by
 * the device as in dmd_stream_push_csr). */
typedef struct {
    const void* x;
    int32_t nnz;
    const int32_t* idx;
    const void* val;
} dmd_frame_t;

/* dmd_batch_tick for any mix of members, dense and sparse (Sec. 3.5), one
 * frame each; the same ordering, outputs and errors.  A tick with FP64 or
 * sparse members runs eagerly even when the batch replays ticks as graphs
 * (their frames reach their kernels as launch arguments). */
int dmd_batch_tick_frames(dmd_batch_t* b, int32_t count, dmd_stream_t* const* streams,
                          const dmd_frame_t* frames, void* const* modes, const int64_t* ld_modes,
                          void* stream);

/* Attached streams, their total device footprint and the budget. */
int dmd_batch_info(dmd_batch_t* b, int32_t* nstreams, int64_t* used_bytes,
                   int64_t* budget);

/* ------------------------------------------------------------ environment */

/* DMD_GRAM_ITER = 1, 2 or 4 (read at every push): 16-byte loads per thread
 * and window column in one workgroup of the one-column Gram update, instead
 * of the default chosen from n (the largest that still gives one workgroup
 * per CU).  Results differ from the default only in the order of the FP64
 * partial sums. */

/* ------------------------------------------------------------ kernel timing */

/* Process-wide per-kernel timing for diagnostics and roofline measurement.
 * When enabled, every kernel launch of every handle is bracketed by HIP events
 * recorded on its launch stream.  Kernel names: "gram_columns",
 * "gram_finalize", "solve_sym", "solve_eig", "project_modes", "project_pod",
 * "background", "csr_gram", "csr_project", "gram_full", "fourier" (the
 * ingest's two DFT kernels); for block pushes "gram_block" (block Gram pass,
 * reduction and commit), "block_solve" (all windows' solves), "pack_block"
 * (packing the projection inputs) and "project_block" (all windows' modes);
 * for batch ticks "batch_gram", "batch_solve", "batch_project" (eager ticks)
 * or "batch_graph" (graph ticks).
 * dmd_profile_read waits for the recorded events and returns the number of
 * launches of `kernel` and their summed duration in milliseconds since the
 * last dmd_profile_reset. */
int dmd_profile_enable(int on);
int dmd_profile_reset(void);
int dmd_profile_read(const char* kernel, int64_t* launches, double* total_ms);

/* Message of the calling thread's last error ("" if none).  Never NULL. */
const char* dmd_last_error(void);

/* Library version string. */
const char* dmd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DMD_STREAM_H */
