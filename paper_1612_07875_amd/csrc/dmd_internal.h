// Internal definitions shared by the HIP kernels and the C-ABI runtime of
// libdmdstream.  Not part of the public interface (see include/dmd_stream.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dmd_stream.h"

namespace dmd {

// Device-resident state of one stream.  It lives at the start of the results
// block so that a single device-to-host copy returns the state together with
// sigma and lambda.  Kernels read and update it, so the host can enqueue a
// whole frame without knowing whether earlier pushes were accepted.
//
// The ring holds slots = m+1+B snapshots: the window (count <= m+1 snapshots
// starting at physical slot `oldest`) and B >= 1 spare slots (B = the largest
// block push allowed) that the next push or block push fills.  A rejected push
// therefore never touches the window.
struct DevState {
    int32_t oldest;             // physical slot of the oldest window snapshot
    int32_t count;              // snapshots in the window (0 .. m+1)
    int32_t rejected_nonfinite; // pushes rejected for non-finite inner products
    int32_t rejected_index;     // sparse pushes rejected for bad indices
    int32_t solve_status;       // status of the latest solve (DMD_* code)
    int32_t r_eff;              // rank used by the latest solve
    int32_t sweeps;             // Jacobi sweeps of the latest solve
    int32_t qr_iters;           // Hessenberg-QR iterations of the latest solve
    int32_t solves;             // solves run on a full window
    int32_t pushes;             // accepted pushes
    int32_t vprev_valid;        // Vfull holds the eigenvectors of a converged solve
    int32_t vprev_push;         // value of `pushes` at that solve
    int32_t warm;               // latest solve was warm-started (1: shifted, 2: same window)
    int32_t skipped;            // latest solve found nothing new and kept the previous results
    int32_t block_rejected;     // the latest block push was rejected (non-finite inner products)
    int32_t bg_index;           // background mode (argmin |log lambda|) of the latest solve
};
static_assert(sizeof(DevState) == 64, "DevState must stay 64 bytes");

// Layout of the results block (device and pinned-host mirror).
struct ResultsLayout {
    size_t sigma_off;  // m doubles
    size_t lam_off;    // 2 r doubles (interleaved complex)
    size_t amp_off;    // 2 r doubles: mode amplitudes b (interleaved complex)
    size_t bytes;
    static ResultsLayout make(int m, int r) {
        ResultsLayout L;
        L.sigma_off = sizeof(DevState);
        L.lam_off = L.sigma_off + sizeof(double) * (size_t)m;
        L.amp_off = L.lam_off + sizeof(double) * 2 * (size_t)r;
        L.bytes = L.amp_off + sizeof(double) * 2 * (size_t)r;
        return L;
    }
};

// Physical slot of logical window column l (0 = oldest).
// Columns of X in the current window: m once the window holds m+1 snapshots;
// during a build-up start (Sec. 5: results while the window fills) count - 1
// from count = 3 on; 0 while there is nothing to solve.
__device__ inline int window_cols(int m, int buildup, const DevState* st) {
    const int c = st->count;
    if (c >= m + 1) return m;
    return (buildup && c >= 3) ? c - 1 : 0;
}

__host__ __device__ inline int slot_of(int oldest, int l, int slots) {
    int s = oldest + l;
    return s >= slots ? s - slots : s;
}

// Status codes (mirror of the public header, usable in device code).
enum : int32_t {
    ST_OK = 0, ST_W_RANK = 1, ST_E_INVAL = -1, ST_E_NOT_READY = -3,
    ST_E_NONFINITE = -4, ST_E_CONVERGENCE = -5
};

// Sets the calling thread's last-error message (dmd_last_error) and returns code.
int api_fail(int code, const char* fmt, ...);

// Maximum sizes supported by the kernels.
constexpr int kMaxM = 256;   // window columns
constexpr int kMaxR = 64;    // truncation rank

// ------------------------------------------------------------------ launchers
// Each returns hipSuccess or the launch error.  All are asynchronous on `s`.

// Dense inner products of one new snapshot with the kept window columns
// (ingest fused), per-workgroup partial sums, then the fixed-order reduction
// and Gram update.  T = float or double.
// Per-workgroup partial sums (ingest fused), then a fixed-order reduction
// kernel that rejects non-finite results or writes the new Gram row/column
// and advances the window.
// `iter` (1, 2 or 4) is the slab form: 16-byte loads per thread and column
// in one workgroup's slab of rows (fixed per stream, see gram_iter_rule).
template <typename T>
hipError_t launch_gram_columns(const T* x, T* ring, int64_t ld, int64_t n, int m, int slots,
                               double* partials, int nblk_cap, const DevState* st, int iter,
                               int* nblk_used, hipStream_t s);
hipError_t launch_gram_finalize(double* G, const double* partials, int nblk, int m, int slots,
                                DevState* st, hipStream_t s);
int gram_push_blocks(int64_t n, int elem_bytes);
// The slab form chosen when neither the tuning table nor DMD_GRAM_ITER
// names one, and the workgroups of a slab form.
int gram_iter_rule(int64_t n, int elem_bytes);
int gram_blocks(int64_t n, int elem_bytes, int iter);

// One stream's share of a grouped (batched) push: FP32 data.
struct GramItem {
    const void* x;
    void* ring;
    int64_t ld, n;
    int m, slots, x_aligned, nblk, iter;
    double* partials;
    double* G;
    DevState* st;
};
// Gram pass and finalize for many streams in two launches; the blocks of item
// i are blk_start[i] .. blk_start[i+1]-1, each item in its stream's slab form.
hipError_t launch_gram_grouped(const GramItem* items, const int* blk_start, int nitems, int total_blocks,
                               hipStream_t s);

// Sparse complex snapshot: ingest into the CSR ring (with index checks),
// Hermitian inner products through a dense scatter vector, fixed-order
// reduction and Gram update, scatter vector cleared again.
hipError_t launch_csr_push(const int32_t* idx, const float2* val, int nnz, int64_t n,
                           int32_t* ring_idx, float2* ring_val, int32_t* ring_nnz,
                           int max_nnz, int m, float2* scatter, int* flag,
                           double* G, double* partials, DevState* st, hipStream_t s);
int csr_partials_per_column();

// FP64 small solves for the current window: Jacobi eig of X^*X, sigma, V,
// A~, eig(A~) by Hessenberg-QR, coefficient matrices for the projections.
struct SolveArgs {
    DevState* st;
    const double* G;       // (m+2)^2 physical Gram (complex: interleaved)
    int m, r, slots;
    int cplx;              // 1 for the Hermitian (sparse complex) path
    double rcond, tol;
    int max_sweeps, max_qr_iter;
    int warm_start;        // start Jacobi from the previous solve's eigenvectors
    int buildup;           // solve partial windows of 3..m snapshots (window_cols)
    double* sigma;         // results block: m sigmas (zero past the window's columns)
    double* lam;           // results block: 2 r doubles
    double* amp;           // results block: 2 r doubles, mode amplitudes b
    double* V;             // m x r (complex: interleaved), canonical columns, leading
                           // dimension m (rows past the window's columns zero)
    double* At;            // r x r (complex: interleaved)
    double* W;             // r x r complex
    double* work;          // global scratch: 4 M (M+1) values (A, V, Q or Z, tail scratch)
    double* Vfull;         // m x m eigenvectors of the latest solve, sigma order
    void* Bphi;            // m x 2r coefficients of Phi (row-major, data precision)
    void* Bpod;            // m x r (real) or m x 2r (complex) coefficients of U
    void* Bbg;             // m complex coefficients of the background (may be null)
    int coef_f64;          // 1: coefficients stored as double, 0: float
    char* res_block;       // device results block (state, sigma, lambda)
    char* res_host;        // device address of its pinned host mirror
    int res_bytes;         // size of the results block
    // single-window eig solve only (may be null): after the solve, copy the
    // state to snap_st and snap_n16 x 16 bytes of Bphi to snap_B (the
    // snapshot a later projection of this solve reads)
    DevState* snap_st;
    void* snap_B;
    int snap_n16;
};
hipError_t launch_solve_sym(const SolveArgs& a, hipStream_t s);
// Same outputs by Householder tridiagonalization, multisection and twisted
// factorizations (no warm start).
hipError_t launch_solve_trid(const SolveArgs& a, hipStream_t s);
// The finalize of a dense push's Gram pass (launch_gram_finalize) and the
// real tridiagonal solve of the new window as one launch.
hipError_t launch_finalize_solve_trid(double* G, const double* partials, int nblk, const SolveArgs& a,
                                      hipStream_t s);
// Grouped real symmetric solves (one workgroup per item; lds: m <= 64) by
// Jacobi or by the tridiagonal method, and the grouped eig of A~.
hipError_t launch_jacobi_grouped(const SolveArgs* items_lds, int n_lds, const SolveArgs* items_glb, int n_glb,
                                 hipStream_t s);
hipError_t launch_trid_grouped(const SolveArgs* items_lds, int n_lds, const SolveArgs* items_glb, int n_glb,
                               hipStream_t s);
// Grouped Hermitian (complex) tridiagonal solves: items_lds m <= 32, items_glb m > 32.
hipError_t launch_trid_grouped_cplx(const SolveArgs* items_lds, int n_lds, const SolveArgs* items_glb, int n_glb,
                                    hipStream_t s);
hipError_t launch_eig_grouped(const SolveArgs* items, int n, hipStream_t s);
hipError_t launch_solve_eig(const SolveArgs& a, hipStream_t s);

// Multi-column update (k new snapshots at once): one pass over the window and
// the k new columns gives the (count+k) x k block of new inner products on the
// matrix cores (FP64 products and sums), with the new columns copied into the
// spare slots in the same pass; a reduction kernel sums the row splits in a
// fixed order into gblock (leading dimension `slots`) and raises *flag on a
// non-finite entry; the commit kernel then rejects the whole block or writes
// the Gram, advances the window by k and prepares the state of every
// intermediate window (window w < k-1 in shadow state kmax-k+w).
struct BlockArgs {
    const void* ring;
    int64_t ld, n;
    const void* xnew;
    int64_t ldx;
    int m, slots, k, x_aligned;
    int ntile_i, ntile_j, nsplit;
    int64_t rows_per_split;
    double* partial;       // [nsplit][ntile_i * ntile_j][64 * 64]
    double* gblock;        // slots x k, column-major
    int* flag;
    double* G;
    DevState* st;
    char* shadow;          // states of the intermediate windows, shadow_stride bytes apart
    int shadow_stride, kmax;
};
hipError_t launch_gram_block(BlockArgs a, int elem_f64, hipStream_t s);
int gram_block_splits(int m, int kmax);
int gram_block_tiles(int m, int kmax);

// Tall-skinny projection out = X_sub * B for the ring's logical columns
// first .. first+m-1 (X' for first = 1, X for first = 0).
struct ProjectArgs {
    const DevState* st;
    const void* ring;      // dense ring (float or double)
    int64_t ld, n;
    int m, slots, first;
    const void* B;         // m x kcols row-major coefficients
    int kmax;              // allocated columns of B (row stride)
    int cplx_out;          // 1: kcols = 2 r_eff interleaved complex columns
    void* out;
    int64_t ldo;
    int elem_f64;          // ring elements are double (else float)
    int coef_f64;          // coefficients, accumulation and output in double
    int precision;         // DMD_PREC_* used for float data
    int block_only;        // a window of a block push: skip it if the block was rejected
    int buildup;           // partial windows (window_cols): X_sub has window_cols columns
};
hipError_t launch_project(const ProjectArgs& a, hipStream_t s);
// Grouped FP32 projections of many streams in one launch.
hipError_t launch_project_grouped(const ProjectArgs* items, const int* blk_start, int nitems, int total_blocks,
                                  hipStream_t s);
int project_item_blocks(int64_t n);

// Modes of every window of a block push in one pass over the ring (FP32 data
// and coefficients).  Window w (0 = oldest) of the block ends w - k + 1
// snapshots before the current window; its X' is the m ring columns starting
// at logical position w - k + 2 of the current window.  Window w < k-1 has its
// state and coefficients in set kmax-k+w of the intermediate-window sets;
// window k-1 uses the stream's own.  Phi of window w goes to out + w * ldw
// complex elements (column j at + j * ldo); windows without a solve are skipped.
//
// The block's inputs are packed right after its solves (launch_pack_block):
// the coefficients in fragment order (cfrag) and a BlockDesc with the ring
// position and the windows' ranks, so that the projection reads nothing that
// the next block push modifies (the ring keeps 2 max_block spare slots).
struct BlockDesc {
    int valid;        // the window is full and the block was accepted
    int base;         // ring slot of the union's first column (before the wrap)
    int pad[2];
    int kc[64];       // 2 r_eff of window w, 0 if it has no solve
    float sink[64 * 4];  // 16 bytes per lane that a projection writes instead of
                         // columns it must leave untouched (never read)
};
struct BlockProjectArgs {
    const void* ring;
    int64_t ld, n;
    int m, r, slots, k, kmax;
    const DevState* st;            // the stream's state (current window)
    const char* shadow;            // states of the intermediate windows
    int shadow_stride;
    const float* Bphi;             // current window's coefficients (m x 2r row-major)
    const float* Bphi_sets;        // intermediate sets, bphi_stride floats apart
    int64_t bphi_stride;
    float2* out;
    int64_t ldo, ldw;
    int bf16x3;                    // products as three BF16 MFMAs (DMD_PREC_BF16X3), else FP32
    int form;                      // 0: rule, 1: one product per window, 2: window pairs where they apply,
                                   // 3: one banded product of all windows (FP32)
    int out16;                     // out, ldo and ldw allow 16-byte stores of two rows
    uint4* cfrag;                  // project_block_frag_bytes(m, kmax): packed coefficients
    BlockDesc* desc;               // packed ring position and ranks
};
// Pack (after the block's solves; reads st, shadow, Bphi, Bphi_sets) and
// project (reads ring, cfrag and desc only).
hipError_t launch_pack_block(const BlockProjectArgs& a, hipStream_t s);
hipError_t launch_project_block(const BlockProjectArgs& a, hipStream_t s);
// Whether the one-pass block projection's LDS tiles fit for these sizes.
bool project_block_fits(int m, int k, int r);
size_t project_block_frag_bytes(int m, int r, int kmax);
// Whether the window-pair form (2r = 8 mod 16) or the banded form (its stage
// fits) can run an FP32 block of k windows.
bool pairs_apply(int m, int r, int k);
bool band_applies(int m, int r, int k);
// The form the built-in rule takes for an FP32 block of k windows (1 or 2).
int block_rule_form(int m, int r, int k);

// Background subtraction of the newest snapshot (Sec. 3.3, Algorithm 3): with
// beta = b_i lambda_i^m C[:, i] (background mode i, written by the eig solve),
// bg = |X' beta| and fg = x_new - bg, x_new being the last column of X'.
struct BackgroundArgs {
    const DevState* st;
    const void* ring;
    int64_t ld, n;
    int m, slots;
    int buildup;           // partial windows (window_cols)
    const void* beta;      // m complex, float or double (elem_f64 / coef_f64)
    void* fg;              // n values of the data type (may be null)
    void* bg;              // n values of the data type (may be null)
    int elem_f64;          // ring elements are double (else float)
    int coef_f64;          // beta and the accumulation in double
};
hipError_t launch_background(const BackgroundArgs& a, hipStream_t s);

// Spatial -> Fourier ingest (Sec. 3.5): the unitary 2-D DFT of an H x W
// FP32 frame (row-major, row stride ld_row) at the nkeep support points
// (ky[c], kx[col[c]]), into val (complex64), through the row transforms R
// (H x nkx, FP64) at the nkx distinct kx bins.  tw_N[j] = e^{-2 pi i j / N}.
constexpr int kFourierMaxW = 16384;  // the row is staged in LDS
struct FourierArgs {
    const float* frame;
    int64_t ld_row;
    int H, W;
    const int* kx;         // nkx distinct kx bins
    int nkx;
    const int* ky;         // ky bin of each kept coefficient
    const int* col;        // index into kx of each kept coefficient
    int nkeep;
    const double2* twW;    // W roots of unity
    const double2* twH;    // H roots of unity
    double2* R;            // H x nkx scratch
    float2* val;           // nkeep coefficients
    double scale;          // (H W)^-1/2
};
hipError_t launch_fourier(const FourierArgs& a, hipStream_t s);

// Sparse projection: out = X_sub * B (complex) into a dense n x r_eff
// complex64 output (zero outside the window's support).
// Scratch of the sparse projection: the index map pos (n entries, all -1
// between calls), the union list U and the dense block D (cap x m) of the
// window on its union; cap = csr_union_cap(n, max_nnz).
struct CsrUnionScratch {
    int32_t* pos;
    int32_t* U;
    int* ucount;
    int* overflow;
    int cap;
    float2* D;
};
int csr_union_cap(int64_t n, int max_nnz);
hipError_t launch_csr_project(const DevState* st, const int32_t* ring_idx, const float2* ring_val,
                              const int32_t* ring_nnz, int max_nnz, int m, int first, const float2* B, int kmax,
                              float2* out, int64_t ldo, int64_t n, const CsrUnionScratch& u, hipStream_t s);

// Whole Gram of the window's first kcols columns on the matrix cores (FP64,
// FP32 or BF16x3 products), split over rows with a fixed-order FP64 sum.
// oldest_override >= 0 places the window at that slot (new window, set_window
// = 1); -1 uses the device state (recomputation, set_window = 2).
hipError_t launch_gram_full(const void* ring, int64_t ld, int64_t n, int m, int slots, int elem_f64,
                            int precision, int kcols, int oldest_override, double* partial, double* G,
                            DevState* st, int set_window, hipStream_t s);
hipError_t launch_copy_columns(const void* X, int64_t ldx, void* ring, int64_t ld, int64_t n, int k,
                               int elem_f64, hipStream_t s);
int gram_full_tiles(int m);
int gram_full_splits(int m);

// Stateless whole Gram of ncols columns of X (column-major, leading dimension
// ldx, 16-byte aligned columns) into G (leading dimension ldg), with the
// kernel's partial tiles in `partial` (window_gram_scratch_bytes(ncols)).
size_t window_gram_scratch_bytes(int32_t ncols);
hipError_t launch_window_gram(const void* X, int64_t ldx, int64_t n, int32_t ncols, int elem_f64, int32_t precision,
                              double* G, int64_t ldg, double* partial, hipStream_t s);

// ------------------------------------------------------------------ tuning
// Launch shapes chosen by measurement (dmd_tune) for a stream shape; a stream
// created later with the same key takes them (else the built-in rules).
struct TuneKey {
    int dtype, precision, nbucket, m, r, kmax;
    bool operator==(const TuneKey& o) const {
        return dtype == o.dtype && precision == o.precision && nbucket == o.nbucket && m == o.m && r == o.r &&
               kmax == o.kmax;
    }
};
struct TuneVal {
    int gram_iter;     // 0: rule
    int proj_form;     // 0: rule, 1: per window, 2: window pairs
    double gram_us;    // measured one-frame Gram pass of the choice
    double step_us;    // measured pipelined block step of the choice (0: not measured)
};
TuneKey tune_key(int64_t n, int m, int r, const dmd_opts_t& o);
bool tune_lookup(const TuneKey& k, TuneVal* v);
void stream_get_shapes(const dmd_stream* h, int* gram_iter, int* proj_form);
void stream_set_shapes(dmd_stream* h, int gram_iter, int proj_form);

}  // namespace dmd
