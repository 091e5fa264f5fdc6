// C-ABI runtime of libdmdstream: stream handles, device memory, argument
// checks and the ordering of kernels for one frame.  See include/dmd_stream.h
// for the contract of every entry point.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dmd_internal.h"
#include "dmd_stream.h"

#define DMD_API extern "C" __attribute__((visibility("default")))

using dmd::DevState;
using dmd::ResultsLayout;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace

// Error reporting for entry points defined in other source files.
int dmd::api_fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

namespace {

int hip_fail(hipError_t e, const char* what) {
    return fail(DMD_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call)                                         \
    do {                                                      \
        hipError_t _e = (call);                               \
        if (_e != hipSuccess) return hip_fail(_e, #call);     \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

// Optional per-kernel timing: HIP events recorded on the launch stream right
// before and after each kernel, resolved when read.
struct ProfRec {
    const char* name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Runs `launch` (a callable returning hipError_t) bracketed by events when profiling.
template <typename F>
hipError_t timed(const char* name, hipStream_t s, F&& launch) {
    if (!g_prof_on) return launch();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfRec r{name, prof_event(), prof_event()};
    (void)hipEventRecord(r.a, s);
    hipError_t e = launch();
    (void)hipEventRecord(r.b, s);
    g_prof.push_back(r);
    return e;
}

}  // namespace

struct dmd_stream {
    int64_t n = 0, ld = 0;
    int32_t m = 0, r = 0, slots = 0;
    dmd_opts_t opts{};
    int device = 0;
    int elem_bytes = 4;     // dense ring element size
    bool cplx = false;      // sparse complex path
    bool coef_f64 = false;  // projection coefficients and accumulation in double
    bool use_trid = true;   // symmetric eig by the tridiagonal method (else Jacobi)

    void* ring = nullptr;       // dense: slots x ld elements
    int32_t* ring_idx = nullptr;  // sparse: slots x max_nnz indices
    float2* ring_val = nullptr;   // sparse: slots x max_nnz values
    int32_t* ring_nnz = nullptr;  // sparse: slots counts
    float2* scatter = nullptr;    // sparse: n dense scratch (kept zero)
    int32_t* upos = nullptr;      // sparse projection: index -> union row (-1 outside)
    int32_t* ulist = nullptr;     // union rows -> index
    int* ucount = nullptr;        // |U| and the overflow flag
    float2* ublock = nullptr;     // window on its union, ucap x m
    int ucap = 0;
    int* flag = nullptr;          // sparse: bad-index flag of the push in flight
    int max_nnz = 0;

    double* G = nullptr;
    double* partials = nullptr;
    int nblk_cap = 0;
    char* res_dev = nullptr;
    char* res_host = nullptr;   // pinned, mapped
    char* res_host_dev = nullptr;
    ResultsLayout L{};
    double* V = nullptr;
    double* At = nullptr;
    double* W = nullptr;
    double* work = nullptr;
    double* Vfull = nullptr;
    double* gfull = nullptr;      // per-split tiles of the whole-window Gram
    void* Bphi = nullptr;
    void* Bpod = nullptr;
    void* Bbg = nullptr;          // background coefficients (m complex)

    // block pushes: up to kmax snapshots at once (ring has kmax spare slots)
    int kmax = 1;
    int bsplit_cap = 0;
    double* bpartial = nullptr;   // per-split partial blocks of new inner products
    double* gblock = nullptr;     // their fixed-order sums
    int* bflag = nullptr;         // non-finite flag of the block in flight
    // one solve set per intermediate window of a block (kmax - 1 sets)
    size_t sh_stride = 0;         // bytes between results blocks
    char* sh_dev = nullptr;
    char* sh_host = nullptr;      // pinned, mapped
    char* sh_host_dev = nullptr;
    double* sh_V = nullptr;
    double* sh_At = nullptr;
    double* sh_W = nullptr;
    double* sh_work = nullptr;
    double* sh_Vfull = nullptr;
    void* sh_Bphi = nullptr;
    void* sh_Bpod = nullptr;
    // Block pushes: the projection inputs of the latest two blocks, packed
    // after their solves (parity = block number & 1), and the events of the
    // projections that read them.  A block push waits only for the
    // projection of the block two back (same parity), so that the projection
    // of block b can run beside the Gram update and solves of block b + 1.
    uint4* cfrag = nullptr;       // 2 x cfrag_elems packed coefficients
    size_t cfrag_elems = 0;
    dmd::BlockDesc* bdesc = nullptr;  // 2 descriptors
    hipEvent_t ev_proj[2] = {nullptr, nullptr};
    hipStream_t proj_stream[2] = {nullptr, nullptr};
    bool proj_pending[2] = {false, false};
    int64_t block_seq = 0;        // block pushes so far
    int last_packed = -1;         // parity packed by the latest push, -1 if none
    // Dense streams: each solve leaves a copy of its state and of its mode
    // coefficients in snapshot parity snap_seq & 1, so that dmd_stream_modes
    // of one solve can run beside the next push (which rewrites both).
    DevState* snap_st = nullptr;  // two DevStates
    char* snap_B = nullptr;       // two copies of Bphi
    size_t snap_B_bytes = 0;
    int64_t snap_seq = 0;
    int snap_par = -1;            // parity of the latest solve's snapshot, -1 if stale
    hipEvent_t ev_sproj[2] = {nullptr, nullptr};
    hipStream_t sproj_stream[2] = {nullptr, nullptr};
    bool sproj_pending[2] = {false, false};
    // Spatial -> Fourier ingest (sparse streams): grid, support and tables
    int four_H = 0, four_W = 0, four_nkeep = 0, four_nkx = 0;
    int32_t* f_idx = nullptr;     // flattened support indices, increasing
    int32_t* f_ky = nullptr;      // ky bin per support point
    int32_t* f_col = nullptr;     // column of R per support point
    int32_t* f_kx = nullptr;      // distinct kx bins
    double2* f_twW = nullptr;
    double2* f_twH = nullptr;
    double2* f_R = nullptr;
    float2* f_val = nullptr;
    std::vector<int32_t> four_support;  // host copy of f_idx
    dmd::SolveArgs* solve_tbl = nullptr;  // device: sets 0 .. kmax-2, then the current window
    int32_t last_block_k = 0;     // k of the latest push if it was a solved block push, else 0

    hipEvent_t ev_last = nullptr;
    hipEvent_t ev_solved = nullptr;
    hipStream_t last_stream = nullptr;
    bool has_last = false;
    bool solve_enqueued = false;
    int32_t reported_nonfinite = 0;
    int32_t reported_index = 0;
    int64_t device_bytes = 0;
    bool dry = false;             // sizing only (dmd_stream_footprint): count bytes, allocate nothing
    // Launch shapes fixed at creation (DMD_GRAM_ITER, the tuning table, or
    // the rules), so that a stream's results never change mid-stream:
    int gram_iter = 0;            // slab form of the one-frame Gram pass (1, 2, 4)
    int proj_form = 0;            // block projection: 0 rule, 1 per window, 2 window pairs
    // Snapshots pushed from host memory are copied here first (allocated by
    // the first such push): dense n elements; sparse max_nnz indices + values.
    void* stage = nullptr;
    int32_t* stage_idx = nullptr;
    float2* stage_val = nullptr;
};

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Order the handle's work across streams: a call on a new stream first waits
// for everything enqueued before it.
hipError_t begin(dmd_stream* h, hipStream_t s) {
    if (h->has_last && h->last_stream != s) {
        hipError_t e = hipStreamWaitEvent(s, h->ev_last, 0);
        if (e != hipSuccess) return e;
    }
    for (int p = 0; p < 2; ++p) {
        if (h->proj_pending[p] && h->proj_stream[p] != s) {
            hipError_t e = hipStreamWaitEvent(s, h->ev_proj[p], 0);
            if (e != hipSuccess) return e;
        }
        if (h->sproj_pending[p] && h->sproj_stream[p] != s) {
            hipError_t e = hipStreamWaitEvent(s, h->ev_sproj[p], 0);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}
// A single push whose solve will write snapshot parity p: after everything
// but the modes of the previous solve (parity 1 - p), which read the window
// of that solve (not the slot this push writes) and its snapshot only.
hipError_t begin_single(dmd_stream* h, hipStream_t s, int p) {
    if (h->has_last && h->last_stream != s) {
        hipError_t e = hipStreamWaitEvent(s, h->ev_last, 0);
        if (e != hipSuccess) return e;
    }
    for (int q = 0; q < 2; ++q)
        if (h->proj_pending[q] && h->proj_stream[q] != s) {
            hipError_t e = hipStreamWaitEvent(s, h->ev_proj[q], 0);
            if (e != hipSuccess) return e;
        }
    if (h->sproj_pending[p] && h->sproj_stream[p] != s) return hipStreamWaitEvent(s, h->ev_sproj[p], 0);
    return hipSuccess;
}
// A block push of parity p: after everything but the projection of the
// previous block (parity 1 - p), which reads neither the slots this push
// writes nor its packed inputs.
hipError_t begin_block(dmd_stream* h, hipStream_t s, int p) {
    if (h->has_last && h->last_stream != s) {
        hipError_t e = hipStreamWaitEvent(s, h->ev_last, 0);
        if (e != hipSuccess) return e;
    }
    for (int q = 0; q < 2; ++q)
        if (h->sproj_pending[q] && h->sproj_stream[q] != s) {
            hipError_t e = hipStreamWaitEvent(s, h->ev_sproj[q], 0);
            if (e != hipSuccess) return e;
        }
    if (h->proj_pending[p] && h->proj_stream[p] != s) return hipStreamWaitEvent(s, h->ev_proj[p], 0);
    return hipSuccess;
}
hipError_t end(dmd_stream* h, hipStream_t s) {
    h->last_stream = s;
    h->has_last = true;
    return hipEventRecord(h->ev_last, s);
}

template <typename P>
int dev_alloc(dmd_stream* h, P** p, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (h->dry) {
        h->device_bytes += (int64_t)bytes;
        return DMD_OK;
    }
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(DMD_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    e = hipMemset(q, 0, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMemset");
    *p = reinterpret_cast<P*>(q);
    h->device_bytes += (int64_t)bytes;
    return DMD_OK;
}

void free_all(dmd_stream* h) {
    void* bufs[] = {h->ring, h->ring_idx, h->ring_val, h->ring_nnz, h->scatter, h->flag, h->G, h->partials,
                    h->res_dev, h->V, h->At, h->W, h->work, h->Vfull, h->gfull, h->Bphi, h->Bpod,
                    h->Bbg, h->bpartial, h->gblock, h->bflag, h->sh_dev, h->sh_V, h->sh_At, h->sh_W, h->sh_work,
                    h->sh_Vfull, h->sh_Bphi, h->sh_Bpod, h->cfrag, h->bdesc, h->solve_tbl,
                    h->f_idx, h->f_ky, h->f_col, h->f_kx, h->f_twW, h->f_twH, h->f_R, h->f_val,
                    h->upos, h->ulist, h->ucount, h->ublock, h->snap_st, h->snap_B,
                    h->stage, h->stage_idx, h->stage_val};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (h->res_host) (void)hipHostFree(h->res_host);
    if (h->sh_host) (void)hipHostFree(h->sh_host);
    if (h->ev_last) (void)hipEventDestroy(h->ev_last);
    for (hipEvent_t e : h->ev_proj)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->ev_sproj)
        if (e) (void)hipEventDestroy(e);
    if (h->ev_solved) (void)hipEventDestroy(h->ev_solved);
}

// Whether the kernels of h's device can read p directly: device memory of
// that device or managed memory.  Anything else (pageable or pinned host
// memory, another device's memory) is copied to a staging buffer first.
bool device_readable(const dmd_stream* h, const void* p) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // unknown to HIP: pageable host memory
        return false;
    }
    if (a.type == hipMemoryTypeManaged || a.isManaged) return true;
    return a.type == hipMemoryTypeDevice && a.device == h->device;
}

// Stream-ordered copy of `bytes` from p into *stage (allocated on first use),
// returning the staged address in *out; p itself when the kernels can read it.
template <typename P>
int stage_input(dmd_stream* h, P** stage, size_t cap_bytes, const void* p, size_t bytes, hipStream_t s,
                const void** out) {
    *out = p;
    if (bytes == 0 || device_readable(h, p)) return DMD_OK;
    if (!*stage)
        if (int rc = dev_alloc(h, stage, cap_bytes)) return rc;
    HIP_TRY(hipMemcpyAsync(*stage, p, bytes, hipMemcpyDefault, s));
    *out = *stage;
    return DMD_OK;
}

int check_handle(dmd_stream* h) {
    if (!h) return fail(DMD_E_INVAL, "null handle");
    return DMD_OK;
}

const DevState& host_state(const dmd_stream* h) {
    return *reinterpret_cast<const DevState*>(h->res_host);
}

// Sizes (in elements) of one solve set's matrices.
struct SetSizes {
    size_t V, At, W, work, Vfull, Bphi, Bpod;  // doubles, except Bphi/Bpod in bytes
};
SetSizes set_sizes(const dmd_stream* h) {
    const size_t cw = h->cplx ? 2 : 1, m = h->m, r = h->r;
    const size_t M = m + (m & 1);
    const size_t coef = h->coef_f64 ? 8 : 4;
    return SetSizes{cw * m * r, cw * r * r, 2 * r * r, cw * 4 * M * (M + 1), cw * m * m, coef * 2 * m * r,
                    coef * cw * m * r};
}

// Solve descriptor of intermediate-window set e (0 .. kmax-2) of block pushes.
void fill_shadow_args(const dmd_stream* h, dmd::SolveArgs& a, int e);

void fill_solve_args(const dmd_stream* h, dmd::SolveArgs& a) {
    a = dmd::SolveArgs{};
    a.st = reinterpret_cast<DevState*>(h->res_dev);
    a.G = h->G;
    a.m = h->m;
    a.r = h->r;
    a.slots = h->slots;
    a.cplx = h->cplx ? 1 : 0;
    a.rcond = h->opts.rcond;
    a.tol = h->opts.tol;
    a.max_sweeps = h->opts.max_sweeps;
    a.max_qr_iter = h->opts.max_qr_iter;
    a.warm_start = h->opts.warm_start;
    a.buildup = h->opts.buildup;
    a.sigma = reinterpret_cast<double*>(h->res_dev + h->L.sigma_off);
    a.lam = reinterpret_cast<double*>(h->res_dev + h->L.lam_off);
    a.amp = reinterpret_cast<double*>(h->res_dev + h->L.amp_off);
    a.V = h->V;
    a.At = h->At;
    a.W = h->W;
    a.work = h->work;
    a.Vfull = h->Vfull;
    a.Bphi = h->Bphi;
    a.Bpod = h->Bpod;
    a.Bbg = h->Bbg;
    a.coef_f64 = h->coef_f64 ? 1 : 0;
    a.res_block = h->res_dev;
    a.res_host = h->res_host_dev;
    a.res_bytes = (int)h->L.bytes;
}

void fill_shadow_args(const dmd_stream* h, dmd::SolveArgs& a, int e) {
    fill_solve_args(h, a);
    const SetSizes z = set_sizes(h);
    char* res = h->sh_dev + (size_t)e * h->sh_stride;
    a.st = reinterpret_cast<DevState*>(res);
    a.warm_start = 0;
    a.buildup = 0;
    a.sigma = reinterpret_cast<double*>(res + h->L.sigma_off);
    a.lam = reinterpret_cast<double*>(res + h->L.lam_off);
    a.amp = reinterpret_cast<double*>(res + h->L.amp_off);
    a.Bbg = nullptr;  // the background split is provided for the current window
    a.V = h->sh_V + e * z.V;
    a.At = h->sh_At + e * z.At;
    a.W = h->sh_W + e * z.W;
    a.work = h->sh_work + e * z.work;
    a.Vfull = h->sh_Vfull + e * z.Vfull;
    a.Bphi = static_cast<char*>(h->sh_Bphi) + e * z.Bphi;
    a.Bpod = static_cast<char*>(h->sh_Bpod) + e * z.Bpod;
    a.res_block = res;
    a.res_host = h->sh_host_dev + (size_t)e * h->sh_stride;
}

void fill_project_args(const dmd_stream* h, dmd::ProjectArgs& a, void* out, int64_t ld, bool modes) {
    a = dmd::ProjectArgs{};
    a.st = reinterpret_cast<const DevState*>(h->res_dev);
    a.ring = h->ring;
    a.ld = h->ld;
    a.n = h->n;
    a.m = h->m;
    a.slots = h->slots;
    a.first = modes ? 1 : 0;
    a.B = modes ? h->Bphi : h->Bpod;
    a.kmax = h->r;
    a.cplx_out = modes ? 1 : 0;
    a.out = out;
    a.ldo = ld;
    a.elem_f64 = h->elem_bytes == 8;
    a.coef_f64 = h->coef_f64;
    a.precision = h->opts.precision;
    a.buildup = h->opts.buildup;
}

// The solves of the current window.  sym_done: the symmetric solve already
// ran, fused with the push's Gram finalize (dmd_stream_push).  The eig solve
// also leaves the snapshot of the solve (state and mode coefficients, parity
// snap_seq & 1) that dmd_stream_modes projects from.
int enqueue_solve(dmd_stream* h, hipStream_t s, bool sym_done = false) {
    h->last_block_k = 0;
    h->last_packed = -1;
    h->snap_par = -1;
    dmd::SolveArgs a;
    fill_solve_args(h, a);
    if (!sym_done)
        HIP_TRY(timed("solve_sym", s, [&] {
            return h->use_trid ? dmd::launch_solve_trid(a, s) : dmd::launch_solve_sym(a, s);
        }));
    int par = -1;
    if (h->snap_st) {
        // every caller has waited for the modes of the solve before last (this parity)
        par = (int)(h->snap_seq & 1);
        a.snap_st = h->snap_st + par;
        a.snap_B = h->snap_B + par * h->snap_B_bytes;
        a.snap_n16 = (int)(h->snap_B_bytes / 16);
    }
    HIP_TRY(timed("solve_eig", s, [&] { return dmd::launch_solve_eig(a, s); }));
    if (par >= 0) {
        h->snap_par = par;
        ++h->snap_seq;
    }
    HIP_TRY(hipEventRecord(h->ev_solved, s));
    h->solve_enqueued = true;
    return DMD_OK;
}

int wait_solved(dmd_stream* h) {
    if (!h->solve_enqueued) return fail(DMD_E_NOT_READY, "no solve has been enqueued");
    HIP_TRY(hipEventSynchronize(h->ev_solved));
    return DMD_OK;
}

// Status of the latest published solve, plus one-shot rejection reports.
int solve_status(dmd_stream* h) {
    const DevState& st = host_state(h);
    if (st.rejected_nonfinite > h->reported_nonfinite) {
        h->reported_nonfinite = st.rejected_nonfinite;
        return fail(DMD_E_NONFINITE, "%d snapshot(s) rejected: non-finite inner products", st.rejected_nonfinite);
    }
    if (st.rejected_index > h->reported_index) {
        h->reported_index = st.rejected_index;
        return fail(DMD_E_INVAL, "%d sparse snapshot(s) rejected: indices not strictly increasing in [0, n)",
                    st.rejected_index);
    }
    switch (st.solve_status) {
        case dmd::ST_E_NOT_READY: return fail(DMD_E_NOT_READY, "window not full (%d of %d snapshots)", st.count, h->m + 1);
        case dmd::ST_E_CONVERGENCE: return fail(DMD_E_CONVERGENCE, "eigensolver did not converge");
        case dmd::ST_W_RANK: return DMD_W_RANK;
        default: return DMD_OK;
    }
}

int read_state(dmd_stream* h, DevState* out) {
    if (h->has_last) HIP_TRY(hipEventSynchronize(h->ev_last));
    HIP_TRY(hipMemcpy(out, h->res_dev, sizeof(DevState), hipMemcpyDeviceToHost));
    return DMD_OK;
}

}  // namespace

DMD_API int dmd_opts_init(dmd_opts_t* o) {
    if (!o) return fail(DMD_E_INVAL, "null opts");
    std::memset(o, 0, sizeof(*o));
    o->dtype = DMD_F32;
    o->precision = DMD_PREC_DEFAULT;
    o->max_nnz = 0;
    o->max_sweeps = 40;
    o->max_qr_iter = 60;
    o->auto_solve = 1;
    o->rcond = -1.0;
    o->tol = 0.0;
    return DMD_OK;
}

DMD_API const char* dmd_last_error(void) { return g_err.c_str(); }

DMD_API const char* dmd_version(void) { return "dmdstream 0.1 (gfx950)"; }

namespace {
// Creates a stream, or with `footprint` set only validates the arguments and
// adds up the device memory the stream would own (nothing is allocated and
// no device is needed).
int create_impl(int64_t n, int32_t m, int32_t r, const dmd_opts_t* opts, dmd_stream_t** out,
                int64_t* footprint) {
    const bool dry = footprint != nullptr;
    if (!dry) {
        if (!out) return fail(DMD_E_INVAL, "null output pointer");
        *out = nullptr;
    }
    dmd_opts_t o;
    dmd_opts_init(&o);
    if (opts) {
        o = *opts;
        for (int i = 0; i < 4; ++i)
            if (o.reserved[i] != 0) return fail(DMD_E_INVAL, "opts.reserved must be zero");
        if (o.max_sweeps == 0) o.max_sweeps = 40;
        if (o.max_qr_iter == 0) o.max_qr_iter = 60;
    }
    if (o.rcond < 0.0) o.rcond = 10.0 * 1.4901161193847656e-08;  // 10 sqrt(2^-52)
    if (o.tol <= 0.0) o.tol = 1e-15;
    if (n < 1) return fail(DMD_E_INVAL, "n must be >= 1 (got %lld)", (long long)n);
    if (m < 2 || m > dmd::kMaxM) return fail(DMD_E_INVAL, "m must be in [2, %d] (got %d)", dmd::kMaxM, m);
    if (r < 1 || r > m || r > 32) return fail(DMD_E_INVAL, "r must be in [1, min(m, 32)] (got %d)", r);
    if (o.dtype != DMD_F32 && o.dtype != DMD_F64 && o.dtype != DMD_C64_CSR)
        return fail(DMD_E_INVAL, "unknown dtype %d", o.dtype);
    if (o.precision < DMD_PREC_DEFAULT || o.precision > DMD_PREC_FP64)
        return fail(DMD_E_INVAL, "unknown precision %d", o.precision);
    if (o.max_sweeps < 1 || o.max_qr_iter < 1) return fail(DMD_E_INVAL, "iteration limits must be positive");
    if (o.auto_solve != 0 && o.auto_solve != 1) return fail(DMD_E_INVAL, "auto_solve must be 0 or 1");
    if (o.warm_start != 0 && o.warm_start != 1) return fail(DMD_E_INVAL, "warm_start must be 0 or 1");
    if (o.buildup != 0 && o.buildup != 1) return fail(DMD_E_INVAL, "buildup must be 0 or 1");
    if (o.eig_solver < DMD_EIG_DEFAULT || o.eig_solver > DMD_EIG_TRIDIAG)
        return fail(DMD_E_INVAL, "unknown eig_solver %d", o.eig_solver);
    if (o.eig_solver == DMD_EIG_TRIDIAG && o.warm_start)
        return fail(DMD_E_INVAL, "warm_start needs the Jacobi eigensolver");
    if (o.max_block == 0) o.max_block = 1;
    if (o.max_block < 1 || o.max_block > 64) return fail(DMD_E_INVAL, "max_block must be in [1, 64] (got %d)", o.max_block);
    if (o.dtype == DMD_C64_CSR && o.max_block != 1) return fail(DMD_E_UNSUPPORTED, "block pushes are for dense streams");
    if (o.buildup && (o.dtype == DMD_C64_CSR || o.max_block != 1))
        return fail(DMD_E_UNSUPPORTED, "the build-up start is for dense streams with single pushes");
    if (o.dtype == DMD_C64_CSR) {
        if (o.max_nnz == 0) o.max_nnz = (int32_t)(n < INT32_MAX ? n : INT32_MAX);
        if (o.max_nnz < 1 || o.max_nnz > n) return fail(DMD_E_INVAL, "max_nnz must be in [1, n]");
        if (n > INT32_MAX) return fail(DMD_E_INVAL, "sparse streams need n <= 2^31-1");
        if (o.precision != DMD_PREC_DEFAULT && o.precision != DMD_PREC_FP32)
            return fail(DMD_E_UNSUPPORTED, "sparse streams project in FP32");
    }
    if (o.precision == DMD_PREC_BF16X3 && o.dtype != DMD_F32)
        return fail(DMD_E_UNSUPPORTED, "BF16X3 applies to FP32 data");

    dmd_stream* h = new (std::nothrow) dmd_stream();
    if (!h) return fail(DMD_E_NOMEM, "host allocation failed");
    h->n = n;
    h->m = m;
    h->r = r;
    h->kmax = o.max_block;
    // a block stream keeps 2 max_block spare slots: the columns of the
    // previous block's windows survive the next block push
    h->slots = m + 1 + (h->kmax > 1 ? 2 * h->kmax : 1);
    h->opts = o;
    h->cplx = (o.dtype == DMD_C64_CSR);
    h->elem_bytes = (o.dtype == DMD_F64) ? 8 : 4;
    h->coef_f64 = (o.dtype == DMD_F64) || (o.precision == DMD_PREC_FP64);
    h->use_trid = o.eig_solver == DMD_EIG_TRIDIAG || (o.eig_solver == DMD_EIG_DEFAULT && !o.warm_start);
    h->ld = (n + 63) / 64 * 64;
    h->L = ResultsLayout::make(m, r);
    h->dry = dry;
    if (!dry && hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(DMD_E_DEVICE, "no HIP device");
    }

    if (!h->cplx) {
        dmd::TuneVal tv{};
        const bool tuned = dmd::tune_lookup(dmd::tune_key(n, m, r, o), &tv);
        h->gram_iter = tuned && tv.gram_iter ? tv.gram_iter : dmd::gram_iter_rule(n, h->elem_bytes);
        h->proj_form = tuned ? tv.proj_form : 0;
        if (const char* e = getenv("DMD_GRAM_ITER")) {  // explicit override (tests, experiments)
            const int v = atoi(e);
            if (v == 1 || v == 2 || v == 4) h->gram_iter = v;
        }
    }

    int rc = DMD_OK;
    const int cw = h->cplx ? 2 : 1;
    const int M = m + (m & 1);
    h->nblk_cap = dmd::gram_push_blocks(n, h->elem_bytes);
    const size_t coef = h->coef_f64 ? 8 : 4;
#define ALLOC(p, bytes)                                  \
    if (rc == DMD_OK) rc = dev_alloc(h, &(p), (bytes));
    if (h->cplx) {
        h->max_nnz = o.max_nnz;
        h->nblk_cap = dmd::csr_partials_per_column();
        ALLOC(h->ring_idx, sizeof(int32_t) * (size_t)h->slots * h->max_nnz);
        ALLOC(h->ring_val, sizeof(float2) * (size_t)h->slots * h->max_nnz);
        ALLOC(h->ring_nnz, sizeof(int32_t) * (size_t)h->slots);
        ALLOC(h->scatter, sizeof(float2) * (size_t)n);
        ALLOC(h->flag, sizeof(int));
        // projection through the union of the window's supports
        h->ucap = dmd::csr_union_cap(n, h->max_nnz);
        ALLOC(h->upos, sizeof(int32_t) * (size_t)n);
        ALLOC(h->ulist, sizeof(int32_t) * (size_t)h->ucap);
        ALLOC(h->ucount, 2 * sizeof(int));
        ALLOC(h->ublock, sizeof(float2) * (size_t)h->ucap * m);
        if (rc == DMD_OK && !dry && hipMemset(h->upos, 0xFF, sizeof(int32_t) * (size_t)n) != hipSuccess)
            rc = fail(DMD_E_DEVICE, "hipMemset(index map)");
    } else {
        ALLOC(h->ring, (size_t)h->slots * h->ld * h->elem_bytes);
        ALLOC(h->gfull, sizeof(double) * 64 * 64 * (size_t)dmd::gram_full_tiles(m) * dmd::gram_full_splits(m));
        h->bsplit_cap = dmd::gram_block_splits(m, h->kmax);
        ALLOC(h->bpartial, sizeof(double) * (size_t)h->bsplit_cap * h->slots * h->kmax);
        ALLOC(h->gblock, sizeof(double) * (size_t)h->slots * h->kmax);
        ALLOC(h->bflag, sizeof(int));
    }
    ALLOC(h->G, sizeof(double) * cw * h->slots * h->slots);
    ALLOC(h->partials, sizeof(double) * cw * (size_t)(m + 2) * h->nblk_cap);
    ALLOC(h->res_dev, h->L.bytes);
    ALLOC(h->V, sizeof(double) * cw * (size_t)m * r);
    ALLOC(h->At, sizeof(double) * cw * (size_t)r * r);
    ALLOC(h->W, sizeof(double) * 2 * (size_t)r * r);
    ALLOC(h->work, sizeof(double) * cw * 4 * (size_t)M * (M + 1));
    ALLOC(h->Vfull, sizeof(double) * cw * (size_t)m * m);
    ALLOC(h->Bphi, coef * 2 * (size_t)m * r);
    if (!h->cplx) {
        h->snap_B_bytes = (coef * 2 * (size_t)m * r + 255) / 256 * 256;
        ALLOC(h->snap_st, 2 * sizeof(DevState));
        ALLOC(h->snap_B, 2 * h->snap_B_bytes);
    }
    ALLOC(h->Bpod, coef * cw * (size_t)m * r);
    ALLOC(h->Bbg, coef * 2 * (size_t)m);
    h->sh_stride = (h->L.bytes + 255) / 256 * 256;
    if (h->kmax > 1) {
        const SetSizes z = set_sizes(h);
        const size_t ns = (size_t)h->kmax - 1;
        ALLOC(h->sh_dev, ns * h->sh_stride);
        ALLOC(h->sh_V, sizeof(double) * ns * z.V);
        ALLOC(h->sh_At, sizeof(double) * ns * z.At);
        ALLOC(h->sh_W, sizeof(double) * ns * z.W);
        ALLOC(h->sh_work, sizeof(double) * ns * z.work);
        ALLOC(h->sh_Vfull, sizeof(double) * ns * z.Vfull);
        ALLOC(h->sh_Bphi, ns * z.Bphi);
        ALLOC(h->sh_Bpod, ns * z.Bpod);
        h->cfrag_elems = dmd::project_block_frag_bytes(m, r, h->kmax) / sizeof(uint4);
        ALLOC(h->cfrag, 2 * h->cfrag_elems * sizeof(uint4));
        ALLOC(h->bdesc, 2 * sizeof(dmd::BlockDesc));
        if (rc == DMD_OK && !dry) {
            hipError_t e = hipHostMalloc((void**)&h->sh_host, ns * h->sh_stride,
                                         hipHostMallocMapped | hipHostMallocCoherent);
            if (e != hipSuccess) rc = fail(DMD_E_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
            else std::memset(h->sh_host, 0, ns * h->sh_stride);
        }
        if (rc == DMD_OK && !dry) {
            hipError_t e = hipHostGetDevicePointer((void**)&h->sh_host_dev, h->sh_host, 0);
            if (e != hipSuccess) rc = hip_fail(e, "hipHostGetDevicePointer");
        }
    }
    if (!h->cplx) ALLOC(h->solve_tbl, sizeof(dmd::SolveArgs) * (size_t)h->kmax);
#undef ALLOC
    if (dry) {
        *footprint = h->device_bytes;
        delete h;
        g_err.clear();
        return rc;
    }
    if (rc == DMD_OK) {
        hipError_t e = hipHostMalloc((void**)&h->res_host, h->L.bytes, hipHostMallocMapped | hipHostMallocCoherent);
        if (e != hipSuccess) rc = fail(DMD_E_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    if (rc == DMD_OK) {
        std::memset(h->res_host, 0, h->L.bytes);
        hipError_t e = hipHostGetDevicePointer((void**)&h->res_host_dev, h->res_host, 0);
        if (e != hipSuccess) rc = hip_fail(e, "hipHostGetDevicePointer");
    }
    if (rc == DMD_OK) {
        DevState init{};
        init.solve_status = dmd::ST_E_NOT_READY;
        std::memcpy(h->res_host, &init, sizeof(init));
        hipError_t e = hipMemcpy(h->res_dev, &init, sizeof(init), hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy(state)");
    }
    if (rc == DMD_OK && h->solve_tbl) {
        std::vector<dmd::SolveArgs> tbl(h->kmax);
        for (int e = 0; e + 1 < h->kmax; ++e) fill_shadow_args(h, tbl[e], e);
        fill_solve_args(h, tbl[h->kmax - 1]);
        hipError_t e = hipMemcpy(h->solve_tbl, tbl.data(), sizeof(dmd::SolveArgs) * tbl.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy(solve table)");
    }
    if (rc == DMD_OK) {
        hipError_t e = hipEventCreateWithFlags(&h->ev_last, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_solved, hipEventDisableTiming);
        for (int p = 0; p < 2 && e == hipSuccess; ++p) e = hipEventCreateWithFlags(&h->ev_proj[p], hipEventDisableTiming);
        for (int p = 0; p < 2 && e == hipSuccess; ++p) e = hipEventCreateWithFlags(&h->ev_sproj[p], hipEventDisableTiming);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = hip_fail(e, "event/sync");
    }
    if (rc != DMD_OK) {
        std::string msg = g_err;
        free_all(h);
        delete h;
        g_err = msg;
        return rc;
    }
    *out = h;
    g_err.clear();
    return DMD_OK;
}
}  // namespace

DMD_API int dmd_stream_create(int64_t n, int32_t m, int32_t r, const dmd_opts_t* opts,
                              dmd_stream_t** out) {
    return create_impl(n, m, r, opts, out, nullptr);
}

// Launch shapes of a stream (the tuner times candidates on streams of its own).
void dmd::stream_get_shapes(const dmd_stream* h, int* gram_iter, int* proj_form) {
    *gram_iter = h->gram_iter;
    *proj_form = h->proj_form;
}
void dmd::stream_set_shapes(dmd_stream* h, int gram_iter, int proj_form) {
    h->gram_iter = gram_iter;
    h->proj_form = proj_form;
}

DMD_API int dmd_stream_footprint(int64_t n, int32_t m, int32_t r, const dmd_opts_t* opts, int64_t* bytes) {
    if (!bytes) return fail(DMD_E_INVAL, "null bytes");
    *bytes = 0;
    return create_impl(n, m, r, opts, nullptr, bytes);
}

DMD_API int dmd_stream_destroy(dmd_stream_t* h) {
    if (!h) return DMD_OK;
    DeviceGuard g(h->device);
    if (h->has_last) (void)hipEventSynchronize(h->ev_last);
    for (int p = 0; p < 2; ++p) {
        if (h->proj_pending[p]) (void)hipEventSynchronize(h->ev_proj[p]);
        if (h->sproj_pending[p]) (void)hipEventSynchronize(h->ev_sproj[p]);
    }
    free_all(h);
    delete h;
    return DMD_OK;
}

DMD_API int dmd_stream_sync(dmd_stream_t* h) {
    if (int rc = check_handle(h)) return rc;
    DeviceGuard g(h->device);
    for (int p = 0; p < 2; ++p) {  // projections that run beside later pushes
        if (h->proj_pending[p]) HIP_TRY(hipEventSynchronize(h->ev_proj[p]));
        if (h->sproj_pending[p]) HIP_TRY(hipEventSynchronize(h->ev_sproj[p]));
    }
    DevState st;
    if (int rc = read_state(h, &st)) return rc;
    if (st.rejected_nonfinite > h->reported_nonfinite) {
        h->reported_nonfinite = st.rejected_nonfinite;
        return fail(DMD_E_NONFINITE, "%d snapshot(s) rejected: non-finite inner products", st.rejected_nonfinite);
    }
    if (st.rejected_index > h->reported_index) {
        h->reported_index = st.rejected_index;
        return fail(DMD_E_INVAL, "%d sparse snapshot(s) rejected: bad indices", st.rejected_index);
    }
    return DMD_OK;
}

namespace dmd {
__global__ void k_reset_state(DevState* st) {
    st->count = 0;
    st->oldest = 0;
    st->vprev_valid = 0;
    st->solve_status = ST_E_NOT_READY;
    st->r_eff = 0;
}
}  // namespace dmd

DMD_API int dmd_stream_reset(dmd_stream_t* h, void* stream) {
    if (int rc = check_handle(h)) return rc;
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    HIP_TRY(begin(h, s));
    hipLaunchKernelGGL(dmd::k_reset_state, dim3(1), dim3(1), 0, s, reinterpret_cast<DevState*>(h->res_dev));
    HIP_TRY(hipGetLastError());
    h->solve_enqueued = false;
    h->last_block_k = 0;
    h->last_packed = -1;
    h->snap_par = -1;
    HIP_TRY(end(h, s));
    return DMD_OK;
}

DMD_API int dmd_stream_push(dmd_stream_t* h, const void* x, void* stream) {
    if (int rc = check_handle(h)) return rc;
    if (!x) return fail(DMD_E_INVAL, "null snapshot");
    if (h->cplx) return fail(DMD_E_INVAL, "sparse stream: use dmd_stream_push_csr");
    if ((uintptr_t)x % h->elem_bytes) return fail(DMD_E_INVAL, "snapshot not %d-byte aligned", h->elem_bytes);
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    if (h->opts.auto_solve && h->snap_st) HIP_TRY(begin_single(h, s, (int)(h->snap_seq & 1)));
    else HIP_TRY(begin(h, s));
    // host memory: staged on `s` (the previous push that read the staging
    // buffer is ordered before this copy by begin / the stream itself)
    if (int rc = stage_input(h, &h->stage, (size_t)h->ld * h->elem_bytes, x, (size_t)h->n * h->elem_bytes, s, &x))
        return rc;
    DevState* st = reinterpret_cast<DevState*>(h->res_dev);
    int nblk = 0;
    hipError_t e = timed("gram_columns", s, [&] {
        if (h->elem_bytes == 8)
            return dmd::launch_gram_columns<double>(static_cast<const double*>(x), static_cast<double*>(h->ring),
                                                    h->ld, h->n, h->m, h->slots, h->partials, h->nblk_cap, st,
                                                    h->gram_iter, &nblk, s);
        return dmd::launch_gram_columns<float>(static_cast<const float*>(x), static_cast<float*>(h->ring), h->ld,
                                               h->n, h->m, h->slots, h->partials, h->nblk_cap, st, h->gram_iter,
                                               &nblk, s);
    });
    // with the tridiagonal solver the finalize and the solve are one launch
    const bool fuse = h->opts.auto_solve && h->use_trid;
    if (e == hipSuccess && !fuse)
        e = timed("gram_finalize", s,
                  [&] { return dmd::launch_gram_finalize(h->G, h->partials, nblk, h->m, h->slots, st, s); });
    if (e == hipSuccess && fuse) {
        dmd::SolveArgs a;
        fill_solve_args(h, a);
        e = timed("solve_sym", s, [&] { return dmd::launch_finalize_solve_trid(h->G, h->partials, nblk, a, s); });
    }
    if (e != hipSuccess) return hip_fail(e, "gram push launch");
    h->last_block_k = 0;
    h->last_packed = -1;
    h->snap_par = -1;
    if (h->opts.auto_solve)
        if (int rc = enqueue_solve(h, s, fuse)) return rc;
    HIP_TRY(end(h, s));
    return DMD_OK;
}

DMD_API int dmd_stream_push_csr(dmd_stream_t* h, int32_t nnz, const int32_t* idx, const void* val,
                                void* stream) {
    if (int rc = check_handle(h)) return rc;
    if (!h->cplx) return fail(DMD_E_INVAL, "dense stream: use dmd_stream_push");
    if (nnz < 0 || nnz > h->max_nnz) return fail(DMD_E_INVAL, "nnz must be in [0, max_nnz=%d] (got %d)", h->max_nnz, nnz);
    if (nnz > 0 && (!idx || !val)) return fail(DMD_E_INVAL, "null idx or val");
    if ((uintptr_t)idx % 4 || (uintptr_t)val % 8) return fail(DMD_E_INVAL, "idx must be 4-byte and val 8-byte aligned");
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    HIP_TRY(begin(h, s));
    if (nnz > 0) {
        const void* pi = idx;
        const void* pv = val;
        if (int rc = stage_input(h, &h->stage_idx, sizeof(int32_t) * (size_t)h->max_nnz, idx,
                                 sizeof(int32_t) * (size_t)nnz, s, &pi))
            return rc;
        if (int rc = stage_input(h, &h->stage_val, sizeof(float2) * (size_t)h->max_nnz, val,
                                 sizeof(float2) * (size_t)nnz, s, &pv))
            return rc;
        idx = static_cast<const int32_t*>(pi);
        val = pv;
    }
    DevState* st = reinterpret_cast<DevState*>(h->res_dev);
    hipError_t e = timed("csr_gram", s, [&] {
        return dmd::launch_csr_push(idx, static_cast<const float2*>(val), nnz, h->n, h->ring_idx, h->ring_val,
                                    h->ring_nnz, h->max_nnz, h->m, h->scatter, h->flag, h->G, h->partials, st, s);
    });
    if (e != hipSuccess) return hip_fail(e, "sparse push launch");
    h->last_block_k = 0;
    h->last_packed = -1;
    h->snap_par = -1;
    if (h->opts.auto_solve)
        if (int rc = enqueue_solve(h, s)) return rc;
    HIP_TRY(end(h, s));
    return DMD_OK;
}

namespace {
// Block projection arguments of a k-column push packed into parity par.
void fill_block_project_args(dmd_stream* h, dmd::BlockProjectArgs& a, int k, int par) {
    a = dmd::BlockProjectArgs{};
    a.ring = h->ring;
    a.ld = h->ld;
    a.n = h->n;
    a.m = h->m;
    a.r = h->r;
    a.slots = h->slots;
    a.k = k;
    a.kmax = h->kmax;
    a.st = reinterpret_cast<const DevState*>(h->res_dev);
    a.shadow = h->sh_dev;
    a.shadow_stride = (int)h->sh_stride;
    a.Bphi = static_cast<const float*>(h->Bphi);
    a.Bphi_sets = static_cast<const float*>(h->sh_Bphi);
    a.bphi_stride = (int64_t)set_sizes(h).Bphi / sizeof(float);
    a.bf16x3 = h->opts.precision == DMD_PREC_BF16X3;
    a.form = h->proj_form;
    a.cfrag = h->cfrag + (size_t)par * h->cfrag_elems;
    a.desc = h->bdesc + par;
}
}  // namespace

DMD_API int dmd_stream_push_block(dmd_stream_t* h, const void* X_new, int64_t ldx, int32_t k,
                                  void* stream) {
    if (int rc = check_handle(h)) return rc;
    if (h->cplx) return fail(DMD_E_UNSUPPORTED, "block pushes are for dense streams");
    if (!X_new) return fail(DMD_E_INVAL, "null X_new");
    if (k < 1 || k > h->kmax) return fail(DMD_E_INVAL, "k must be in [1, max_block=%d] (got %d)", h->kmax, k);
    if (ldx < h->n) return fail(DMD_E_INVAL, "ldx < n");
    if ((uintptr_t)X_new % h->elem_bytes) return fail(DMD_E_INVAL, "X_new not %d-byte aligned", h->elem_bytes);
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    const int par = (int)(h->block_seq & 1);
    HIP_TRY(begin_block(h, s, par));
    dmd::BlockArgs a{};
    a.ring = h->ring;
    a.ld = h->ld;
    a.n = h->n;
    a.xnew = X_new;
    a.ldx = ldx;
    a.m = h->m;
    a.slots = h->slots;
    a.k = k;
    a.x_aligned = ((uintptr_t)X_new % 16 == 0) && ((ldx * h->elem_bytes) % 16 == 0);
    a.partial = h->bpartial;
    a.gblock = h->gblock;
    a.flag = h->bflag;
    a.G = h->G;
    a.st = reinterpret_cast<DevState*>(h->res_dev);
    a.shadow = h->sh_dev;
    a.shadow_stride = (int)h->sh_stride;
    a.kmax = h->kmax;
    HIP_TRY(timed("gram_block", s, [&] { return dmd::launch_gram_block(a, h->elem_bytes == 8, s); }));
    h->last_block_k = 0;
    h->last_packed = -1;
    h->snap_par = -1;
    if (h->opts.auto_solve) {
        const dmd::SolveArgs* t = h->solve_tbl + (h->kmax - k);
        const bool lds = h->m + (h->m & 1) <= 64;
        HIP_TRY(timed("block_solve", s, [&] {
            hipError_t e = h->use_trid ? dmd::launch_trid_grouped(t, lds ? k : 0, t, lds ? 0 : k, s)
                                       : dmd::launch_jacobi_grouped(t, lds ? k : 0, t, lds ? 0 : k, s);
            return e != hipSuccess ? e : dmd::launch_eig_grouped(t, k, s);
        }));
        HIP_TRY(hipEventRecord(h->ev_solved, s));
        h->solve_enqueued = true;
        h->last_block_k = k;
        if (h->elem_bytes == 4 && !h->coef_f64 && dmd::project_block_fits(h->m, k, h->r)) {
            dmd::BlockProjectArgs pa;
            fill_block_project_args(h, pa, k, par);
            HIP_TRY(timed("pack_block", s, [&] { return dmd::launch_pack_block(pa, s); }));
            h->last_packed = par;
        }
    }
    ++h->block_seq;
    HIP_TRY(end(h, s));
    return DMD_OK;
}

DMD_API int dmd_stream_block_eigs(dmd_stream_t* h, int32_t* k, double* lam_re, double* lam_im, double* sigma,
                                  int64_t ld, int32_t* r_eff, int32_t* status) {
    if (int rc = check_handle(h)) return rc;
    if (!k) return fail(DMD_E_INVAL, "null k");
    *k = 0;
    if (h->last_block_k == 0) return fail(DMD_E_NOT_READY, "the latest push was not a solved block push");
    if ((lam_re || lam_im || sigma) && ld < h->r) return fail(DMD_E_INVAL, "ld < r");
    DeviceGuard g(h->device);
    if (int rc = wait_solved(h)) return rc;
    const int kb = h->last_block_k;
    *k = kb;
    for (int w = 0; w < kb; ++w) {
        const char* res = (w == kb - 1) ? h->res_host : h->sh_host + (size_t)(h->kmax - kb + w) * h->sh_stride;
        const DevState& st = *reinterpret_cast<const DevState*>(res);
        const bool rejected = reinterpret_cast<const DevState*>(h->res_host)->block_rejected != 0;
        int code = st.solve_status;
        if (rejected) code = DMD_E_NONFINITE;
        const int re = (code == DMD_OK || code == DMD_W_RANK) ? st.r_eff : 0;
        if (status) status[w] = code;
        if (r_eff) r_eff[w] = re;
        const double* sg = reinterpret_cast<const double*>(res + h->L.sigma_off);
        const double* lm = reinterpret_cast<const double*>(res + h->L.lam_off);
        for (int i = 0; i < re; ++i) {
            if (lam_re) lam_re[w * ld + i] = lm[2 * i];
            if (lam_im) lam_im[w * ld + i] = lm[2 * i + 1];
            if (sigma) sigma[w * ld + i] = sg[i];
        }
    }
    return solve_status(h);
}

DMD_API int dmd_stream_block_modes(dmd_stream_t* h, void* phi, int64_t ld, int64_t ldw, void* stream) {
    if (int rc = check_handle(h)) return rc;
    if (!phi) return fail(DMD_E_INVAL, "null output");
    if (ld < h->n) return fail(DMD_E_INVAL, "ld < n");
    if (ldw < ld * h->r) return fail(DMD_E_INVAL, "ldw < ld * r");
    if (h->last_block_k == 0) return fail(DMD_E_NOT_READY, "the latest push was not a solved block push");
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    const int k = h->last_block_k;
    const size_t celem = h->coef_f64 ? 16 : 8;  // complex128 or complex64
    if (h->last_packed >= 0) {
        // reads only the ring columns of the block's windows and the inputs
        // packed after its solves: ordered after the push, not after later
        // calls' other work; later calls that touch those inputs wait for it
        const int par = h->last_packed;
        if (h->has_last && h->last_stream != s) HIP_TRY(hipStreamWaitEvent(s, h->ev_last, 0));
        if (h->proj_pending[par] && h->proj_stream[par] != s) HIP_TRY(hipStreamWaitEvent(s, h->ev_proj[par], 0));
        dmd::BlockProjectArgs a;
        fill_block_project_args(h, a, k, par);
        a.out = static_cast<float2*>(phi);
        a.ldo = ld;
        a.ldw = ldw;
        a.out16 = (reinterpret_cast<uintptr_t>(phi) % 16 == 0) && ld % 2 == 0 && ldw % 2 == 0;
        HIP_TRY(timed("project_block", s, [&] { return dmd::launch_project_block(a, s); }));
        HIP_TRY(hipEventRecord(h->ev_proj[par], s));
        h->proj_stream[par] = s;
        h->proj_pending[par] = true;
        return DMD_OK;
    }
    HIP_TRY(begin(h, s));
    {
        // FP64 data or coefficients, or tiles beyond the LDS: one projection per window from its own state
        for (int w = 0; w < k; ++w) {
            dmd::ProjectArgs a;
            char* out = static_cast<char*>(phi) + (size_t)w * ldw * celem;
            fill_project_args(h, a, out, ld, true);
            if (w < k - 1) {
                const int set = h->kmax - k + w;
                a.st = reinterpret_cast<const DevState*>(h->sh_dev + (size_t)set * h->sh_stride);
                a.B = static_cast<char*>(h->sh_Bphi) + (size_t)set * set_sizes(h).Bphi;
            }
            a.block_only = 1;
            HIP_TRY(timed("project_block", s, [&] { return dmd::launch_project(a, s); }));
        }
    }
    HIP_TRY(end(h, s));
    return DMD_OK;
}

DMD_API int dmd_stream_solve(dmd_stream_t* h, void* stream) {
    if (int rc = check_handle(h)) return rc;
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    HIP_TRY(begin(h, s));
    if (int rc = enqueue_solve(h, s)) return rc;
    HIP_TRY(end(h, s));
    return DMD_OK;
}

DMD_API int dmd_stream_eigs(dmd_stream_t* h, double* lam_re, double* lam_im, double* sigma,
                            int32_t* r_eff) {
    if (int rc = check_handle(h)) return rc;
    DeviceGuard g(h->device);
    if (int rc = wait_solved(h)) return rc;
    const DevState& st = host_state(h);
    const int k = st.solve_status == dmd::ST_E_NOT_READY ? 0 : st.r_eff;
    if (r_eff) *r_eff = k;
    const double* sig = reinterpret_cast<const double*>(h->res_host + h->L.sigma_off);
    const double* lam = reinterpret_cast<const double*>(h->res_host + h->L.lam_off);
    for (int i = 0; i < k; ++i) {
        if (lam_re) lam_re[i] = lam[2 * i];
        if (lam_im) lam_im[i] = lam[2 * i + 1];
        if (sigma) sigma[i] = sig[i];
    }
    return solve_status(h);
}

DMD_API int dmd_stream_svd(dmd_stream_t* h, double* sigma, double* V, int64_t ldv, int32_t* r_eff) {
    if (int rc = check_handle(h)) return rc;
    if (V && ldv < h->m) return fail(DMD_E_INVAL, "ldv < m");
    DeviceGuard g(h->device);
    if (int rc = wait_solved(h)) return rc;
    const DevState& st = host_state(h);
    const int k = st.solve_status == dmd::ST_E_NOT_READY ? 0 : st.r_eff;
    if (r_eff) *r_eff = k;
    if (sigma && k > 0) std::memcpy(sigma, h->res_host + h->L.sigma_off, sizeof(double) * h->m);
    if (V && k > 0) {
        const int cw = h->cplx ? 2 : 1;
        HIP_TRY(hipMemcpy2D(V, sizeof(double) * cw * ldv, h->V, sizeof(double) * cw * h->m,
                            sizeof(double) * cw * h->m, k, hipMemcpyDeviceToHost));
    }
    return solve_status(h);
}

DMD_API int dmd_stream_atilde(dmd_stream_t* h, double* Atilde, int64_t lda, double* W, int64_t ldw,
                              int32_t* r_eff) {
    if (int rc = check_handle(h)) return rc;
    DeviceGuard g(h->device);
    if (int rc = wait_solved(h)) return rc;
    const DevState& st = host_state(h);
    const int k = st.solve_status == dmd::ST_E_NOT_READY ? 0 : st.r_eff;
    if (r_eff) *r_eff = k;
    if ((Atilde && lda < k) || (W && ldw < k)) return fail(DMD_E_INVAL, "leading dimension < r_eff");
    const int cw = h->cplx ? 2 : 1;
    if (Atilde && k > 0)
        HIP_TRY(hipMemcpy2D(Atilde, sizeof(double) * cw * lda, h->At, sizeof(double) * cw * k,
                            sizeof(double) * cw * k, k, hipMemcpyDeviceToHost));
    if (W && k > 0)
        HIP_TRY(hipMemcpy2D(W, sizeof(double) * 2 * ldw, h->W, sizeof(double) * 2 * k, sizeof(double) * 2 * k, k,
                            hipMemcpyDeviceToHost));
    return solve_status(h);
}

DMD_API int dmd_stream_gram(dmd_stream_t* h, double* G, int64_t ldg, int32_t* ncols) {
    if (int rc = check_handle(h)) return rc;
    if (!G || ldg < h->m + 1) return fail(DMD_E_INVAL, "null G or ldg < m+1");
    DeviceGuard g(h->device);
    DevState st;
    if (int rc = read_state(h, &st)) return rc;
    const int cw = h->cplx ? 2 : 1;
    const size_t cnt = (size_t)cw * h->slots * h->slots;
    double* tmp = new (std::nothrow) double[cnt];
    if (!tmp) return fail(DMD_E_NOMEM, "host allocation failed");
    hipError_t e = hipMemcpy(tmp, h->G, sizeof(double) * cnt, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        delete[] tmp;
        return hip_fail(e, "hipMemcpy(G)");
    }
    if (ncols) *ncols = st.count;
    for (int j = 0; j < st.count; ++j)
        for (int i = 0; i < st.count; ++i) {
            const int si = dmd::slot_of(st.oldest, i, h->slots), sj = dmd::slot_of(st.oldest, j, h->slots);
            for (int c = 0; c < cw; ++c) G[cw * (i + j * ldg) + c] = tmp[cw * (si + (size_t)sj * h->slots) + c];
        }
    delete[] tmp;
    return DMD_OK;
}

// ------------------------------------------------------------ spatial -> Fourier ingest (Sec. 3.5)

namespace {
// Bin k of N as a signed wavenumber (FFT order: 0, 1, ..., then negatives).
int signed_bin(int k, int N) { return k < (N + 1) / 2 ? k : k - N; }

void free_fourier(dmd_stream* h) {
    void* bufs[] = {h->f_idx, h->f_ky, h->f_col, h->f_kx, h->f_twW, h->f_twH, h->f_R, h->f_val};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    h->f_idx = h->f_ky = h->f_col = h->f_kx = nullptr;
    h->f_twW = h->f_twH = h->f_R = nullptr;
    h->f_val = nullptr;
    h->four_H = h->four_W = h->four_nkeep = h->four_nkx = 0;
    h->four_support.clear();
}

std::vector<double2> roots_of_unity(int N) {
    std::vector<double2> w(N);
    for (int j = 0; j < N; ++j) {
        const double t = 2.0 * 3.14159265358979323846 * (double)j / (double)N;
        w[j] = double2{std::cos(t), -std::sin(t)};
    }
    return w;
}

template <typename T>
int upload(dmd_stream* h, T** dst, const std::vector<T>& src) {
    if (int rc = dev_alloc(h, dst, sizeof(T) * src.size())) return rc;
    HIP_TRY(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return DMD_OK;
}
}  // namespace

DMD_API int dmd_stream_fourier_setup(dmd_stream_t* h, int32_t height, int32_t width, int32_t nkeep) {
    if (int rc = check_handle(h)) return rc;
    if (!h->cplx) return fail(DMD_E_UNSUPPORTED, "the Fourier ingest feeds sparse (DMD_C64_CSR) streams");
    if (height < 1 || width < 1 || (int64_t)height * width != h->n)
        return fail(DMD_E_INVAL, "height x width must equal n = %lld", (long long)h->n);
    if (width > dmd::kFourierMaxW) return fail(DMD_E_INVAL, "width must be <= %d", dmd::kFourierMaxW);
    if (nkeep < 1 || nkeep > h->max_nnz) return fail(DMD_E_INVAL, "nkeep must be in [1, max_nnz=%d]", h->max_nnz);
    DeviceGuard g(h->device);
    if (h->has_last) HIP_TRY(hipEventSynchronize(h->ev_last));  // buffers may be in use by earlier pushes
    free_fourier(h);
    // the nkeep bins of smallest ky^2 + kx^2 (signed), ties by flattened index
    const int64_t n = h->n;
    std::vector<std::pair<int64_t, int32_t>> key((size_t)n);
    for (int y = 0; y < height; ++y) {
        const int64_t ky = signed_bin(y, height);
        for (int x = 0; x < width; ++x) {
            const int64_t kx = signed_bin(x, width);
            const int32_t i = y * width + x;
            key[(size_t)i] = {ky * ky + kx * kx, i};
        }
    }
    std::nth_element(key.begin(), key.begin() + (nkeep - 1), key.end());
    std::vector<int32_t> idx(nkeep);
    for (int c = 0; c < nkeep; ++c) idx[c] = key[(size_t)c].second;
    // nth_element leaves the nkeep smallest (k^2, index) pairs first, in any order
    std::sort(idx.begin(), idx.end());
    std::vector<int32_t> kxs;
    for (int32_t i : idx) kxs.push_back(i % width);
    std::sort(kxs.begin(), kxs.end());
    kxs.erase(std::unique(kxs.begin(), kxs.end()), kxs.end());
    std::vector<int32_t> ky(nkeep), col(nkeep);
    for (int c = 0; c < nkeep; ++c) {
        ky[c] = idx[c] / width;
        col[c] = (int32_t)(std::lower_bound(kxs.begin(), kxs.end(), idx[c] % width) - kxs.begin());
    }
    int rc = DMD_OK;
    if (!rc) rc = upload(h, &h->f_idx, idx);
    if (!rc) rc = upload(h, &h->f_ky, ky);
    if (!rc) rc = upload(h, &h->f_col, col);
    if (!rc) rc = upload(h, &h->f_kx, kxs);
    if (!rc) rc = upload(h, &h->f_twW, roots_of_unity(width));
    if (!rc) rc = upload(h, &h->f_twH, roots_of_unity(height));
    if (!rc) rc = dev_alloc(h, &h->f_R, sizeof(double2) * (size_t)height * kxs.size());
    if (!rc) rc = dev_alloc(h, &h->f_val, sizeof(float2) * (size_t)nkeep);
    if (rc) {
        free_fourier(h);
        return rc;
    }
    h->four_H = height;
    h->four_W = width;
    h->four_nkeep = nkeep;
    h->four_nkx = (int)kxs.size();
    h->four_support = idx;
    return DMD_OK;
}

DMD_API int dmd_stream_fourier_support(dmd_stream_t* h, int32_t* idx, int32_t cap, int32_t* nkeep) {
    if (int rc = check_handle(h)) return rc;
    if (!nkeep) return fail(DMD_E_INVAL, "null nkeep");
    if (h->four_nkeep == 0) return fail(DMD_E_NOT_READY, "no Fourier ingest set up");
    *nkeep = h->four_nkeep;
    if (idx) {
        if (cap < h->four_nkeep) return fail(DMD_E_INVAL, "cap < nkeep (%d)", h->four_nkeep);
        std::memcpy(idx, h->four_support.data(), sizeof(int32_t) * h->four_nkeep);
    }
    return DMD_OK;
}

DMD_API int dmd_stream_push_fourier(dmd_stream_t* h, const float* frame, int64_t ld_row, void* stream) {
    if (int rc = check_handle(h)) return rc;
    if (h->four_nkeep == 0) return fail(DMD_E_NOT_READY, "no Fourier ingest set up (dmd_stream_fourier_setup)");
    if (!frame) return fail(DMD_E_INVAL, "null frame");
    if (ld_row < h->four_W) return fail(DMD_E_INVAL, "ld_row < width");
    if ((uintptr_t)frame % 4) return fail(DMD_E_INVAL, "frame not 4-byte aligned");
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    HIP_TRY(begin(h, s));
    dmd::FourierArgs a{};
    a.frame = frame;
    a.ld_row = ld_row;
    a.H = h->four_H;
    a.W = h->four_W;
    a.kx = h->f_kx;
    a.nkx = h->four_nkx;
    a.ky = h->f_ky;
    a.col = h->f_col;
    a.nkeep = h->four_nkeep;
    a.twW = h->f_twW;
    a.twH = h->f_twH;
    a.R = h->f_R;
    a.val = h->f_val;
    a.scale = 1.0 / std::sqrt((double)h->n);
    HIP_TRY(timed("fourier", s, [&] { return dmd::launch_fourier(a, s); }));
    HIP_TRY(end(h, s));
    return dmd_stream_push_csr(h, h->four_nkeep, h->f_idx, h->f_val, stream);
}

// ------------------------------------------------------------ checkpoint / resume

namespace {
// A checkpoint: this header, then the window's Gram (count x count, window
// order, column-major FP64; interleaved complex for sparse streams), then the
// window's snapshots in window order (dense: count x n elements; sparse: the
// count nnz values, then each snapshot's indices and complex64 values).
struct CkptHeader {
    char magic[8];          // "DMDCKPT1"
    int32_t version;        // 1
    int32_t dtype;
    int64_t n;
    int32_t m, r, count, max_nnz;
    int32_t pushes, solves, rejected_nonfinite, rejected_index;
    int64_t gram_bytes, data_bytes;
};
constexpr char kCkptMagic[8] = {'D', 'M', 'D', 'C', 'K', 'P', 'T', '1'};

// Bytes of the window's snapshots in a checkpoint (sparse: needs the nnz of each).
int ckpt_data_bytes(dmd_stream* h, const DevState& st, std::vector<int32_t>* nnz, int64_t* bytes) {
    if (!h->cplx) {
        *bytes = (int64_t)st.count * h->n * h->elem_bytes;
        return DMD_OK;
    }
    std::vector<int32_t> all(h->slots);
    HIP_TRY(hipMemcpy(all.data(), h->ring_nnz, sizeof(int32_t) * h->slots, hipMemcpyDeviceToHost));
    int64_t b = sizeof(int32_t) * (int64_t)st.count;
    nnz->resize(st.count);
    for (int j = 0; j < st.count; ++j) {
        (*nnz)[j] = all[dmd::slot_of(st.oldest, j, h->slots)];
        b += (int64_t)(*nnz)[j] * (sizeof(int32_t) + sizeof(float2));
    }
    *bytes = b;
    return DMD_OK;
}
}  // namespace

DMD_API int dmd_stream_checkpoint_bytes(dmd_stream_t* h, int64_t* bytes) {
    if (int rc = check_handle(h)) return rc;
    if (!bytes) return fail(DMD_E_INVAL, "null bytes");
    DeviceGuard g(h->device);
    DevState st;
    if (int rc = read_state(h, &st)) return rc;
    std::vector<int32_t> nnz;
    int64_t data = 0;
    if (int rc = ckpt_data_bytes(h, st, &nnz, &data)) return rc;
    const int cw = h->cplx ? 2 : 1;
    *bytes = (int64_t)sizeof(CkptHeader) + (int64_t)sizeof(double) * cw * st.count * st.count + data;
    return DMD_OK;
}

DMD_API int dmd_stream_save(dmd_stream_t* h, void* buf, int64_t bytes) {
    if (int rc = check_handle(h)) return rc;
    if (!buf) return fail(DMD_E_INVAL, "null buffer");
    DeviceGuard g(h->device);
    DevState st;
    if (int rc = read_state(h, &st)) return rc;  // waits for the handle's state-changing work
    std::vector<int32_t> nnz;
    int64_t data = 0;
    if (int rc = ckpt_data_bytes(h, st, &nnz, &data)) return rc;
    const int cw = h->cplx ? 2 : 1;
    const int64_t gbytes = (int64_t)sizeof(double) * cw * st.count * st.count;
    if (bytes < (int64_t)sizeof(CkptHeader) + gbytes + data)
        return fail(DMD_E_INVAL, "buffer too small (%lld < %lld bytes)", (long long)bytes,
                    (long long)(sizeof(CkptHeader) + gbytes + data));
    char* out = static_cast<char*>(buf);
    CkptHeader hd{};
    std::memcpy(hd.magic, kCkptMagic, 8);
    hd.version = 1;
    hd.dtype = h->opts.dtype;
    hd.n = h->n;
    hd.m = h->m;
    hd.r = h->r;
    hd.count = st.count;
    hd.max_nnz = h->cplx ? h->max_nnz : 0;
    hd.pushes = st.pushes;
    hd.solves = st.solves;
    hd.rejected_nonfinite = st.rejected_nonfinite;
    hd.rejected_index = st.rejected_index;
    hd.gram_bytes = gbytes;
    hd.data_bytes = data;
    std::memcpy(out, &hd, sizeof(hd));
    out += sizeof(hd);
    // Gram in window order
    std::vector<double> G((size_t)cw * h->slots * h->slots);
    HIP_TRY(hipMemcpy(G.data(), h->G, sizeof(double) * G.size(), hipMemcpyDeviceToHost));
    double* go = reinterpret_cast<double*>(out);
    for (int j = 0; j < st.count; ++j)
        for (int i = 0; i < st.count; ++i) {
            const int si = dmd::slot_of(st.oldest, i, h->slots), sj = dmd::slot_of(st.oldest, j, h->slots);
            for (int c = 0; c < cw; ++c)
                go[cw * (i + (size_t)j * st.count) + c] = G[cw * (si + (size_t)sj * h->slots) + c];
        }
    out += gbytes;
    // snapshots in window order
    if (!h->cplx) {
        const size_t col = (size_t)h->n * h->elem_bytes;
        for (int j = 0; j < st.count; ++j) {
            const char* src = static_cast<const char*>(h->ring) +
                              (size_t)dmd::slot_of(st.oldest, j, h->slots) * h->ld * h->elem_bytes;
            HIP_TRY(hipMemcpy(out + j * col, src, col, hipMemcpyDeviceToHost));
        }
    } else {
        std::memcpy(out, nnz.data(), sizeof(int32_t) * st.count);
        out += sizeof(int32_t) * st.count;
        for (int j = 0; j < st.count; ++j) {
            const size_t sl = (size_t)dmd::slot_of(st.oldest, j, h->slots);
            HIP_TRY(hipMemcpy(out, h->ring_idx + sl * h->max_nnz, sizeof(int32_t) * nnz[j], hipMemcpyDeviceToHost));
            out += sizeof(int32_t) * nnz[j];
            HIP_TRY(hipMemcpy(out, h->ring_val + sl * h->max_nnz, sizeof(float2) * nnz[j], hipMemcpyDeviceToHost));
            out += sizeof(float2) * nnz[j];
        }
    }
    return DMD_OK;
}

DMD_API int dmd_stream_restore(dmd_stream_t* h, const void* buf, int64_t bytes, void* stream) {
    if (int rc = check_handle(h)) return rc;
    if (!buf || bytes < (int64_t)sizeof(CkptHeader)) return fail(DMD_E_INVAL, "null or short checkpoint");
    CkptHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    if (std::memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.version != 1)
        return fail(DMD_E_INVAL, "not a checkpoint of this library");
    if (hd.dtype != h->opts.dtype || hd.n != h->n || hd.m != h->m || hd.r != h->r)
        return fail(DMD_E_INVAL, "checkpoint of another shape (dtype %d, n %lld, m %d, r %d)", hd.dtype,
                    (long long)hd.n, hd.m, hd.r);
    const int cw = h->cplx ? 2 : 1;
    if (hd.count < 0 || hd.count > h->m + 1 ||
        hd.gram_bytes != (int64_t)sizeof(double) * cw * hd.count * hd.count || hd.data_bytes < 0 ||
        bytes < (int64_t)sizeof(CkptHeader) + hd.gram_bytes + hd.data_bytes)
        return fail(DMD_E_INVAL, "truncated or inconsistent checkpoint");
    const char* in = static_cast<const char*>(buf) + sizeof(hd);
    const double* gi = reinterpret_cast<const double*>(in);
    const char* data = in + hd.gram_bytes;
    // validate the snapshot part before touching the device
    std::vector<int32_t> nnz;
    if (!h->cplx) {
        if (hd.data_bytes != (int64_t)hd.count * h->n * h->elem_bytes) return fail(DMD_E_INVAL, "inconsistent checkpoint");
    } else {
        if (hd.data_bytes < (int64_t)sizeof(int32_t) * hd.count) return fail(DMD_E_INVAL, "inconsistent checkpoint");
        nnz.resize(hd.count);
        if (hd.count > 0) std::memcpy(nnz.data(), data, sizeof(int32_t) * hd.count);
        int64_t b = sizeof(int32_t) * (int64_t)hd.count;
        for (int j = 0; j < hd.count; ++j) {
            if (nnz[j] < 0 || nnz[j] > h->max_nnz)
                return fail(DMD_E_INVAL, "checkpoint snapshot %d has %d nonzeros (max_nnz %d)", j, nnz[j], h->max_nnz);
            b += (int64_t)nnz[j] * (sizeof(int32_t) + sizeof(float2));
        }
        if (b != hd.data_bytes) return fail(DMD_E_INVAL, "inconsistent checkpoint");
        // the indices become addresses in the sparse kernels (scatter, index
        // map, projection rows): the rule of dmd_stream_push_csr applies
        const char* p = data + sizeof(int32_t) * hd.count;
        for (int j = 0; j < hd.count; ++j) {
            int32_t prev = -1;
            for (int e = 0; e < nnz[j]; ++e) {
                int32_t i;
                std::memcpy(&i, p + sizeof(int32_t) * (size_t)e, sizeof(i));
                if (i <= prev || (int64_t)i >= h->n)
                    return fail(DMD_E_INVAL, "checkpoint snapshot %d: index %d at entry %d not strictly increasing in [0, n)",
                                j, i, e);
                prev = i;
            }
            p += (sizeof(int32_t) + sizeof(float2)) * (size_t)nnz[j];
        }
    }
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    HIP_TRY(begin(h, s));
    HIP_TRY(hipStreamSynchronize(s));  // the window is rewritten from host memory below
    // window snapshot j goes to slot j (oldest = 0); the other slots keep
    // whatever they hold: they are outside the window
    if (!h->cplx) {
        const size_t col = (size_t)h->n * h->elem_bytes;
        for (int j = 0; j < hd.count; ++j)
            HIP_TRY(hipMemcpy(static_cast<char*>(h->ring) + (size_t)j * h->ld * h->elem_bytes, data + j * col, col,
                              hipMemcpyHostToDevice));
    } else {
        const char* p = data + sizeof(int32_t) * hd.count;
        std::vector<int32_t> all(h->slots, 0);
        for (int j = 0; j < hd.count; ++j) {
            all[j] = nnz[j];
            HIP_TRY(hipMemcpy(h->ring_idx + (size_t)j * h->max_nnz, p, sizeof(int32_t) * nnz[j], hipMemcpyHostToDevice));
            p += sizeof(int32_t) * nnz[j];
            HIP_TRY(hipMemcpy(h->ring_val + (size_t)j * h->max_nnz, p, sizeof(float2) * nnz[j], hipMemcpyHostToDevice));
            p += sizeof(float2) * nnz[j];
        }
        HIP_TRY(hipMemcpy(h->ring_nnz, all.data(), sizeof(int32_t) * h->slots, hipMemcpyHostToDevice));
    }
    std::vector<double> G((size_t)cw * h->slots * h->slots, 0.0);
    for (int j = 0; j < hd.count; ++j)
        for (int i = 0; i < hd.count; ++i)
            for (int c = 0; c < cw; ++c) G[cw * (i + (size_t)j * h->slots) + c] = gi[cw * (i + (size_t)j * hd.count) + c];
    HIP_TRY(hipMemcpy(h->G, G.data(), sizeof(double) * G.size(), hipMemcpyHostToDevice));
    DevState st{};
    st.oldest = 0;
    st.count = hd.count;
    st.pushes = hd.pushes;
    st.solves = hd.solves;
    st.rejected_nonfinite = hd.rejected_nonfinite;
    st.rejected_index = hd.rejected_index;
    st.solve_status = dmd::ST_E_NOT_READY;
    HIP_TRY(hipMemcpy(h->res_dev, &st, sizeof(st), hipMemcpyHostToDevice));
    h->reported_nonfinite = hd.rejected_nonfinite;
    h->reported_index = hd.rejected_index;
    h->solve_enqueued = false;
    h->last_block_k = 0;
    h->last_packed = -1;
    h->snap_par = -1;
    if (h->opts.auto_solve)
        if (int rc = enqueue_solve(h, s)) return rc;
    HIP_TRY(end(h, s));
    return DMD_OK;
}

static int project(dmd_stream_t* h, void* out, int64_t ld, void* stream, bool modes) {
    if (int rc = check_handle(h)) return rc;
    if (!out) return fail(DMD_E_INVAL, "null output");
    if (ld < h->n) return fail(DMD_E_INVAL, "ld < n");
    if (!h->solve_enqueued) return fail(DMD_E_NOT_READY, "no solve has been enqueued");
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    if (h->cplx) {
        HIP_TRY(begin(h, s));
        HIP_TRY(timed("csr_project", s, [&] {
            return dmd::launch_csr_project(reinterpret_cast<const DevState*>(h->res_dev), h->ring_idx, h->ring_val,
                                           h->ring_nnz, h->max_nnz, h->m, modes ? 1 : 0,
                                           static_cast<const float2*>(modes ? h->Bphi : h->Bpod), h->r,
                                           static_cast<float2*>(out), ld, h->n,
                                           dmd::CsrUnionScratch{h->upos, h->ulist, h->ucount, h->ucount + 1,
                                                                h->ucap, h->ublock},
                                           s);
        }));
        HIP_TRY(end(h, s));
        return DMD_OK;
    }
    dmd::ProjectArgs a;
    fill_project_args(h, a, out, ld, modes);
    if (modes && h->snap_par >= 0) {
        // the latest solve's snapshot: after that solve, beside the next push
        const int par = h->snap_par;
        if (h->has_last && h->last_stream != s) HIP_TRY(hipStreamWaitEvent(s, h->ev_last, 0));
        if (h->sproj_pending[par] && h->sproj_stream[par] != s) HIP_TRY(hipStreamWaitEvent(s, h->ev_sproj[par], 0));
        a.st = h->snap_st + par;
        a.B = h->snap_B + par * h->snap_B_bytes;
        HIP_TRY(timed("project_modes", s, [&] { return dmd::launch_project(a, s); }));
        HIP_TRY(hipEventRecord(h->ev_sproj[par], s));
        h->sproj_stream[par] = s;
        h->sproj_pending[par] = true;
        return DMD_OK;
    }
    HIP_TRY(begin(h, s));
    HIP_TRY(timed(modes ? "project_modes" : "project_pod", s, [&] { return dmd::launch_project(a, s); }));
    HIP_TRY(end(h, s));
    return DMD_OK;
}

DMD_API int dmd_stream_modes(dmd_stream_t* h, void* phi, int64_t ld, void* stream) {
    return project(h, phi, ld, stream, true);
}

DMD_API int dmd_stream_pod(dmd_stream_t* h, void* U, int64_t ld, void* stream) {
    return project(h, U, ld, stream, false);
}

DMD_API int dmd_stream_amplitudes(dmd_stream_t* h, double* b_re, double* b_im, int32_t* bg_index,
                                  int32_t* r_eff) {
    if (int rc = check_handle(h)) return rc;
    DeviceGuard g(h->device);
    if (int rc = wait_solved(h)) return rc;
    const DevState& st = host_state(h);
    const int k = st.solve_status == dmd::ST_E_NOT_READY ? 0 : st.r_eff;
    if (r_eff) *r_eff = k;
    if (bg_index) *bg_index = k > 0 ? st.bg_index : -1;
    const double* b = reinterpret_cast<const double*>(h->res_host + h->L.amp_off);
    for (int i = 0; i < k; ++i) {
        if (b_re) b_re[i] = b[2 * i];
        if (b_im) b_im[i] = b[2 * i + 1];
    }
    return solve_status(h);
}

DMD_API int dmd_stream_background(dmd_stream_t* h, void* fg, void* bg, void* stream) {
    if (int rc = check_handle(h)) return rc;
    if (h->cplx) return fail(DMD_E_UNSUPPORTED, "background subtraction is for dense streams");
    if (!fg && !bg) return fail(DMD_E_INVAL, "fg and bg are both null");
    if (!h->solve_enqueued) return fail(DMD_E_NOT_READY, "no solve has been enqueued");
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    HIP_TRY(begin(h, s));
    dmd::BackgroundArgs a{};
    a.st = reinterpret_cast<const DevState*>(h->res_dev);
    a.ring = h->ring;
    a.ld = h->ld;
    a.n = h->n;
    a.m = h->m;
    a.slots = h->slots;
    a.buildup = h->opts.buildup;
    a.beta = h->Bbg;
    a.fg = fg;
    a.bg = bg;
    a.elem_f64 = h->elem_bytes == 8;
    a.coef_f64 = h->coef_f64;
    HIP_TRY(timed("background", s, [&] { return dmd::launch_background(a, s); }));
    HIP_TRY(end(h, s));
    return DMD_OK;
}

DMD_API int dmd_stream_load_window(dmd_stream_t* h, const void* X, int64_t ldx, int32_t ncols, void* stream) {
    if (int rc = check_handle(h)) return rc;
    if (h->cplx) return fail(DMD_E_UNSUPPORTED, "bulk window load is for dense streams");
    if (!X) return fail(DMD_E_INVAL, "null X");
    if (ncols < 1 || ncols > h->m + 1) return fail(DMD_E_INVAL, "ncols must be in [1, m+1] (got %d)", ncols);
    if (ldx < h->n) return fail(DMD_E_INVAL, "ldx < n");
    if ((uintptr_t)X % h->elem_bytes) return fail(DMD_E_INVAL, "X not %d-byte aligned", h->elem_bytes);
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    HIP_TRY(begin(h, s));
    DevState* st = reinterpret_cast<DevState*>(h->res_dev);
    h->last_block_k = 0;
    h->last_packed = -1;
    h->snap_par = -1;
    HIP_TRY(dmd::launch_copy_columns(X, ldx, h->ring, h->ld, h->n, ncols, h->elem_bytes == 8, s));
    HIP_TRY(timed("gram_full", s, [&] {
        return dmd::launch_gram_full(h->ring, h->ld, h->n, h->m, h->slots, h->elem_bytes == 8, h->opts.precision,
                                     ncols, 0, h->gfull, h->G, st, 1, s);
    }));
    if (h->opts.auto_solve)
        if (int rc = enqueue_solve(h, s)) return rc;
    HIP_TRY(end(h, s));
    return DMD_OK;
}

DMD_API int dmd_stream_resync(dmd_stream_t* h, void* stream) {
    if (int rc = check_handle(h)) return rc;
    if (h->cplx) return fail(DMD_E_UNSUPPORTED, "Gram resync is for dense streams");
    DeviceGuard g(h->device);
    hipStream_t s = as_stream(stream);
    HIP_TRY(begin(h, s));
    DevState* st = reinterpret_cast<DevState*>(h->res_dev);
    h->last_block_k = 0;
    h->last_packed = -1;
    h->snap_par = -1;
    HIP_TRY(timed("gram_full", s, [&] {
        return dmd::launch_gram_full(h->ring, h->ld, h->n, h->m, h->slots, h->elem_bytes == 8, h->opts.precision,
                                     h->m + 1, -1, h->gfull, h->G, st, 2, s);
    }));
    if (h->opts.auto_solve)
        if (int rc = enqueue_solve(h, s)) return rc;
    HIP_TRY(end(h, s));
    return DMD_OK;
}

DMD_API int dmd_stream_info(dmd_stream_t* h, dmd_info_t* info) {
    if (int rc = check_handle(h)) return rc;
    if (!info) return fail(DMD_E_INVAL, "null info");
    DeviceGuard g(h->device);
    DevState st;
    if (int rc = read_state(h, &st)) return rc;
    info->n = h->n;
    info->m = h->m;
    info->r = h->r;
    info->dtype = h->opts.dtype;
    info->precision = h->opts.precision;
    info->count = st.count;
    info->r_eff = st.r_eff;
    info->sweeps = st.sweeps;
    info->qr_iters = st.qr_iters;
    info->device_bytes = h->device_bytes;
    info->gram_iter = h->gram_iter;
    info->proj_form = h->proj_form;
    return DMD_OK;
}

DMD_API int dmd_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return DMD_OK;
}

DMD_API int dmd_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof) {
        (void)hipEventSynchronize(r.b);
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_prof.clear();
    return DMD_OK;
}

DMD_API int dmd_profile_read(const char* kernel, int64_t* launches, double* total_ms) {
    if (!kernel || !launches || !total_ms) return fail(DMD_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    int64_t cnt = 0;
    double tot = 0.0;
    for (auto& r : g_prof) {
        if (std::strcmp(r.name, kernel) != 0) continue;
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        tot += ms;
        ++cnt;
    }
    *launches = cnt;
    *total_ms = tot;
    return DMD_OK;
}

// ------------------------------------------------------------------ batches

namespace {

// Per-tick argument tables: one contiguous block, staged in pinned memory and
// copied to the device before the grouped launches (two copies alternate so
// that the host never overwrites a table a tick in flight still reads).
struct TickLayout {
    size_t gram, gblk, lds, glb, tlds, tglb, clds, cglb, all, proj, pblk, bytes;
    static TickLayout make(int cap) {
        TickLayout L;
        auto al = [](size_t x) { return (x + 255) / 256 * 256; };
        L.gram = 0;
        L.gblk = al(L.gram + sizeof(dmd::GramItem) * cap);
        L.lds = al(L.gblk + sizeof(int) * (cap + 1));
        L.glb = al(L.lds + sizeof(dmd::SolveArgs) * cap);
        L.tlds = al(L.glb + sizeof(dmd::SolveArgs) * cap);
        L.tglb = al(L.tlds + sizeof(dmd::SolveArgs) * cap);
        L.clds = al(L.tglb + sizeof(dmd::SolveArgs) * cap);
        L.cglb = al(L.clds + sizeof(dmd::SolveArgs) * cap);
        L.all = al(L.cglb + sizeof(dmd::SolveArgs) * cap);
        L.proj = al(L.all + sizeof(dmd::SolveArgs) * cap);
        L.pblk = al(L.proj + sizeof(dmd::ProjectArgs) * cap);
        L.bytes = al(L.pblk + sizeof(int) * (cap + 1));
        return L;
    }
};

}  // namespace

// A tick replayed as a HIP graph: its launches depend only on these counts
// and on the descriptor buffer, everything else reaches the kernels through
// the descriptors that the graph's first node copies from pinned memory.
struct TickShape {
    int buf, count, nl, ng, ntl, ntg, gtot, np, ptot;
    bool operator==(const TickShape& o) const {
        return buf == o.buf && count == o.count && nl == o.nl && ng == o.ng && ntl == o.ntl && ntg == o.ntg &&
               gtot == o.gtot && np == o.np && ptot == o.ptot;
    }
};
struct TickGraph {
    TickShape shape;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

struct dmd_batch {
    int device = 0;
    int cap = 0;
    int graphs = 0;                    // > 0: ticks replayed as graphs, at most this many cached
    std::vector<TickGraph> tick_graphs;
    uint64_t uses = 0;
    hipStream_t cap_stream = nullptr;  // capture stream (default priority)
    int64_t budget = 0, used = 0;
    std::vector<dmd_stream*> members;
    TickLayout L{};
    char* host[2] = {nullptr, nullptr};
    char* dev[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    bool used_buf[2] = {false, false};
    int next = 0;
    hipEvent_t ev_last = nullptr;
    hipStream_t last_stream = nullptr;
    bool has_last = false;
};

DMD_API int dmd_batch_opts_init(dmd_batch_opts_t* o) {
    if (!o) return fail(DMD_E_INVAL, "null opts");
    std::memset(o, 0, sizeof(*o));
    o->max_streams = 256;
    return DMD_OK;
}

static void batch_free(dmd_batch* b) {
    for (TickGraph& g : b->tick_graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    b->tick_graphs.clear();
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (int i = 0; i < 2; ++i) {
        if (b->host[i]) (void)hipHostFree(b->host[i]);
        if (b->dev[i]) (void)hipFree(b->dev[i]);
        if (b->done[i]) (void)hipEventDestroy(b->done[i]);
    }
    if (b->ev_last) (void)hipEventDestroy(b->ev_last);
}

DMD_API int dmd_batch_create(const dmd_batch_opts_t* opts, dmd_batch_t** out) {
    if (!out) return fail(DMD_E_INVAL, "null output pointer");
    *out = nullptr;
    dmd_batch_opts_t o;
    dmd_batch_opts_init(&o);
    if (opts) {
        o = *opts;
        if (o.graphs < 0 || o.graphs > 256) return fail(DMD_E_INVAL, "graphs must be in [0, 256]");
        for (int i = 0; i < 8; ++i)
            if (o.reserved[i]) return fail(DMD_E_INVAL, "opts.reserved must be zero");
        if (o.max_streams == 0) o.max_streams = 256;
    }
    if (o.max_streams < 1 || o.max_streams > 1024) return fail(DMD_E_INVAL, "max_streams must be in [1, 1024]");
    if (o.hbm_budget < 0) return fail(DMD_E_INVAL, "hbm_budget must be >= 0");
    dmd_batch* b = new (std::nothrow) dmd_batch();
    if (!b) return fail(DMD_E_NOMEM, "host allocation failed");
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return fail(DMD_E_DEVICE, "no HIP device");
    }
    b->cap = o.max_streams;
    b->graphs = o.graphs;
    b->budget = o.hbm_budget;
    if (b->budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete b;
            return fail(DMD_E_DEVICE, "hipMemGetInfo failed");
        }
        b->budget = (int64_t)(0.9 * (double)fr);
    }
    b->L = TickLayout::make(b->cap);
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipHostMalloc((void**)&b->host[i], b->L.bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void**)&b->dev[i], b->L.bytes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_last, hipEventDisableTiming);
    if (e == hipSuccess && b->graphs > 0) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        batch_free(b);
        delete b;
        return fail(DMD_E_NOMEM, "batch tables: %s", hipGetErrorString(e));
    }
    *out = b;
    return DMD_OK;
}

DMD_API int dmd_batch_destroy(dmd_batch_t* b) {
    if (!b) return DMD_OK;
    DeviceGuard g(b->device);
    if (b->has_last) (void)hipEventSynchronize(b->ev_last);
    batch_free(b);
    delete b;
    return DMD_OK;
}

DMD_API int dmd_batch_attach(dmd_batch_t* b, dmd_stream_t* h) {
    if (!b) return fail(DMD_E_INVAL, "null batch");
    if (int rc = check_handle(h)) return rc;
    if (h->device != b->device) return fail(DMD_E_UNSUPPORTED, "stream and batch are on different devices");
    if (!h->opts.auto_solve) return fail(DMD_E_UNSUPPORTED, "batch members solve every push (auto_solve)");
    if (h->cplx && !h->use_trid)
        return fail(DMD_E_UNSUPPORTED, "sparse batch members use the tridiagonal solver (no warm start)");
    for (dmd_stream* x : b->members)
        if (x == h) return fail(DMD_E_INVAL, "stream already attached");
    if ((int)b->members.size() >= b->cap) return fail(DMD_E_INVAL, "batch is full (%d streams)", b->cap);
    if (b->used + h->device_bytes > b->budget)
        return fail(DMD_E_NOMEM, "admission refused: %lld + %lld bytes exceed the budget of %lld",
                    (long long)b->used, (long long)h->device_bytes, (long long)b->budget);
    b->members.push_back(h);
    b->used += h->device_bytes;
    return DMD_OK;
}

DMD_API int dmd_batch_detach(dmd_batch_t* b, dmd_stream_t* h) {
    if (!b) return fail(DMD_E_INVAL, "null batch");
    if (int rc = check_handle(h)) return rc;
    for (size_t i = 0; i < b->members.size(); ++i)
        if (b->members[i] == h) {
            b->members.erase(b->members.begin() + i);
            b->used -= h->device_bytes;
            return DMD_OK;
        }
    return fail(DMD_E_INVAL, "stream is not attached");
}

DMD_API int dmd_batch_info(dmd_batch_t* b, int32_t* nstreams, int64_t* used_bytes, int64_t* budget) {
    if (!b) return fail(DMD_E_INVAL, "null batch");
    if (nstreams) *nstreams = (int32_t)b->members.size();
    if (used_bytes) *used_bytes = b->used;
    if (budget) *budget = b->budget;
    return DMD_OK;
}

namespace {
// One member's frame of a tick: dense x, or a sparse snapshot (nnz, idx, val).
struct TickFrame {
    const void* x;
    int32_t nnz;
    const int32_t* idx;
    const void* val;
};

// A tick over any mix of members.  Dense FP32 members with FP32 projections
// (class A) take the grouped Gram pass and the grouped projection; FP64
// members (FP64 data or FP64 projections) and sparse members run their own
// Gram (or sparse ingest) and projection kernels inside the tick, on the same
// stream; the small solves of every member are grouped (real tridiagonal or
// Jacobi, Hermitian tridiagonal, eig).  Each member's kernels are the ones its
// own push would run, so its results equal its results alone, bit for bit.
int batch_tick_impl(dmd_batch* b, int count, dmd_stream* const* streams, const TickFrame* frames,
                    void* const* modes, const int64_t* ld_modes, void* stream) {
    if (count < 0 || count > b->cap) return fail(DMD_E_INVAL, "count must be in [0, %d]", b->cap);
    if (count == 0) return DMD_OK;
    if (!streams || !frames) return fail(DMD_E_INVAL, "null streams or frames");
    for (int i = 0; i < count; ++i) {
        dmd_stream* h = streams[i];
        bool member = false;
        for (dmd_stream* x : b->members) member |= (x == h);
        if (!member) return fail(DMD_E_INVAL, "streams[%d] is not attached to the batch", i);
        for (int j = 0; j < i; ++j)
            if (streams[j] == h) return fail(DMD_E_INVAL, "streams[%d] appears twice in one tick", i);
        const TickFrame& f = frames[i];
        if (h->cplx) {
            if (f.nnz < 0 || f.nnz > h->max_nnz)
                return fail(DMD_E_INVAL, "frames[%d]: nnz must be in [0, max_nnz=%d]", i, h->max_nnz);
            if (f.nnz > 0 && (!f.idx || !f.val)) return fail(DMD_E_INVAL, "frames[%d]: null idx or val", i);
            if ((uintptr_t)f.idx % 4 || (uintptr_t)f.val % 8)
                return fail(DMD_E_INVAL, "frames[%d]: idx must be 4-byte and val 8-byte aligned", i);
        } else if (!f.x || (uintptr_t)f.x % h->elem_bytes) {
            return fail(DMD_E_INVAL, "snapshots[%d] null or not %d-byte aligned", i, h->elem_bytes);
        }
        if (modes && modes[i]) {
            if (!ld_modes || ld_modes[i] < h->n) return fail(DMD_E_INVAL, "ld_modes[%d] < n", i);
        }
    }
    DeviceGuard g(b->device);
    hipStream_t s = as_stream(stream);
    const int buf = b->next;
    if (b->used_buf[buf]) HIP_TRY(hipEventSynchronize(b->done[buf]));
    char* H = b->host[buf];
    char* D = b->dev[buf];
    auto* gi = reinterpret_cast<dmd::GramItem*>(H + b->L.gram);
    int* gblk = reinterpret_cast<int*>(H + b->L.gblk);
    auto* sl = reinterpret_cast<dmd::SolveArgs*>(H + b->L.lds);
    auto* sg = reinterpret_cast<dmd::SolveArgs*>(H + b->L.glb);
    auto* tl = reinterpret_cast<dmd::SolveArgs*>(H + b->L.tlds);
    auto* tg = reinterpret_cast<dmd::SolveArgs*>(H + b->L.tglb);
    auto* cl = reinterpret_cast<dmd::SolveArgs*>(H + b->L.clds);
    auto* cg = reinterpret_cast<dmd::SolveArgs*>(H + b->L.cglb);
    auto* sa = reinterpret_cast<dmd::SolveArgs*>(H + b->L.all);
    auto* pa = reinterpret_cast<dmd::ProjectArgs*>(H + b->L.proj);
    int* pblk = reinterpret_cast<int*>(H + b->L.pblk);
    int na = 0, nl = 0, ng = 0, ntl = 0, ntg = 0, ncl = 0, ncg = 0, np = 0, gtot = 0, ptot = 0;
    std::vector<int> own;  // members that run their own Gram and projection kernels
    for (int i = 0; i < count; ++i) {
        dmd_stream* h = streams[i];
        const bool grouped = !h->cplx && h->elem_bytes == 4 && !h->coef_f64;
        if (grouped) {
            dmd::GramItem& it = gi[na];
            it = dmd::GramItem{};
            it.x = frames[i].x;
            it.ring = h->ring;
            it.ld = h->ld;
            it.n = h->n;
            it.m = h->m;
            it.slots = h->slots;
            it.x_aligned = ((uintptr_t)frames[i].x % 16) == 0;
            it.iter = h->gram_iter;
            it.nblk = dmd::gram_blocks(h->n, h->elem_bytes, h->gram_iter);
            it.partials = h->partials;
            it.G = h->G;
            it.st = reinterpret_cast<DevState*>(h->res_dev);
            gblk[na] = gtot;
            gtot += it.nblk;
            ++na;
            if (modes && modes[i]) {
                fill_project_args(h, pa[np], modes[i], ld_modes[i], true);
                pblk[np] = ptot;
                ptot += dmd::project_item_blocks(h->n);
                ++np;
            }
        } else {
            own.push_back(i);
        }
        dmd::SolveArgs a;
        fill_solve_args(h, a);
        sa[i] = a;
        if (h->cplx) {
            if (h->m <= 32) cl[ncl++] = a;
            else cg[ncg++] = a;
        } else {
            const bool small = h->m + (h->m & 1) <= 64;
            if (h->use_trid) {
                if (small) tl[ntl++] = a;
                else tg[ntg++] = a;
            } else {
                if (small) sl[nl++] = a;
                else sg[ng++] = a;
            }
        }
    }
    gblk[na] = gtot;
    pblk[np] = ptot;
    // order after every member's earlier work and the batch's previous tick
    for (int i = 0; i < count; ++i) HIP_TRY(begin(streams[i], s));
    if (b->has_last && b->last_stream != s) HIP_TRY(hipStreamWaitEvent(s, b->ev_last, 0));
    // the Gram pass (or sparse ingest) of a member with kernels of its own
    auto own_gram = [&](hipStream_t q, int i) -> hipError_t {
        dmd_stream* h = streams[i];
        DevState* st = reinterpret_cast<DevState*>(h->res_dev);
        if (h->cplx)
            return dmd::launch_csr_push(frames[i].idx, static_cast<const float2*>(frames[i].val), frames[i].nnz, h->n,
                                        h->ring_idx, h->ring_val, h->ring_nnz, h->max_nnz, h->m, h->scatter, h->flag,
                                        h->G, h->partials, st, q);
        int nblk = 0;
        hipError_t e;
        if (h->elem_bytes == 8)
            e = dmd::launch_gram_columns<double>(static_cast<const double*>(frames[i].x), static_cast<double*>(h->ring),
                                                 h->ld, h->n, h->m, h->slots, h->partials, h->nblk_cap, st,
                                                 h->gram_iter, &nblk, q);
        else
            e = dmd::launch_gram_columns<float>(static_cast<const float*>(frames[i].x), static_cast<float*>(h->ring),
                                                h->ld, h->n, h->m, h->slots, h->partials, h->nblk_cap, st,
                                                h->gram_iter, &nblk, q);
        if (e != hipSuccess) return e;
        return dmd::launch_gram_finalize(h->G, h->partials, nblk, h->m, h->slots, st, q);
    };
    auto own_project = [&](hipStream_t q, int i) -> hipError_t {
        dmd_stream* h = streams[i];
        if (!modes || !modes[i]) return hipSuccess;
        if (h->cplx)
            return dmd::launch_csr_project(reinterpret_cast<const DevState*>(h->res_dev), h->ring_idx, h->ring_val,
                                           h->ring_nnz, h->max_nnz, h->m, 1, static_cast<const float2*>(h->Bphi), h->r,
                                           static_cast<float2*>(modes[i]), ld_modes[i], h->n,
                                           dmd::CsrUnionScratch{h->upos, h->ulist, h->ucount, h->ucount + 1,
                                                                h->ucap, h->ublock},
                                           q);
        dmd::ProjectArgs a;
        fill_project_args(h, a, modes[i], ld_modes[i], true);
        return dmd::launch_project(a, q);
    };
    // the tick's work: descriptors to the device, then one grouped launch per phase
    auto enqueue = [&](hipStream_t q, bool time_phases) -> hipError_t {
        hipError_t e = hipMemcpyAsync(D, H, b->L.bytes, hipMemcpyHostToDevice, q);
        if (e != hipSuccess) return e;
        auto phase = [&](const char* name, auto&& fn) { return time_phases ? timed(name, q, fn) : fn(); };
        auto* dgi = reinterpret_cast<const dmd::GramItem*>(D + b->L.gram);
        auto* dgblk = reinterpret_cast<const int*>(D + b->L.gblk);
        e = phase("batch_gram", [&] {
            hipError_t f = na > 0 ? dmd::launch_gram_grouped(dgi, dgblk, na, gtot, q) : hipSuccess;
            for (size_t u = 0; u < own.size() && f == hipSuccess; ++u) f = own_gram(q, own[u]);
            return f;
        });
        if (e != hipSuccess) return e;
        e = phase("batch_solve", [&] {
            hipError_t f = dmd::launch_jacobi_grouped(reinterpret_cast<const dmd::SolveArgs*>(D + b->L.lds), nl,
                                                      reinterpret_cast<const dmd::SolveArgs*>(D + b->L.glb), ng, q);
            if (f == hipSuccess)
                f = dmd::launch_trid_grouped(reinterpret_cast<const dmd::SolveArgs*>(D + b->L.tlds), ntl,
                                             reinterpret_cast<const dmd::SolveArgs*>(D + b->L.tglb), ntg, q);
            if (f == hipSuccess)
                f = dmd::launch_trid_grouped_cplx(reinterpret_cast<const dmd::SolveArgs*>(D + b->L.clds), ncl,
                                                  reinterpret_cast<const dmd::SolveArgs*>(D + b->L.cglb), ncg, q);
            if (f == hipSuccess)
                f = dmd::launch_eig_grouped(reinterpret_cast<const dmd::SolveArgs*>(D + b->L.all), count, q);
            return f;
        });
        if (e != hipSuccess || !modes) return e;
        return phase("batch_project", [&] {
            hipError_t f = np > 0 ? dmd::launch_project_grouped(reinterpret_cast<const dmd::ProjectArgs*>(D + b->L.proj),
                                                                reinterpret_cast<const int*>(D + b->L.pblk), np, ptot, q)
                                  : hipSuccess;
            for (size_t u = 0; u < own.size() && f == hipSuccess; ++u) f = own_project(q, own[u]);
            return f;
        });
    };
    // graph replays take every per-tick value from the descriptors; members
    // with kernels of their own pass their frames as launch arguments, so
    // such ticks run eagerly
    if (b->graphs > 0 && own.empty()) {
        const TickShape shape{buf, count, nl, ng, ntl, ntg, gtot, np, ptot};
        TickGraph* tg = nullptr;
        for (TickGraph& g : b->tick_graphs)
            if (g.shape == shape) tg = &g;
        if (!tg) {
            if ((int)b->tick_graphs.size() >= b->graphs) {  // evict the least recently used
                size_t lru = 0;
                for (size_t i = 1; i < b->tick_graphs.size(); ++i)
                    if (b->tick_graphs[i].last_use < b->tick_graphs[lru].last_use) lru = i;
                // the evicted graph may still run: destroy it only after the last tick
                if (b->has_last) HIP_TRY(hipEventSynchronize(b->ev_last));
                HIP_TRY(hipGraphExecDestroy(b->tick_graphs[lru].exec));
                HIP_TRY(hipGraphDestroy(b->tick_graphs[lru].graph));
                b->tick_graphs.erase(b->tick_graphs.begin() + (long)lru);
            }
            TickGraph g;
            g.shape = shape;
            HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed));
            const hipError_t ce = enqueue(b->cap_stream, false);
            hipGraph_t graph = nullptr;
            const hipError_t ee = hipStreamEndCapture(b->cap_stream, &graph);
            if (ce != hipSuccess || ee != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return hip_fail(ce != hipSuccess ? ce : ee, "tick capture");
            }
            g.graph = graph;
            const hipError_t ie = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return hip_fail(ie, "hipGraphInstantiate");
            }
            b->tick_graphs.push_back(g);
            tg = &b->tick_graphs.back();
        }
        tg->last_use = ++b->uses;
        HIP_TRY(timed("batch_graph", s, [&] { return hipGraphLaunch(tg->exec, s); }));
    } else {
        HIP_TRY(enqueue(s, true));
    }
    HIP_TRY(hipEventRecord(b->done[buf], s));
    b->used_buf[buf] = true;
    b->next ^= 1;
    for (int i = 0; i < count; ++i) {
        dmd_stream* h = streams[i];
        HIP_TRY(hipEventRecord(h->ev_solved, s));
        h->solve_enqueued = true;
        h->last_block_k = 0;
        h->last_packed = -1;
        h->snap_par = -1;
        HIP_TRY(end(h, s));
    }
    b->last_stream = s;
    b->has_last = true;
    HIP_TRY(hipEventRecord(b->ev_last, s));
    return DMD_OK;
}
}  // namespace

DMD_API int dmd_batch_tick(dmd_batch_t* b, int32_t count, dmd_stream_t* const* streams,
                           const void* const* snapshots, void* const* modes, const int64_t* ld_modes,
                           void* stream) {
    if (!b) return fail(DMD_E_INVAL, "null batch");
    if (count < 0 || count > b->cap) return fail(DMD_E_INVAL, "count must be in [0, %d]", b->cap);
    if (count == 0) return DMD_OK;
    if (!streams || !snapshots) return fail(DMD_E_INVAL, "null streams or snapshots");
    std::vector<TickFrame> f((size_t)count);
    for (int i = 0; i < count; ++i) {
        if (int rc = check_handle(streams[i])) return rc;
        if (streams[i]->cplx) return fail(DMD_E_INVAL, "streams[%d] is sparse: use dmd_batch_tick_frames", i);
        f[i] = TickFrame{snapshots[i], 0, nullptr, nullptr};
    }
    return batch_tick_impl(b, count, streams, f.data(), modes, ld_modes, stream);
}

DMD_API int dmd_batch_tick_frames(dmd_batch_t* b, int32_t count, dmd_stream_t* const* streams,
                                  const dmd_frame_t* frames, void* const* modes, const int64_t* ld_modes,
                                  void* stream) {
    if (!b) return fail(DMD_E_INVAL, "null batch");
    if (count < 0 || count > b->cap) return fail(DMD_E_INVAL, "count must be in [0, %d]", b->cap);
    if (count == 0) return DMD_OK;
    if (!streams || !frames) return fail(DMD_E_INVAL, "null streams or frames");
    std::vector<TickFrame> f((size_t)count);
    for (int i = 0; i < count; ++i) {
        if (int rc = check_handle(streams[i])) return rc;
        f[i] = TickFrame{frames[i].x, frames[i].nnz, frames[i].idx, frames[i].val};
    }
    return batch_tick_impl(b, count, streams, f.data(), modes, ld_modes, stream);
}
