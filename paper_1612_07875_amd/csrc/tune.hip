// Launch-shape tuner: picks, by measurement on the device, the slab form of
// the one-frame Gram pass and the form of the block projection for a stream
// shape (n, m, r, options), keeps the choice in a process-wide table that
// dmd_stream_create consults, and saves / loads the table as a text file.
//
// What is measured is what a caller runs: the Gram pass as back-to-back
// pushes (no solves), and the block projection form as the pipelined block
// step (block push with its solves on one HIP stream, the projection of the
// previous block on another), since a projection form that is faster alone
// can be slower beside the next block's solves.  The data are uniform random
// numbers from a counter-based hash (timing only; no result is kept).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "dmd_internal.h"
#include "dmd_stream.h"

#define DMD_API extern "C" __attribute__((visibility("default")))

namespace dmd {
namespace {

struct Entry {
    TuneKey key;
    TuneVal val;
};
std::mutex g_mu;
std::vector<Entry> g_table;
bool g_env_loaded = false;

int load_file_locked(const char* path, bool strict);

void load_env_locked() {
    if (g_env_loaded) return;
    g_env_loaded = true;
    if (const char* p = getenv("DMD_TUNE_CACHE"))
        if (*p) (void)load_file_locked(p, false);
}

void store_locked(const TuneKey& k, const TuneVal& v) {
    for (Entry& e : g_table)
        if (e.key == k) {
            e.val = v;
            return;
        }
    g_table.push_back(Entry{k, v});
}

int load_file_locked(const char* path, bool strict) {
    FILE* f = fopen(path, "r");
    if (!f) return strict ? api_fail(DMD_E_INVAL, "cannot open tuning file %s", path) : DMD_OK;
    char line[512];
    int lineno = 0;
    std::vector<Entry> got;
    while (fgets(line, sizeof(line), f)) {
        ++lineno;
        if (line[0] == '#' || line[0] == '\n') continue;
        Entry e{};
        const int nf = sscanf(line, "%d %d %d %d %d %d %d %d %lf %lf", &e.key.dtype, &e.key.precision,
                              &e.key.nbucket, &e.key.m, &e.key.r, &e.key.kmax, &e.val.gram_iter, &e.val.proj_form,
                              &e.val.gram_us, &e.val.step_us);
        const bool ok = nf == 10 && (e.val.gram_iter == 0 || e.val.gram_iter == 1 || e.val.gram_iter == 2 ||
                                     e.val.gram_iter == 4) &&
                        e.val.proj_form >= 0 && e.val.proj_form <= 3;
        if (!ok) {
            fclose(f);
            return strict ? api_fail(DMD_E_INVAL, "%s:%d: not a tuning entry", path, lineno) : DMD_OK;
        }
        got.push_back(e);
    }
    fclose(f);
    for (const Entry& e : got) store_locked(e.key, e.val);
    return DMD_OK;
}

// Uniform [0, 1) values from a counter-based hash of the element index.
template <typename T>
__global__ void k_fill_uniform(T* __restrict__ x, int64_t count, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        x[i] = (T)((double)(z >> 11) * 0x1.0p-53);
    }
}

hipError_t fill_uniform(void* x, int64_t count, int elem_bytes, uint64_t seed, hipStream_t s) {
    const dim3 grid(1024), block(256);
    if (elem_bytes == 8) hipLaunchKernelGGL(k_fill_uniform<double>, grid, block, 0, s, static_cast<double*>(x), count, seed);
    else hipLaunchKernelGGL(k_fill_uniform<float>, grid, block, 0, s, static_cast<float*>(x), count, seed);
    return hipGetLastError();
}

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Average time of `reps` calls of f() on s, after `warm` untimed ones.
template <typename F>
int time_calls(hipStream_t s, int warm, int reps, F&& f, double* us) {
    for (int i = 0; i < warm; ++i)
        if (int rc = f()) return rc;
    Events ev;
    if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess)
        return api_fail(DMD_E_DEVICE, "hipEventCreate");
    if (hipEventRecord(ev.a, s) != hipSuccess) return api_fail(DMD_E_DEVICE, "hipEventRecord");
    for (int i = 0; i < reps; ++i)
        if (int rc = f()) return rc;
    if (hipEventRecord(ev.b, s) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess)
        return api_fail(DMD_E_DEVICE, "hipEventRecord/Synchronize");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess) return api_fail(DMD_E_DEVICE, "hipEventElapsedTime");
    *us = 1000.0 * ms / reps;
    return DMD_OK;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};
struct StreamHandle {
    dmd_stream_t* h = nullptr;
    ~StreamHandle() {
        if (h) (void)dmd_stream_destroy(h);
    }
};

// Gram slab form: back-to-back pushes of one random snapshot (solves off).
int tune_gram(int64_t n, int32_t m, int32_t r, const dmd_opts_t& o, hipStream_t s, int* best_iter, double* best_us) {
    dmd_opts_t g = o;
    g.auto_solve = 0;
    g.max_block = 1;
    g.buildup = 0;
    StreamHandle sh;
    if (int rc = dmd_stream_create(n, m, r, &g, &sh.h)) return rc;
    const int eb = o.dtype == DMD_F64 ? 8 : 4;
    DevBuf x;
    if (hipMalloc(&x.p, (size_t)n * eb) != hipSuccess) return api_fail(DMD_E_NOMEM, "tuning buffer");
    if (fill_uniform(x.p, n, eb, 0x5eed, s) != hipSuccess) return api_fail(DMD_E_DEVICE, "fill");
    for (int t = 0; t <= m; ++t)
        if (int rc = dmd_stream_push(sh.h, x.p, s)) return rc;
    int cur = 0, form = 0;
    stream_get_shapes(sh.h, &cur, &form);
    const int rule = gram_iter_rule(n, eb);
    const int cands[3] = {1, 2, 4};
    double times[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
        stream_set_shapes(sh.h, cands[c], form);
        if (int rc = time_calls(s, 3, 12, [&] { return dmd_stream_push(sh.h, x.p, s); }, &times[c])) return rc;
    }
    // the rule's form unless another is more than 2 % faster
    int bi = rule == 4 ? 2 : rule == 2 ? 1 : 0;
    for (int c = 0; c < 3; ++c)
        if (times[c] < 0.98 * times[bi]) bi = c;
    *best_iter = cands[bi];
    *best_us = times[bi];
    return dmd_stream_sync(sh.h);
}

// Block projection form: the pipelined step (block push + solves on s, the
// projection of the same block on a second stream, overlapping the next push).
int tune_block_form(int64_t n, int32_t m, int32_t r, const dmd_opts_t& o, int gram_iter, hipStream_t s,
                    int* best_form, double* best_us) {
    StreamHandle sh;
    dmd_opts_t b = o;
    b.auto_solve = 1;
    if (int rc = dmd_stream_create(n, m, r, &b, &sh.h)) return rc;
    const int kb = o.max_block;
    const int64_t ld = (n + 63) / 64 * 64;
    DevBuf X, phi;
    if (hipMalloc(&X.p, (size_t)ld * kb * 4) != hipSuccess) return api_fail(DMD_E_NOMEM, "tuning buffer");
    const int64_t ldw = ld * r;  // complex64 elements per window's modes
    if (hipMalloc(&phi.p, (size_t)ldw * kb * 8) != hipSuccess) return api_fail(DMD_E_NOMEM, "tuning mode buffer");
    if (fill_uniform(X.p, ld * kb, 4, 0x5eed + 1, s) != hipSuccess) return api_fail(DMD_E_DEVICE, "fill");
    hipStream_t s2 = nullptr;
    if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess) return api_fail(DMD_E_DEVICE, "stream");
    struct S2 {
        hipStream_t s;
        ~S2() { (void)hipStreamDestroy(s); }
    } s2g{s2};
    for (int t = 0; t < m + 1; t += kb)
        if (int rc = dmd_stream_push_block(sh.h, X.p, ld, kb, s)) return rc;
    // one product per window, window pairs (where 2r = 8 mod 16 allows them)
    // and the banded product (where its stage fits)
    int forms[3], nf = 0;
    forms[nf++] = 1;
    if (pairs_apply(m, r, kb)) forms[nf++] = 2;
    if (band_applies(m, r, kb)) forms[nf++] = 3;
    double times[3] = {0, 0, 0};
    Events ev;
    hipEvent_t join = nullptr;
    if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess ||
        hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess)
        return api_fail(DMD_E_DEVICE, "hipEventCreate");
    struct J {
        hipEvent_t e;
        ~J() { (void)hipEventDestroy(e); }
    } jg{join};
    constexpr int kWarm = 2, kReps = 4;
    for (int c = 0; c < nf; ++c) {
        stream_set_shapes(sh.h, gram_iter, forms[c]);
        auto step = [&]() -> int {
            if (int rc = dmd_stream_push_block(sh.h, X.p, ld, kb, s)) return rc;
            return dmd_stream_block_modes(sh.h, phi.p, ld, ldw, s2);
        };
        for (int i = 0; i < kWarm; ++i)
            if (int rc = step()) return rc;
        if (hipDeviceSynchronize() != hipSuccess || hipEventRecord(ev.a, s) != hipSuccess)
            return api_fail(DMD_E_DEVICE, "sync");
        for (int i = 0; i < kReps; ++i)
            if (int rc = step()) return rc;
        // the last projection joins the timing stream
        if (hipEventRecord(join, s2) != hipSuccess || hipStreamWaitEvent(s, join, 0) != hipSuccess ||
            hipEventRecord(ev.b, s) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess)
            return api_fail(DMD_E_DEVICE, "join");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess) return api_fail(DMD_E_DEVICE, "hipEventElapsedTime");
        times[c] = 1000.0 * ms / kReps;
    }
    // the built-in rule's form unless another is more than 2 % faster
    const int rule = block_rule_form(m, r, kb);
    int bi = 0;
    for (int c = 0; c < nf; ++c)
        if (forms[c] == rule) bi = c;
    for (int c = 0; c < nf; ++c)
        if (times[c] < 0.98 * times[bi]) bi = c;
    *best_form = forms[bi];
    *best_us = times[bi];
    if (hipStreamSynchronize(s2) != hipSuccess) return api_fail(DMD_E_DEVICE, "sync");
    return dmd_stream_sync(sh.h);
}

}  // namespace

TuneKey tune_key(int64_t n, int m, int r, const dmd_opts_t& o) {
    TuneKey k{};
    k.dtype = o.dtype;
    k.precision = o.precision;
    k.nbucket = (int)std::lround(8.0 * std::log2((double)(n > 0 ? n : 1)));
    k.m = m;
    k.r = r;
    k.kmax = o.max_block < 1 ? 1 : o.max_block;
    return k;
}

bool tune_lookup(const TuneKey& k, TuneVal* v) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    for (const Entry& e : g_table)
        if (e.key == k) {
            *v = e.val;
            return true;
        }
    return false;
}

}  // namespace dmd

namespace {
int resolve_opts(const dmd_opts_t* opts, dmd_opts_t* o) {
    if (int rc = dmd_opts_init(o)) return rc;
    if (opts) *o = *opts;
    if (o->max_block == 0) o->max_block = 1;
    return DMD_OK;
}
void to_public(const dmd::TuneVal& v, dmd_tuning_t* out) {
    std::memset(out, 0, sizeof(*out));
    out->gram_iter = v.gram_iter;
    out->proj_form = v.proj_form;
    out->gram_us = v.gram_us;
    out->step_us = v.step_us;
}
}  // namespace

DMD_API int dmd_tune(int64_t n, int32_t m, int32_t r, const dmd_opts_t* opts, dmd_tuning_t* out, void* stream) {
    if (!out) return dmd::api_fail(DMD_E_INVAL, "null output");
    dmd_opts_t o;
    if (int rc = resolve_opts(opts, &o)) return rc;
    int64_t bytes = 0;
    if (int rc = dmd_stream_footprint(n, m, r, &o, &bytes)) return rc;  // the checks of dmd_stream_create
    if (o.dtype == DMD_C64_CSR) return dmd::api_fail(DMD_E_UNSUPPORTED, "tuning is for dense streams");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    dmd::TuneVal v{};
    if (int rc = dmd::tune_gram(n, m, r, o, s, &v.gram_iter, &v.gram_us)) return rc;
    // the block projection form, where there is a choice: FP32 block streams
    // (FP32 data, FP32 products) with more than one form that applies
    const bool fp32_block = o.max_block > 1 && o.dtype == DMD_F32 && o.precision != DMD_PREC_BF16X3 &&
                            o.precision != DMD_PREC_FP64 && dmd::project_block_fits(m, o.max_block, r);
    if (fp32_block && (dmd::pairs_apply(m, r, o.max_block) || dmd::band_applies(m, r, o.max_block))) {
        if (int rc = dmd::tune_block_form(n, m, r, o, v.gram_iter, s, &v.proj_form, &v.step_us)) return rc;
    }
    {
        std::lock_guard<std::mutex> lk(dmd::g_mu);
        dmd::load_env_locked();
        dmd::store_locked(dmd::tune_key(n, m, r, o), v);
    }
    to_public(v, out);
    return DMD_OK;
}

DMD_API int dmd_tune_lookup(int64_t n, int32_t m, int32_t r, const dmd_opts_t* opts, dmd_tuning_t* out) {
    if (!out) return dmd::api_fail(DMD_E_INVAL, "null output");
    dmd_opts_t o;
    if (int rc = resolve_opts(opts, &o)) return rc;
    dmd::TuneVal v{};
    if (!dmd::tune_lookup(dmd::tune_key(n, m, r, o), &v)) {
        std::memset(out, 0, sizeof(*out));
        return dmd::api_fail(DMD_E_NOT_READY, "no tuning entry for this shape");
    }
    to_public(v, out);
    return DMD_OK;
}

DMD_API int dmd_tune_save(const char* path) {
    if (!path) return dmd::api_fail(DMD_E_INVAL, "null path");
    std::lock_guard<std::mutex> lk(dmd::g_mu);
    dmd::load_env_locked();
    FILE* f = fopen(path, "w");
    if (!f) return dmd::api_fail(DMD_E_INVAL, "cannot write %s", path);
    fprintf(f, "# dmdstream tuning table: dtype precision nbucket(8 log2 n) m r max_block gram_iter proj_form "
               "gram_us step_us\n");
    for (const dmd::Entry& e : dmd::g_table)
        fprintf(f, "%d %d %d %d %d %d %d %d %.3f %.3f\n", e.key.dtype, e.key.precision, e.key.nbucket, e.key.m,
                e.key.r, e.key.kmax, e.val.gram_iter, e.val.proj_form, e.val.gram_us, e.val.step_us);
    const bool ok = fclose(f) == 0;
    return ok ? DMD_OK : dmd::api_fail(DMD_E_INVAL, "write error on %s", path);
}

DMD_API int dmd_tune_load(const char* path) {
    if (!path) return dmd::api_fail(DMD_E_INVAL, "null path");
    std::lock_guard<std::mutex> lk(dmd::g_mu);
    dmd::load_env_locked();
    return dmd::load_file_locked(path, true);
}

DMD_API int dmd_tune_clear(void) {
    std::lock_guard<std::mutex> lk(dmd::g_mu);
    dmd::g_env_loaded = true;  // a cleared table stays empty until loaded or tuned again
    dmd::g_table.clear();
    return DMD_OK;
}
