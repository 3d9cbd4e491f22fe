// C ABI of the clustering library: argument checks, workspace handling,
// stream selection, diagnostics and kernel timing.  The computation itself
// is enqueued by fec::launch_pipeline (fec_device.hip).

#include "../../include/fec.h"
#include "fec_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int32_t fail(int32_t code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int32_t ok() {
    g_err.clear();
    return FEC_OK;
}

// Host-side argument checks shared by both forms.
int32_t check_args(const float *xyz, int64_t n, float d, int32_t min_size, int32_t max_size,
                   const int32_t *labels_out) {
    if (n < 0 || n > 2147483647LL)
        return fail(FEC_EINVAL, "n=%lld outside [0, 2^31-1]", (long long)n);
    if (!std::isfinite(d) || !(d > 0.0f))
        return fail(FEC_EINVAL, "d=%g must be finite and > 0", (double)d);
    const float d2 = d * d;
    if (!std::isnormal(d2))
        return fail(FEC_EINVAL, "d*d=%g is not a normal binary32 number", (double)d2);
    if (min_size > max_size)
        return fail(FEC_EINVAL, "min_size=%d > max_size=%d", min_size, max_size);
    if (n > 0 && (xyz == nullptr || labels_out == nullptr))
        return fail(FEC_EINVAL, "null xyz or labels_out with n=%lld", (long long)n);
    return FEC_OK;
}

// ----------------------------------------------------------------- timing
struct EventTimer final : fec::Timer {
    uint64_t mask = 0;
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[fec::kNumStages] = {};
    int64_t count[fec::kNumStages] = {};
    hipEvent_t open_ev = nullptr;

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void begin(int stage, hipStream_t s) override {
        if (!((mask >> stage) & 1)) return;
        open_ev = get();
        if (open_ev) (void)hipEventRecord(open_ev, s);
    }
    void end(int stage, hipStream_t s) override {
        if (!((mask >> stage) & 1) || !open_ev) return;
        hipEvent_t b = get();
        if (!b) return;
        (void)hipEventRecord(b, s);
        pending.push_back({stage, open_ev, b});
        open_ev = nullptr;
    }
    int collect() {
        for (auto &r : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(r.b) == hipSuccess &&
                hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                total_ms[r.stage] += ms;
                count[r.stage] += 1;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
        return fec::kNumStages;
    }
};

std::mutex g_mu;
EventTimer g_timer;

// ----------------------------------------------------------------- no-allocation form
// The workspace of fec_cluster_noalloc: a static device array, one copy per
// GPU.  In host code its name only stands for the symbol; its device address
// on the current GPU comes from hipGetSymbolAddress, taken once per device
// and kept.
constexpr size_t kScratchBytes = FEC_NOALLOC_SCRATCH_BYTES;
static_assert(fec::make_layout(FEC_NOALLOC_MAX_POINTS, 1, fec::kColGridPerPointNoAlloc).total <=
                  kScratchBytes,
              "the scratch array holds the workspace of the largest call it admits");
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the scratch array on the current GPU.
int32_t scratch_address(void **out) {
    int dev = -1;
    const hipError_t e0 = hipGetDevice(&dev);
    if (e0 != hipSuccess) return fail(FEC_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e0));
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(FEC_EDEVICE, "device %d beyond the %d the library tracks", dev,
                    kMaxScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(FEC_EDEVICE, "hipGetSymbolAddress of the scratch array failed: %s",
                        hipGetErrorString(e));
        if ((reinterpret_cast<uintptr_t>(p) & 255u) != 0)
            return fail(FEC_EDEVICE, "scratch array is not 256-byte aligned");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FEC_OK;
}

// ----------------------------------------------------------------- blocking form state
struct Cached {
    void *ws = nullptr;
    size_t bytes = 0;
    int32_t *k_dev = nullptr;
    hipStream_t stream = nullptr;
} g_cache;

}  // namespace

extern "C" {

const char *fec_version(void) { return "fec-mi355x 0.1 (gfx950)"; }

const char *fec_last_error(void) { return g_err.c_str(); }

size_t fec_workspace_bytes(int64_t n) {
    if (n <= 0) return 0;
    return fec::make_layout(n).total;
}

int32_t fec_cluster_async(const float *xyz, int64_t n, float d, int32_t min_size,
                          int32_t max_size, int32_t *labels_out, int32_t *k_out, void *workspace,
                          size_t workspace_bytes, void *stream) {
    int32_t rc = check_args(xyz, n, d, min_size, max_size, labels_out);
    if (rc != FEC_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n == 0) {  // k = 0, written on the stream (no host synchronisation)
        if (k_out) {
            const hipError_t e = fec::launch_set_count(k_out, 0, st);
            if (e != hipSuccess)
                return fail(FEC_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
        }
        return ok();
    }
    const fec::Layout L = fec::make_layout(n);
    if (workspace == nullptr || workspace_bytes < L.total)
        return fail(FEC_EINVAL, "workspace of %zu bytes is smaller than the %zu needed",
                    workspace_bytes, L.total);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
        return fail(FEC_EINVAL, "workspace is not 256-byte aligned");
    fec::CallArgs a{};
    a.xyz = xyz;
    a.n = n;
    a.nframes = 1;
    a.d = d;
    a.min_size = min_size;
    a.max_size = max_size;
    a.labels_out = labels_out;
    a.k_out = k_out;
    hipError_t e;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        e = fec::launch_pipeline(a, workspace, L, st, g_timer.mask ? &g_timer : nullptr);
    }
    if (e != hipSuccess) return fail(FEC_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return ok();
}

int32_t fec_cluster_noalloc(const float *xyz, int64_t n, float d, int32_t min_size,
                            int32_t max_size, int32_t *labels_out, int32_t *k_out,
                            void *stream) {
    int32_t rc = check_args(xyz, n, d, min_size, max_size, labels_out);
    if (rc != FEC_OK) return rc;
    if (n > FEC_NOALLOC_MAX_POINTS)
        return fail(FEC_EINVAL, "n=%lld exceeds the no-allocation form's %d points",
                    (long long)n, FEC_NOALLOC_MAX_POINTS);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n == 0) {
        if (k_out) {
            const hipError_t e = fec::launch_set_count(k_out, 0, st);
            if (e != hipSuccess)
                return fail(FEC_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
        }
        return ok();
    }
    void *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != FEC_OK) return rc;
    const fec::Layout L = fec::make_layout(n, 1, fec::kColGridPerPointNoAlloc);
    fec::CallArgs a{};
    a.xyz = xyz;
    a.n = n;
    a.nframes = 1;
    a.d = d;
    a.min_size = min_size;
    a.max_size = max_size;
    a.labels_out = labels_out;
    a.k_out = k_out;
    hipError_t e;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        e = fec::launch_pipeline(a, ws, L, st, g_timer.mask ? &g_timer : nullptr);
    }
    if (e != hipSuccess) return fail(FEC_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return ok();
}

size_t fec_batch_workspace_bytes(int64_t n_total, int32_t nframes) {
    if (n_total < 0 || nframes < 1 || nframes > fec::kMaxFrames) return 0;
    return fec::make_layout(n_total, nframes).total;
}

int32_t fec_cluster_batch_async(const float *xyz, int64_t n_total, int32_t nframes,
                                const int64_t *offsets, const float *d, const int32_t *min_size,
                                const int32_t *max_size, int32_t *labels_out, int32_t *k_out,
                                void *workspace, size_t workspace_bytes, void *stream) {
    if (n_total < 0 || n_total > 2147483647LL)
        return fail(FEC_EINVAL, "n_total=%lld outside [0, 2^31-1]", (long long)n_total);
    if (nframes < 1 || nframes > fec::kMaxFrames)
        return fail(FEC_EINVAL, "nframes=%d outside [1, %d]", nframes, fec::kMaxFrames);
    if (!offsets || !d || !min_size || !max_size || !k_out)
        return fail(FEC_EINVAL, "null offsets, d, min_size, max_size or k_out");
    if (n_total > 0 && (xyz == nullptr || labels_out == nullptr))
        return fail(FEC_EINVAL, "null xyz or labels_out with n_total=%lld", (long long)n_total);
    const fec::Layout L = fec::make_layout(n_total, nframes);
    if (workspace == nullptr || workspace_bytes < L.total)
        return fail(FEC_EINVAL, "workspace of %zu bytes is smaller than the %zu needed",
                    workspace_bytes, L.total);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
        return fail(FEC_EINVAL, "workspace is not 256-byte aligned");
    fec::CallArgs a{};
    a.xyz = xyz;
    a.n = n_total;
    a.nframes = nframes;
    a.offsets = offsets;
    a.d_arr = d;
    a.min_arr = min_size;
    a.max_arr = max_size;
    a.labels_out = labels_out;
    a.k_out = k_out;
    hipError_t e;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        e = fec::launch_pipeline(a, workspace, L, static_cast<hipStream_t>(stream),
                                 g_timer.mask ? &g_timer : nullptr);
    }
    if (e != hipSuccess) return fail(FEC_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return ok();
}

int32_t fec_set_stream(void *stream) {
    g_cache.stream = static_cast<hipStream_t>(stream);
    return ok();
}

void fec_release(void) {
    if (g_cache.ws) (void)hipFree(g_cache.ws);
    if (g_cache.k_dev) (void)hipFree(g_cache.k_dev);
    g_cache.ws = nullptr;
    g_cache.k_dev = nullptr;
    g_cache.bytes = 0;
}

int32_t fec_cluster(const float *xyz, int64_t n, float d, int32_t min_size, int32_t max_size,
                    int32_t *labels_out) {
    int32_t rc = check_args(xyz, n, d, min_size, max_size, labels_out);
    if (rc != FEC_OK) return rc;
    if (n == 0) return ok();
    const size_t need = fec_workspace_bytes(n);
    if (g_cache.bytes < need) {
        if (g_cache.ws) (void)hipFree(g_cache.ws);
        g_cache.ws = nullptr;
        g_cache.bytes = 0;
        if (hipMalloc(&g_cache.ws, need) != hipSuccess) {
            g_cache.ws = nullptr;
            return fail(FEC_ENOMEM, "hipMalloc of %zu workspace bytes failed", need);
        }
        g_cache.bytes = need;
    }
    if (!g_cache.k_dev && hipMalloc(&g_cache.k_dev, sizeof(int32_t)) != hipSuccess) {
        g_cache.k_dev = nullptr;
        return fail(FEC_ENOMEM, "hipMalloc of the result word failed");
    }
    rc = fec_cluster_async(xyz, n, d, min_size, max_size, labels_out, g_cache.k_dev, g_cache.ws,
                           g_cache.bytes, g_cache.stream);
    if (rc != FEC_OK) return rc;
    int32_t k = 0;
    if (hipMemcpyAsync(&k, g_cache.k_dev, sizeof k, hipMemcpyDeviceToHost, g_cache.stream) !=
            hipSuccess ||
        hipStreamSynchronize(g_cache.stream) != hipSuccess)
        return fail(FEC_EDEVICE, "reading the result failed: %s",
                    hipGetErrorString(hipGetLastError()));
    if (k == FEC_ERANGE) return fail(FEC_ERANGE, "grid key of the cloud's extent exceeds 64 bits");
    if (k < 0) return fail(k, "device-side failure (status %d)", k);
    return k;
}

int32_t fec_workspace_stats(const void *workspace, void *stream, int64_t *out, int32_t max_out) {
    if (!workspace || !out || max_out <= 0) return fail(FEC_EINVAL, "bad arguments");
    fec::Params P;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(&P, workspace, sizeof P, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(FEC_EDEVICE, "reading the workspace failed");
    const int64_t v[23] = {P.n,  P.nvalid, P.M,  P.Mcol,     P.key_bits, P.npasses, P.NX,
                           P.NY, P.NZ,     P.max_cell, P.status, P.nwork,   P.giant,
                           (int64_t)P.counters[0], (int64_t)P.counters[1],
                           (int64_t)P.counters[2], (int64_t)P.counters[3],
                           (int64_t)P.counters[4], (int64_t)P.counters[5],
                           (int64_t)P.counters[6], (int64_t)P.counters[7],
                           P.dense_cols ? 1 : (P.hashed_cols ? 2 : 0), P.nwork0};
    const int32_t c = max_out < 23 ? max_out : 23;
    for (int32_t i = 0; i < c; ++i) out[i] = v[i];
    ok();
    return c;
}

int32_t fec_profile_enable(uint64_t stage_mask) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_timer.mask = stage_mask;
    return ok();
}

int32_t fec_profile_read(double *ms_total, int64_t *launches, int32_t max_stages) {
    std::lock_guard<std::mutex> lock(g_mu);
    const int ns = g_timer.collect();
    for (int i = 0; i < ns && i < max_stages; ++i) {
        if (ms_total) ms_total[i] = g_timer.total_ms[i];
        if (launches) launches[i] = g_timer.count[i];
    }
    return ns;
}

void fec_profile_reset(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_timer.collect();
    for (int i = 0; i < fec::kNumStages; ++i) {
        g_timer.total_ms[i] = 0.0;
        g_timer.count[i] = 0;
    }
}

int32_t fec_tuning_set(int32_t cell_blocks, int32_t stream_blocks, int32_t radix_bits,
                       int32_t hook_block, int32_t near_sampling) {
    if (cell_blocks < 0 || stream_blocks < 0 || cell_blocks > (1 << 20) ||
        stream_blocks > (1 << 20))
        return fail(FEC_EINVAL, "block counts outside [0, 2^20]");
    if (radix_bits != 0 && (radix_bits < fec::kMinRadixBits || radix_bits > fec::kMaxRadixBits))
        return fail(FEC_EINVAL, "radix_bits=%d not in {0, 8, 9, 10, 11}", radix_bits);
    if (hook_block != 0 && hook_block != 64 && hook_block != 128 && hook_block != 256)
        return fail(FEC_EINVAL, "hook_block=%d not in {0, 64, 128, 256}", hook_block);
    if (near_sampling < 0 || near_sampling > 2)
        return fail(FEC_EINVAL, "near_sampling=%d not in {0, 1, 2}", near_sampling);
    fec::set_tuning({cell_blocks ? cell_blocks : fec::kDefaultCellBlocks,
                     stream_blocks ? stream_blocks : fec::kDefaultStreamBlocks,
                     radix_bits ? radix_bits : fec::kDefaultRadixBits,
                     hook_block ? hook_block : fec::kDefaultHookBlock, near_sampling});
    return ok();
}

int32_t fec_tuning_get(int32_t *cell_blocks, int32_t *stream_blocks, int32_t *radix_bits,
                       int32_t *hook_block, int32_t *near_sampling) {
    const fec::Tuning t = fec::tuning();
    if (cell_blocks) *cell_blocks = t.cell_blocks;
    if (stream_blocks) *stream_blocks = t.stream_blocks;
    if (radix_bits) *radix_bits = t.radix_bits;
    if (hook_block) *hook_block = t.hook_block;
    if (near_sampling) *near_sampling = t.near_sampling;
    return ok();
}

int32_t fec_stage_count(void) { return fec::kNumStages; }

const char *fec_stage_name(int32_t stage) { return fec::stage_name(stage); }

}  // extern "C"
