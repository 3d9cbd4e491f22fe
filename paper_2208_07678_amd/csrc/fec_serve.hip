// Serving engine: continuous batching of independent clustering requests.
//
// Requests (one point cloud each, with its own d and size bounds) are queued
// in arrival order.  The engine owns `nslots` batch slots; each slot has its
// own stream, batched-form workspace and point / label buffers, sized from
// an HBM budget (the admission limit: a batch takes requests from the head
// of the queue while their points fit the slot).  Whenever a slot is free
// and requests wait, they are launched at once as one batched call (no
// waiting for a batch to fill), so batches of different sizes run on the
// device side by side and a request arriving while others are on the GPU
// joins the next free slot.  Every request's result is the batched form's,
// which is, frame by frame, the single-cloud result.
//
// Per batch: one small host-to-device copy of the batch table (frame
// offsets, d, bounds, caller pointers), a gather kernel that packs the
// requests' points into the slot, the batched pipeline, a scatter kernel
// that writes each request's labels to the caller's buffer, and a copy of
// the kept counts back to pinned host memory, followed by an event.  A batch
// of one request runs the single-cloud pipeline on the caller's buffers.

#include "../../include/fec.h"
#include "fec_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

constexpr int32_t kMaxSlotFrames = 1024;

struct Req {
    int64_t ticket;
    const float *xyz;
    int64_t n;
    float d;
    int32_t min_size, max_size;
    int32_t *labels;
    Clock::time_point t_submit;
    bool alone;  // runs as a batch of its own (its batch was refused as a whole)
};

// Batch table, laid out in one buffer (host pinned copy -> device):
// offsets[F + 1] int64, src[F] pointers, dst[F] pointers, d[F] float,
// min[F] int32, max[F] int32.
struct TableView {
    int64_t *offsets;
    const float **src;
    int32_t **dst;
    float *d;
    int32_t *mn, *mx;
};

size_t table_bytes(int32_t F) {
    return (size_t)(F + 1) * 8 + (size_t)F * (8 + 8 + 4 + 4 + 4) + 64;
}

TableView table_view(void *base, int32_t F) {
    char *p = static_cast<char *>(base);
    TableView t;
    t.offsets = reinterpret_cast<int64_t *>(p);
    p += (size_t)(F + 1) * 8;
    t.src = reinterpret_cast<const float **>(p);
    p += (size_t)F * 8;
    t.dst = reinterpret_cast<int32_t **>(p);
    p += (size_t)F * 8;
    t.d = reinterpret_cast<float *>(p);
    p += (size_t)F * 4;
    t.mn = reinterpret_cast<int32_t *>(p);
    p += (size_t)F * 4;
    t.mx = reinterpret_cast<int32_t *>(p);
    return t;
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    float *xyz = nullptr;
    int32_t *labels = nullptr;
    int32_t *k_dev = nullptr;
    void *table_dev = nullptr;
    void *table_host = nullptr;  // pinned
    int32_t *k_host = nullptr;   // pinned
    std::vector<Req> reqs;       // the batch in flight
    bool busy = false;
};

// ------------------------------------------------------------ kernels
constexpr int kServeBlock = 256;

// Frame holding batch element i (offsets in LDS): last f with off[f] <= i.
__device__ __forceinline__ int serve_frame(const int64_t *off, int F, int64_t i) {
    int lo = 0, hi = F - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Packs the requests' points one after the other (float by float).
__global__ __launch_bounds__(kServeBlock) void k_serve_gather(const int64_t *__restrict__ offsets,
                                                              const float *const *__restrict__ src,
                                                              int F, float *__restrict__ dst) {
    __shared__ int64_t s_off[kMaxSlotFrames + 1];
    for (int f = threadIdx.x; f <= F; f += kServeBlock) s_off[f] = offsets[f];
    __syncthreads();
    const int64_t nf = 3 * s_off[F];
    for (int64_t j = (int64_t)blockIdx.x * kServeBlock + threadIdx.x; j < nf;
         j += (int64_t)gridDim.x * kServeBlock) {
        const int64_t i = j / 3;
        const int f = serve_frame(s_off, F, i);
        dst[j] = src[f][j - 3 * s_off[f]];
    }
}

// Writes each request's (frame-local) labels to its caller's buffer.
__global__ __launch_bounds__(kServeBlock) void k_serve_scatter(const int64_t *__restrict__ offsets,
                                                               int32_t *const *__restrict__ dst,
                                                               int F,
                                                               const int32_t *__restrict__ labels) {
    __shared__ int64_t s_off[kMaxSlotFrames + 1];
    for (int f = threadIdx.x; f <= F; f += kServeBlock) s_off[f] = offsets[f];
    __syncthreads();
    const int64_t n = s_off[F];
    for (int64_t i = (int64_t)blockIdx.x * kServeBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kServeBlock) {
        const int f = serve_frame(s_off, F, i);
        dst[f][i - s_off[f]] = labels[i];
    }
}

}  // namespace

struct fec_server {
    int device = 0;
    int32_t slot_frames = 0;
    int64_t slot_points = 0;
    size_t slot_bytes = 0;
    std::vector<Slot> slots;
    std::deque<Req> queue;
    struct Done {
        int64_t ticket;
        int32_t k;
        double latency_ms;
    };
    std::deque<Done> done;
    int64_t next_ticket = 0;
    int64_t n_submitted = 0, n_completed = 0, n_batches = 0;
    int64_t max_batch_frames = 0, max_in_flight = 0;
    int64_t n_requeued = 0;
    int32_t error = FEC_OK;
};

namespace {

// HBM bytes of one slot: batched-form workspace (with room for the partial
// boxes of any smaller batch), points, labels, kept counts, batch table.
size_t slot_bytes_for(int64_t P, int32_t F) {
    const size_t ws = fec_batch_workspace_bytes(P, F) + (size_t)(fec::kBboxBlocks + F) * 32 + 4096;
    return ws + (size_t)P * 12 + (size_t)P * 4 + (size_t)F * 4 + table_bytes(F) + 4 * 256;
}

void free_slot(Slot &s) {
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.ws) (void)hipFree(s.ws);
    if (s.xyz) (void)hipFree(s.xyz);
    if (s.labels) (void)hipFree(s.labels);
    if (s.k_dev) (void)hipFree(s.k_dev);
    if (s.table_dev) (void)hipFree(s.table_dev);
    if (s.table_host) (void)hipHostFree(s.table_host);
    if (s.k_host) (void)hipHostFree(s.k_host);
    s = Slot{};
}

int32_t check_request(int64_t n, float d, int32_t min_size, int32_t max_size, const float *xyz,
                      const int32_t *labels) {
    if (n < 0 || n > 2147483647LL) return FEC_EINVAL;
    if (!std::isfinite(d) || !(d > 0.0f)) return FEC_EINVAL;
    if (!std::isnormal(d * d)) return FEC_EINVAL;
    if (min_size > max_size) return FEC_EINVAL;
    if (n > 0 && (!xyz || !labels)) return FEC_EINVAL;
    return FEC_OK;
}

// Retires slot s if its batch has finished (or, with block, once it has).
// Returns the number of requests completed.
int32_t retire(fec_server *S, Slot &s, bool block) {
    if (!s.busy) return 0;
    hipError_t e = block ? hipEventSynchronize(s.done) : hipEventQuery(s.done);
    if (e == hipErrorNotReady) return 0;
    if (e != hipSuccess) {
        S->error = FEC_EDEVICE;
        return FEC_EDEVICE;
    }
    // A batch's frames share one stacked grid, and its key can need more
    // than 64 bits although each frame's alone fits (frames far apart in
    // extent): the whole batch then comes back FEC_ERANGE.  Its requests go
    // back to the head of the queue, in order, each to run alone, where the
    // result is its own (FEC_ERANGE again only if the frame itself is).
    if (s.reqs.size() > 1) {
        bool all_range = true;
        for (size_t i = 0; i < s.reqs.size(); ++i) all_range &= s.k_host[i] == FEC_ERANGE;
        if (all_range) {
            for (auto it = s.reqs.rbegin(); it != s.reqs.rend(); ++it) {
                Req r = *it;
                r.alone = true;
                S->queue.push_front(r);
            }
            S->n_requeued += (int64_t)s.reqs.size();
            s.reqs.clear();
            s.busy = false;
            return 0;
        }
    }
    const auto now = Clock::now();
    int32_t c = 0;
    for (size_t i = 0; i < s.reqs.size(); ++i) {
        const Req &r = s.reqs[i];
        const double ms = std::chrono::duration<double, std::milli>(now - r.t_submit).count();
        S->done.push_back({r.ticket, s.k_host[i], ms});
        ++c;
    }
    S->n_completed += c;
    s.reqs.clear();
    s.busy = false;
    return c;
}

// Launches the head of the queue into free slot s.
int32_t launch(fec_server *S, Slot &s) {
    std::vector<Req> batch;
    int64_t pts = 0;
    while (!S->queue.empty() && (int32_t)batch.size() < S->slot_frames &&
           pts + S->queue.front().n <= S->slot_points) {
        if (S->queue.front().alone && !batch.empty()) break;  // it runs on its own
        pts += S->queue.front().n;
        batch.push_back(S->queue.front());
        S->queue.pop_front();
        if (batch.back().alone) break;
    }
    if (batch.empty()) return 0;
    const int32_t F = (int32_t)batch.size();
    if (F == 1 && batch[0].n > 0) {
        // a lone request runs the single-cloud pipeline on the caller's own
        // buffers: no table, gather or scatter (the common case at low load)
        const Req &r = batch[0];
        const fec::Layout L1 = fec::make_layout(r.n, 1);
        fec::CallArgs a{};
        a.xyz = r.xyz;
        a.n = r.n;
        a.nframes = 1;
        a.d = r.d;
        a.min_size = r.min_size;
        a.max_size = r.max_size;
        a.labels_out = r.labels;
        a.k_out = s.k_dev;
        hipError_t e = L1.total <= s.ws_bytes ? fec::launch_pipeline(a, s.ws, L1, s.stream, nullptr)
                                              : hipErrorInvalidValue;
        if (e == hipSuccess)
            e = hipMemcpyAsync(s.k_host, s.k_dev, sizeof(int32_t), hipMemcpyDeviceToHost,
                               s.stream);
        if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) {
            S->error = FEC_EDEVICE;
            return FEC_EDEVICE;
        }
        s.reqs = std::move(batch);
        s.busy = true;
        ++S->n_batches;
        S->max_batch_frames = std::max<int64_t>(S->max_batch_frames, 1);
        int64_t busy = 0;
        for (auto &q : S->slots) busy += q.busy ? 1 : 0;
        S->max_in_flight = std::max(S->max_in_flight, busy);
        return 1;
    }
    const fec::Layout L = fec::make_layout(pts, F);
    if (L.total > s.ws_bytes) {  // cannot happen with the slot sizing; refuse loudly
        for (auto it = batch.rbegin(); it != batch.rend(); ++it) S->queue.push_front(*it);
        S->error = FEC_EDEVICE;
        return FEC_EDEVICE;
    }
    TableView th = table_view(s.table_host, F);
    int64_t off = 0;
    for (int32_t f = 0; f < F; ++f) {
        th.offsets[f] = off;
        off += batch[f].n;
        th.src[f] = batch[f].xyz;
        th.dst[f] = batch[f].labels;
        th.d[f] = batch[f].d;
        th.mn[f] = batch[f].min_size;
        th.mx[f] = batch[f].max_size;
    }
    th.offsets[F] = off;
    TableView td = table_view(s.table_dev, F);
    hipError_t e = hipMemcpyAsync(s.table_dev, s.table_host, table_bytes(F),
                                  hipMemcpyHostToDevice, s.stream);
    const int nb = (int)std::min<int64_t>(std::max<int64_t>((3 * pts + 255) / 256, 1), 8192);
    if (e == hipSuccess) {
        k_serve_gather<<<nb, kServeBlock, 0, s.stream>>>(td.offsets, td.src, F, s.xyz);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        fec::CallArgs a{};
        a.xyz = s.xyz;
        a.n = pts;
        a.nframes = F;
        a.offsets = td.offsets;
        a.d_arr = td.d;
        a.min_arr = td.mn;
        a.max_arr = td.mx;
        a.labels_out = s.labels;
        a.k_out = s.k_dev;
        e = fec::launch_pipeline(a, s.ws, L, s.stream, nullptr);
    }
    if (e == hipSuccess) {
        k_serve_scatter<<<nb, kServeBlock, 0, s.stream>>>(td.offsets, td.dst, F, s.labels);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.k_host, s.k_dev, sizeof(int32_t) * F, hipMemcpyDeviceToHost,
                           s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    if (e != hipSuccess) {
        S->error = FEC_EDEVICE;
        return FEC_EDEVICE;
    }
    s.reqs = std::move(batch);
    s.busy = true;
    ++S->n_batches;
    S->max_batch_frames = std::max<int64_t>(S->max_batch_frames, F);
    int64_t busy = 0;
    for (auto &q : S->slots) busy += q.busy ? 1 : 0;
    S->max_in_flight = std::max(S->max_in_flight, busy);
    return F;
}

}  // namespace

extern "C" {

size_t fec_server_slot_bytes(int64_t slot_points, int32_t slot_frames) {
    if (slot_points < 1 || slot_frames < 1 || slot_frames > kMaxSlotFrames) return 0;
    return slot_bytes_for(slot_points, slot_frames);
}

int32_t fec_server_create(size_t hbm_budget, int32_t nslots, int32_t slot_frames,
                          fec_server **out) {
    if (!out || nslots < 1 || nslots > 64 || slot_frames < 1 || slot_frames > kMaxSlotFrames)
        return FEC_EINVAL;
    *out = nullptr;
    const size_t per = hbm_budget / (size_t)nslots;
    // the largest point capacity whose slot fits the per-slot budget
    int64_t lo = 0, hi = 2147483647LL;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (slot_bytes_for(mid, slot_frames) <= per) lo = mid;
        else hi = mid - 1;
    }
    if (lo < 1) return FEC_ENOMEM;
    fec_server *S = new fec_server();
    (void)hipGetDevice(&S->device);
    S->slot_frames = slot_frames;
    S->slot_points = lo;
    S->slot_bytes = slot_bytes_for(lo, slot_frames);
    S->slots.resize(nslots);
    for (auto &s : S->slots) {
        s.ws_bytes = fec_batch_workspace_bytes(lo, slot_frames) +
                     (size_t)(fec::kBboxBlocks + slot_frames) * 32 + 4096;
        bool ok = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess &&
                  hipMalloc(&s.ws, s.ws_bytes) == hipSuccess &&
                  hipMalloc((void **)&s.xyz, (size_t)lo * 12) == hipSuccess &&
                  hipMalloc((void **)&s.labels, (size_t)lo * 4) == hipSuccess &&
                  hipMalloc((void **)&s.k_dev, (size_t)slot_frames * 4) == hipSuccess &&
                  hipMalloc(&s.table_dev, table_bytes(slot_frames)) == hipSuccess &&
                  hipHostMalloc(&s.table_host, table_bytes(slot_frames), 0) == hipSuccess &&
                  hipHostMalloc((void **)&s.k_host, (size_t)slot_frames * 4, 0) == hipSuccess;
        if (!ok) {
            for (auto &q : S->slots) free_slot(q);
            delete S;
            return FEC_ENOMEM;
        }
    }
    *out = S;
    return FEC_OK;
}

int64_t fec_server_slot_points(const fec_server *S) { return S ? S->slot_points : 0; }

int32_t fec_server_submit(fec_server *S, const float *xyz, int64_t n, float d, int32_t min_size,
                          int32_t max_size, int32_t *labels_out, int64_t *ticket) {
    if (!S) return FEC_EINVAL;
    const int32_t rc = check_request(n, d, min_size, max_size, xyz, labels_out);
    if (rc != FEC_OK) return rc;
    if (n > S->slot_points) return FEC_ENOMEM;  // never fits a slot
    Req r{S->next_ticket++, xyz, n, d, min_size, max_size, labels_out, Clock::now(), false};
    S->queue.push_back(r);
    ++S->n_submitted;
    if (ticket) *ticket = r.ticket;
    return FEC_OK;
}

int32_t fec_server_pump(fec_server *S, int32_t wait) {
    if (!S) return FEC_EINVAL;
    if (S->error != FEC_OK) return S->error;
    int32_t completed = 0;
    for (auto &s : S->slots) {
        const int32_t c = retire(S, s, false);
        if (c < 0) return c;
        completed += c;
    }
    int32_t launched = 0;
    for (auto &s : S->slots) {
        if (S->queue.empty()) break;
        if (s.busy) continue;
        const int32_t f = launch(S, s);
        if (f < 0) return f;
        launched += f;
    }
    if (wait && completed == 0 && launched == 0) {
        // block on the batch launched first among those in flight
        Slot *oldest = nullptr;
        for (auto &s : S->slots)
            if (s.busy && (!oldest || s.reqs.front().ticket < oldest->reqs.front().ticket))
                oldest = &s;
        if (oldest) {
            const int32_t c = retire(S, *oldest, true);
            if (c < 0) return c;
            completed += c;
            for (auto &s : S->slots) {
                if (S->queue.empty()) break;
                if (s.busy) continue;
                const int32_t f = launch(S, s);
                if (f < 0) return f;
            }
        }
    }
    return completed;
}

int32_t fec_server_pump_for(fec_server *S, int64_t max_wait_us) {
    if (!S || max_wait_us < 0) return FEC_EINVAL;
    int32_t completed = fec_server_pump(S, 0);
    if (completed != 0 || max_wait_us == 0) return completed;
    // spin on the events of the batches in flight (a completion is seen
    // within one event query, not one sleep of the caller)
    const auto until = Clock::now() + std::chrono::microseconds(max_wait_us);
    bool busy = true;
    while (busy && Clock::now() < until) {
        busy = false;
        for (auto &s : S->slots) {
            if (!s.busy) continue;
            busy = true;
            const int32_t c = retire(S, s, false);
            if (c < 0) return c;
            completed += c;
        }
        if (completed) break;
    }
    if (completed) {  // refill the slots just freed
        for (auto &s : S->slots) {
            if (S->queue.empty()) break;
            if (s.busy) continue;
            const int32_t f = launch(S, s);
            if (f < 0) return f;
        }
    }
    return completed;
}

int32_t fec_server_poll(fec_server *S, int64_t *tickets, int32_t *k, double *latency_ms,
                        int32_t max) {
    if (!S || max < 0) return FEC_EINVAL;
    int32_t c = 0;
    while (c < max && !S->done.empty()) {
        const auto &d = S->done.front();
        if (tickets) tickets[c] = d.ticket;
        if (k) k[c] = d.k;
        if (latency_ms) latency_ms[c] = d.latency_ms;
        S->done.pop_front();
        ++c;
    }
    return c;
}

int32_t fec_server_stats(const fec_server *S, int64_t *out, int32_t max_out) {
    if (!S || !out || max_out <= 0) return FEC_EINVAL;
    int64_t busy = 0;
    for (auto &s : S->slots) busy += s.busy ? 1 : 0;
    const int64_t v[10] = {S->n_submitted,
                           S->n_completed,
                           S->n_batches,
                           (int64_t)S->queue.size(),
                           busy,
                           S->max_batch_frames,
                           S->max_in_flight,
                           S->slot_points,
                           (int64_t)S->slot_bytes,
                           S->n_requeued};
    const int32_t c = max_out < 10 ? max_out : 10;
    for (int32_t i = 0; i < c; ++i) out[i] = v[i];
    return c;
}

void fec_server_destroy(fec_server *S) {
    if (!S) return;
    for (auto &s : S->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        free_slot(s);
    }
    delete S;
}

}  // extern "C"
