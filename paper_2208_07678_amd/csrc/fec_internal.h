// Internal definitions shared by the device pipeline and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fec {

// ---------------------------------------------------------------- tiling
constexpr int kBlock = 256;            // threads per block of the streaming kernels
constexpr int kItems = 16;             // elements per thread in tiled kernels
constexpr int kTile = kBlock * kItems; // elements per tile (sort, gather, cells)
// Row pitch of the sort's per-tile tables: the tile count rounded up to a
// multiple of 4, so that every row starts on a 16-byte boundary.
constexpr int64_t tile_pitch(int64_t ntiles) { return (ntiles + 3) & ~(int64_t)3; }
constexpr int kListBlocks = 1024;      // most blocks of the work-list kernels
// Radix sort digits: 8 to 11 bits per pass, chosen per call on the host
// (the autotuner's knob); tables are sized for the widest.
constexpr int kMinRadixBits = 8;
constexpr int kMaxRadixBits = 11;
constexpr int kMaxRadix = 1 << kMaxRadixBits;
constexpr int kMaxPasses = (64 + kMinRadixBits - 1) / kMinRadixBits;
constexpr int kDefaultRadixBits = 9;
// Pass schedule: pass p sorts key bits [pass_bit0(rb, p), + pass_width(rb, p)).
// At 9-bit digits the passes after the first four (36 bits, the map's 34-bit
// key and narrower) take 10 bits each, so 7 passes cover a 64-bit key
// instead of 8; every pass the host enqueues costs a launch even when the
// device-side pass count makes it return at once.  Other widths are uniform.
__host__ __device__ constexpr int pass_width(int rb, int p) {
    return (rb == 9 && p >= 4) ? 10 : rb;
}
__host__ __device__ constexpr int pass_bit0(int rb, int p) {
    return (rb == 9 && p > 4) ? 36 + 10 * (p - 4) : rb * p;
}
__host__ __device__ constexpr int passes_for(int rb, int key_bits) {
    return (rb == 9 && key_bits > 36) ? 4 + (key_bits - 36 + 9) / 10 : (key_bits + rb - 1) / rb;
}
static_assert(passes_for(9, 64) == 7 && pass_bit0(9, 6) + pass_width(9, 6) >= 64 &&
                  pass_bit0(9, 4) == 36 && passes_for(9, 36) == 4 && passes_for(9, 37) == 5,
              "the 9-bit schedule covers 64 key bits in 7 passes");
static_assert(passes_for(kMinRadixBits, 64) <= kMaxPasses, "per-pass tables");
constexpr int kBboxBlocks = 1024;      // max blocks of the bounding-box reduction
constexpr int kCellBlocks = 4096;      // grid of the grid-stride per-cell kernels
// Dense column index: one entry per (cx, cy) when the plane has at most
// kColGridPerPoint entries per point (else hashed or binary-searched).  A
// batch of single scans stacks its frames' planes along x and needs about
// 11 (sized to the largest frame's width in y); the no-allocation entry
// point keeps 8, to fit its static workspace.
constexpr int kColGridPerPoint = 16;
constexpr int kColGridPerPointNoAlloc = 8;
// Frames of one batched call (each frame is an independent cloud).
constexpr int32_t kMaxFrames = 65536;


// Device-side status values (mirror the public FEC_* codes).
constexpr int32_t kStatusOk = 0;
constexpr int32_t kStatusInval = -1;
constexpr int32_t kStatusRange = -2;
constexpr int32_t kStatusDevice = -4;

// One frame of a batched call.  Every frame has its own grid (its own d,
// hence cell side, and its own bounding box); the grids are laid side by
// side along x, frame after frame, with two empty cell columns between
// consecutive frames, so the stencil (reach two cells) never joins cells of
// different frames and one sorted key order covers the whole batch.
struct Frame {
    int64_t off0, off1;  // the frame's points [off0, off1) of the batch
    int64_t nvalid;      // finite points (0 when the frame's arguments are refused)
    int64_t xoff;        // first x cell of the frame in the stacked grid
    double ox, oy, oz;   // grid origin: bounding box minimum of the finite points
    double inv_s;        // 1 / cell side (0 for a refused frame)
    int64_t NX, NY, NZ;  // the frame's own grid extent
    float d, d2;         // threshold and fl32(d * d)
    int32_t min_size;    // clamped to >= 1
    int32_t max_size;
    int32_t status;      // kStatusOk, kStatusInval (arguments) or kStatusRange (extent)
    int32_t kept;        // kept clusters
    int32_t giant;       // root of the frame's largest component after sampling (-1: none)
    uint32_t cell0;      // the frame's first cell (when nvalid > 0)
};

// Per-call state, kept at the start of the workspace.  Written by the
// planning kernel, read by every later kernel of the call.  With several
// frames the grid fields describe the stacked grid; d, d2, origin and the
// size bounds are those of frame 0 (the only frame of a single-cloud call).
struct Params {
    int64_t n;
    float d;
    float d2;          // fl32(d * d): the predicate's threshold
    int32_t min_size;  // already clamped to >= 1
    int32_t max_size;
    int32_t status;
    int32_t nframes;
    int64_t nvalid;    // points with three finite coordinates (of accepted frames)
    double ox, oy, oz; // grid origin: the bounding box minimum of finite points
    double inv_s;      // 1 / cell side
    int64_t NX, NY, NZ;
    int64_t NYp;          // row stride of the dense column index: NY rounded up to 32
    int32_t bx, by, bz;   // key bits per axis: key = cx << (by+bz) | cy << bz | cz
    int32_t key_bits;     // bits sorted (grid key, plus one for non-finite points)
    int32_t idx_bits;     // bits of the point index packed below the key
    int32_t npasses;      // radix passes actually run
    int32_t radix_bits;   // bits per radix pass
    int32_t pad0;
    int32_t pair_mode;    // 0: one word (key << idx_bits | index); 1: key and index arrays
    int32_t key_shift;    // idx_bits in one-word mode, 0 in pair mode
    uint64_t idx_mask;
    int64_t M;            // occupied cells
    int64_t Mcol;         // occupied columns (cells sharing cx, cy)
    int32_t dense_cols;   // 1: column lookups through the dense (cx, cy) index
    int32_t giant;        // root of the largest component (-1: none)
    uint32_t nwork;       // cells outside it after the near shell (far-shell work list)
    uint32_t nwork0;      // cells outside it after the sampling links (near-shell work list)
    // Cell pairs whose first points are not joined, queued by the near and
    // the far shell for a full test once the shell's other joins are in.
    uint32_t ndefer[2];
    // Consecutive cell pairs of the runs pass whose first points are not
    // joined, tested after the near shell with the queued pairs above.
    uint32_t nrunq;
    uint32_t pad2;
    int32_t kept;         // kept clusters
    int32_t max_cell;     // largest number of points in one cell
    // Hashed column index (when the dense one does not fit): open addressing
    // with linear probing over 64-bit slots (column key << 31 | first cell,
    // all ones = empty) in the dense index's memory.
    int32_t hashed_cols;  // 1: column lookups through the hash table
    int32_t hshift;       // slot of key k: (k * golden) >> hshift
    uint64_t hmask;       // slots - 1
    uint64_t hcap;        // slots that fit in the dense index's memory (a power of two)
    unsigned long long counters[8];  // diagnostic event counts (counting builds only)
};

// ---------------------------------------------------------------- workspace
struct Layout {
    size_t params, frames, partials, tile_cnt, tile_off;
    size_t keys0, keys1, vals0, vals1, th, dtot;
    size_t spts, sorig, cell_start, cell_key, cpar, csize, ccanon;
    size_t col_key, col_cell, colgrid, colbits, heads, blkhead, gbits, listcnt, work, cell_frame,
        defer, runq;
    uint64_t defer_cap;  // entries of the deferred-pair queue
    uint64_t colgrid_cap;
    size_t total;
    int64_t ntiles;
    int32_t nframes;
    int32_t bbox_per_frame;  // blocks of the bounding-box reduction per frame
};

constexpr uint64_t next_pow2(uint64_t v) {
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bounding-box blocks per frame: about kBboxBlocks in all, at most one per
// 1024 points of an average frame, at least one.
constexpr int32_t bbox_blocks_per_frame(int64_t n, int32_t nframes) {
    const int64_t f = nframes > 0 ? nframes : 1;
    int64_t b = kBboxBlocks / f;
    const int64_t need = (n / f + 1023) / 1024;
    if (b > need) b = need;
    return (int32_t)(b < 1 ? 1 : b);
}

constexpr Layout make_layout(int64_t n, int32_t nframes = 1,
                             int col_per_point = kColGridPerPoint) {
    Layout L{};
    L.nframes = nframes;
    L.bbox_per_frame = bbox_blocks_per_frame(n, nframes);
    const size_t A = 256;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, A);
        return o;
    };
    const size_t un = (size_t)(n > 0 ? n : 1);
    L.ntiles = (int64_t)((un + kTile - 1) / kTile);
    L.params = take(sizeof(Params));
    L.frames = take((size_t)nframes * sizeof(Frame));
    L.partials = take((size_t)nframes * L.bbox_per_frame * 8 * sizeof(float));
    L.tile_cnt = take((size_t)L.ntiles * 2 * sizeof(uint32_t));
    L.tile_off = take((size_t)L.ntiles * 2 * sizeof(uint32_t));
    L.keys0 = take(un * sizeof(uint64_t));
    L.keys1 = take(un * sizeof(uint64_t));
    L.vals0 = take(un * sizeof(uint32_t));
    L.vals1 = take(un * sizeof(uint32_t));
    L.th = take((size_t)tile_pitch(L.ntiles) * kMaxRadix * sizeof(uint32_t));
    L.dtot = take((size_t)kMaxPasses * kMaxRadix * sizeof(uint32_t));
    L.spts = take(un * sizeof(float4));
    L.sorig = take(un * sizeof(uint32_t));
    L.cell_start = take((un + 1) * sizeof(uint32_t));
    L.cell_key = take(un * sizeof(uint64_t));
    L.cpar = take(un * sizeof(int32_t));
    L.csize = take(un * sizeof(int32_t));
    L.ccanon = take(un * sizeof(int32_t));
    L.col_key = take(un * sizeof(uint64_t));
    L.col_cell = take((un + 1) * sizeof(uint32_t));
    L.colgrid_cap = (uint64_t)col_per_point * un + 1024;
    L.colgrid = take((size_t)L.colgrid_cap * sizeof(uint32_t));
    L.colbits = take((size_t)(L.colgrid_cap / 32 + 2) * sizeof(uint32_t));
    L.heads = take(un);
    L.blkhead = take((size_t)L.ntiles * sizeof(int32_t));
    L.gbits = take((un / 64 + 1) * sizeof(uint64_t));
    L.listcnt = take((size_t)kListBlocks * sizeof(uint32_t));
    L.work = take(un * sizeof(uint32_t));
    L.defer_cap = un / 2 + 1024;
    L.defer = take((size_t)L.defer_cap * sizeof(uint64_t));
    // at most one pair per cell; in the memory of the sort's second index
    // array, which nothing reads after the gather
    L.runq = L.vals1;
    L.cell_frame = take(nframes > 1 ? un * sizeof(uint32_t) : 0);  // frame of every cell
    L.total = off;
    return L;
}

// ---------------------------------------------------------------- stages
enum Stage : int {
    kStBbox = 0,
    kStPlan,
    kStKeys,
    kStSortHist,
    kStSortScan,
    kStSort,
    kStGather,
    kStTileScan,
    kStCells,
    kStColGrid,
    kStRuns,
    kStSample,
    kStGiant0,
    kStHookNear,
    kStDeferred,
    kStCompress1,
    kStGiant,
    kStWorkList,
    kStHookFar,
    kStCompress2,
    kStFinalCells,
    kStFinalLabels,
    kStFinish,
    kNumStages
};

const char *stage_name(int s);

// Timing hook: called around each launch; records events when enabled.
struct Timer {
    virtual void begin(int stage, hipStream_t s) = 0;
    virtual void end(int stage, hipStream_t s) = 0;
    virtual ~Timer() {}
};

// Arguments of one call: a single cloud (nframes == 1, the scalars d,
// min_size, max_size; offsets and the per-frame arrays null) or a batch of
// frames (device arrays offsets[nframes + 1], d[nframes], min_size[nframes],
// max_size[nframes]).  Labels are frame-local: the smallest index of the
// cluster counted from the frame's first point.  k_out holds one value per
// frame.
struct CallArgs {
    const float *xyz;
    int64_t n;
    int32_t nframes;
    const int64_t *offsets;
    const float *d_arr;
    const int32_t *min_arr, *max_arr;
    float d;
    int32_t min_size, max_size;
    int32_t *labels_out;
    int32_t *k_out;
};

// Launch shape of the grid-stride kernels, settable at run time (the
// autotuner's knobs): blocks of the per-cell kernels (near / far shells,
// compression, finalize) and of the per-point streaming kernels.  Results do
// not depend on them.
struct Tuning {
    int32_t cell_blocks;
    int32_t stream_blocks;
    int32_t radix_bits;  // bits per radix-sort pass (8 .. 11)
    int32_t hook_block;  // threads per block of the hooking kernels (64, 128, 256)
    int32_t near_sampling;  // sampling links before the near shell: 0 by size, 1 on, 2 off
};
constexpr int32_t kDefaultCellBlocks = kCellBlocks;
constexpr int32_t kDefaultStreamBlocks = 4096;
constexpr int32_t kDefaultHookBlock = 256;
Tuning tuning();
void set_tuning(Tuning t);

// Enqueues one kernel that writes v to *k_out (the count of an empty call:
// no host-side write, so the asynchronous form stays capturable).
hipError_t launch_set_count(int32_t *k_out, int32_t v, hipStream_t stream);

// Enqueues the whole pipeline.  Returns hipSuccess or the first launch error.
hipError_t launch_pipeline(const CallArgs &a, void *ws, const Layout &L, hipStream_t stream,
                           Timer *timer);

}  // namespace fec
