// Fixed-radius Euclidean clustering on gfx950: the device pipeline.
//
// The result is the clustering of Sec. 2.2 (Eq. (1), Alg. 1): connected
// components of the graph that joins points closer than d, then the inclusive
// min/max size filter, labels = smallest member index.  The paper's serial
// point-wise loop is replaced by a grid-based design:
//
//   bbox -> plan -> keys -> radix sort passes -> gather -> cell table
//   -> column index (dense table, hash or search) -> runs -> sampling links
//   -> compress -> giant component / work list -> hook (near shell)
//   -> compress -> giant component / work list -> hook (far shell)
//   -> compress -> cluster sizes/ids -> labels
//
// One call covers one cloud or a batch of frames: every frame has its own
// grid, and the frames' grids are laid side by side along x (see k_plan).
//
// Grid.  Cells are cubes of side s = d (1 - 2^-10) / sqrt(3).  Any two points
// of one cell are closer than s*sqrt(3) < d (with room for the rounding of
// the binary32 test), so every cell is a clique of the graph and the
// union-find runs over cells, not points.  A pair the binary32 test accepts
// is closer than d (1 + 2^-22) < 2 s, so joined points lie in cells at most
// two apart on every axis: the 5x5x5 stencil.  Half of it is visited
// (forward offsets), so each unordered cell pair is examined once.
//
// Hooking.  Two cells are in one cluster as soon as ONE pair of their points
// is joined, so a cell pair is tested point pair by point pair only until
// the first joined pair, and not at all when both cells already share a
// union-find root.  The near shell (offsets within 1) runs first; after a
// compression most of a dense surface is one component, and the far shell
// (offsets of 2) visits only the cells outside it.  On large clouds the near
// shell itself is preceded by one round of sampled links and runs only for
// the cells outside the component these form.
//
// Determinism.  The union-find always hooks the root of higher rank under
// the other (rank: a fixed scramble of the cell id); the partition it
// reaches is the unique set of components, and the labels (smallest
// original index per component) do not depend on timing.

#include "fec_internal.h"

#include <float.h>
#include <math.h>

#include <atomic>

namespace fec {

// ------------------------------------------------------------------ helpers

// Diagnostic event counts, compiled in with -DFEC_COUNTERS only.
#ifdef FEC_COUNTERS
#define FEC_COUNT(P, i, v) atomicAdd(&((Params *)(P))->counters[i], (unsigned long long)(v))
#else
#define FEC_COUNT(P, i, v) ((void)0)
#endif

__device__ __forceinline__ uint64_t lanemask_lt() {
    const unsigned l = __lane_id();
    return l ? (~0ull >> (64 - l)) : 0ull;
}

__device__ __forceinline__ int first_lane(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ int bits_for(int64_t v) {  // bits to hold 0 .. v-1
    return v <= 1 ? 0 : 64 - __clzll((unsigned long long)(v - 1));
}

// Eq. (1), strict, in binary32 with the fixed order (dx*dx + dy*dy) + dz*dz.
__device__ __forceinline__ bool joined(float ax, float ay, float az, float4 b, float d2) {
#pragma clang fp contract(off)
    const float dx = ax - b.x;
    const float dy = ay - b.y;
    const float dz = az - b.z;
    float s = dx * dx + dy * dy;
    s = s + dz * dz;
    return s < d2;
}

__device__ __forceinline__ bool finite3(float x, float y, float z) {
    return isfinite(x) && isfinite(y) && isfinite(z);
}

// Block-wide exclusive scan of one value per thread (kBlock threads).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_tmp, uint32_t &total) {
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_tmp[wave] = x;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        uint32_t t = s_tmp[w];
        before += (w < wave) ? t : 0u;
        tot += t;
    }
    total = tot;
    return before + x - v;
}

// ------------------------------------------------------------- 1. bbox
// The point range of frame f: [0, n) for a single cloud, else the caller's
// offsets clamped into [0, n] (the planning kernel refuses a batch whose
// offsets do not partition [0, n), so clamping only keeps reads in range).
__device__ __forceinline__ void frame_range(const int64_t *offs, int64_t n, int f, int64_t &lo,
                                            int64_t &hi) {
    if (!offs) {
        lo = 0;
        hi = n;
        return;
    }
    int64_t a = offs[f], b = offs[f + 1];
    a = a < 0 ? 0 : (a > n ? n : a);
    b = b < a ? a : (b > n ? n : b);
    lo = a;
    hi = b;
}

// Frame holding original point index i: the last frame with off0 <= i.
__device__ __forceinline__ int frame_of_point(const Frame *frames, int nframes, int64_t i) {
    int lo = 0, hi = nframes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (frames[mid].off0 <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Per-block min/max of the finite points of one frame and their count;
// block f * per_frame + j takes the j-th share of frame f.
__global__ __launch_bounds__(kBlock) void k_bbox(const float *__restrict__ xyz, int64_t n,
                                                 const int64_t *__restrict__ offs, int per_frame,
                                                 float *__restrict__ partials) {
    const int f = blockIdx.x / per_frame, j = blockIdx.x % per_frame;
    int64_t lo, hi;
    frame_range(offs, n, f, lo, hi);
    float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY;
    float hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    uint32_t cnt = 0;
    auto take = [&](float x, float y, float z) {
        if (finite3(x, y, z)) {
            lo0 = fminf(lo0, x); lo1 = fminf(lo1, y); lo2 = fminf(lo2, z);
            hi0 = fmaxf(hi0, x); hi1 = fmaxf(hi1, y); hi2 = fmaxf(hi2, z);
            ++cnt;
        }
    };
    const int64_t stride = (int64_t)per_frame * kBlock;
    int64_t i = lo + (int64_t)j * kBlock + threadIdx.x;
    constexpr int kU = 4;  // points per lane whose loads are in flight together
    for (; i + (kU - 1) * stride < hi; i += kU * stride) {
        float x[kU], y[kU], z[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t q = i + u * stride;
            x[u] = xyz[3 * q];
            y[u] = xyz[3 * q + 1];
            z[u] = xyz[3 * q + 2];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) take(x[u], y[u], z[u]);
    }
    for (; i < hi; i += stride) take(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo0 = fminf(lo0, __shfl_xor(lo0, o)); lo1 = fminf(lo1, __shfl_xor(lo1, o));
        lo2 = fminf(lo2, __shfl_xor(lo2, o)); hi0 = fmaxf(hi0, __shfl_xor(hi0, o));
        hi1 = fmaxf(hi1, __shfl_xor(hi1, o)); hi2 = fmaxf(hi2, __shfl_xor(hi2, o));
        cnt += __shfl_xor(cnt, o);
    }
    __shared__ float s[kBlock / 64][7];
    const int wave = threadIdx.x >> 6;
    if (__lane_id() == 0) {
        s[wave][0] = lo0; s[wave][1] = lo1; s[wave][2] = lo2;
        s[wave][3] = hi0; s[wave][4] = hi1; s[wave][5] = hi2;
        s[wave][6] = __uint_as_float(cnt);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float r[6] = {s[0][0], s[0][1], s[0][2], s[0][3], s[0][4], s[0][5]};
        uint32_t c = __float_as_uint(s[0][6]);
        for (int w = 1; w < kBlock / 64; ++w) {
            for (int a = 0; a < 3; ++a) r[a] = fminf(r[a], s[w][a]);
            for (int a = 3; a < 6; ++a) r[a] = fmaxf(r[a], s[w][a]);
            c += __float_as_uint(s[w][6]);
        }
        float *o = partials + (size_t)blockIdx.x * 8;
        for (int a = 0; a < 6; ++a) o[a] = r[a];
        o[6] = __uint_as_float(c);
    }
}

// ------------------------------------------------------------- 2. plan
// Block-wide exclusive scan of 64-bit values (kBlock threads).
__device__ __forceinline__ int64_t block_excl_scan_i64(int64_t v, int64_t *s_tmp, int64_t &total) {
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_tmp[wave] = x;
    __syncthreads();
    int64_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const int64_t t = s_tmp[w];
        before += (w < wave) ? t : 0;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return before + x - v;
}

// Plans frame f from its reduced bounding box (r = min x, y, z, max x, y,
// z) and finite-point count: argument checks, origin, cell side, extent.
// One thread per frame.
__device__ void plan_frame(int f, const float (&r)[6], uint64_t cnt, Frame *__restrict__ frames,
                           int nframes, int64_t n, const int64_t *__restrict__ offs,
                           const float *__restrict__ d_arr, const int32_t *__restrict__ min_arr,
                           const int32_t *__restrict__ max_arr, float d_one, int32_t min_one,
                           int32_t max_one, int32_t *s_bad) {
    Frame F;
    if (offs) {
        const int64_t a = offs[f], b = offs[f + 1];
        if (a > b || (f == 0 && a != 0) || (f == nframes - 1 && b != n)) *s_bad = 1;
    }
    frame_range(offs, n, f, F.off0, F.off1);
    F.d = d_arr ? d_arr[f] : d_one;
    const int32_t mn = min_arr ? min_arr[f] : min_one;
    F.max_size = max_arr ? max_arr[f] : max_one;
    F.min_size = mn < 1 ? 1 : mn;
    F.d2 = __fmul_rn(F.d, F.d);
    F.status = kStatusOk;
    // the same argument checks as the host applies to a single cloud
    if (!isfinite(F.d) || !(F.d > 0.0f) || !(F.d2 >= FLT_MIN) || isinf(F.d2) ||
        mn > F.max_size)
        F.status = kStatusInval;
    F.kept = 0;
    F.giant = -1;
    F.cell0 = 0;
    F.xoff = 0;
    int64_t N3[3] = {1, 1, 1};
    double o3[3] = {0.0, 0.0, 0.0};
    double inv = 0.0;
    if (F.status == kStatusOk) {
        const double side = (double)F.d * (1.0 - 0x1p-10) / sqrt(3.0);
        inv = 1.0 / side;
        if (cnt > 0) {
            for (int a = 0; a < 3; ++a) {
                o3[a] = (double)r[a];
                const double ext = ((double)r[a + 3] - (double)r[a]) * inv;
                if (!(ext < 0x1p31)) {
                    F.status = kStatusRange;
                } else {
                    N3[a] = (int64_t)floor(ext) + 1;
                }
            }
        }
    }
    if (F.status != kStatusOk) {  // a refused frame holds no cell
        inv = 0.0;
        N3[0] = N3[1] = N3[2] = 1;
        o3[0] = o3[1] = o3[2] = 0.0;
        cnt = 0;
    }
    F.nvalid = (int64_t)cnt;
    F.inv_s = inv;
    F.ox = o3[0]; F.oy = o3[1]; F.oz = o3[2];
    F.NX = N3[0]; F.NY = N3[1]; F.NZ = N3[2];
    frames[f] = F;
}

// Fixes every frame's grid, stacks the frames' grids along x, and fixes the
// key layout and the number of radix passes.  One block: wave w plans the
// frames w, w + 4, ...; then the block scans the frames' widths.
__global__ __launch_bounds__(kBlock) void k_plan(const float *__restrict__ partials,
                                                 int per_frame, Params *__restrict__ P,
                                                 Frame *__restrict__ frames, int nframes,
                                                 int64_t n, const int64_t *__restrict__ offs,
                                                 const float *__restrict__ d_arr,
                                                 const int32_t *__restrict__ min_arr,
                                                 const int32_t *__restrict__ max_arr, float d_one,
                                                 int32_t min_one, int32_t max_one,
                                                 uint64_t colgrid_cap, int radix_bits) {
    __shared__ int64_t s_tmp[kBlock / 64];
    __shared__ int32_t s_bad;
    const int wave = threadIdx.x >> 6, lane = __lane_id();

    if (threadIdx.x < 8) P->counters[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();

    if (nframes == 1) {
        // one cloud: the whole block reduces its partial boxes
        float r[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        uint64_t cnt = 0;
#pragma unroll 4
        for (int b = threadIdx.x; b < per_frame; b += kBlock) {
            const float *q = partials + (size_t)b * 8;
            for (int a = 0; a < 3; ++a) r[a] = fminf(r[a], q[a]);
            for (int a = 3; a < 6; ++a) r[a] = fmaxf(r[a], q[a]);
            cnt += __float_as_uint(q[6]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            for (int a = 0; a < 3; ++a) r[a] = fminf(r[a], __shfl_xor(r[a], o));
            for (int a = 3; a < 6; ++a) r[a] = fmaxf(r[a], __shfl_xor(r[a], o));
            cnt += __shfl_xor(cnt, o);
        }
        __shared__ float s_r[kBlock / 64][6];
        __shared__ uint64_t s_c[kBlock / 64];
        if (lane == 0) {
            for (int a = 0; a < 6; ++a) s_r[wave][a] = r[a];
            s_c[wave] = cnt;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < kBlock / 64; ++w) {
                for (int a = 0; a < 3; ++a) r[a] = fminf(r[a], s_r[w][a]);
                for (int a = 3; a < 6; ++a) r[a] = fmaxf(r[a], s_r[w][a]);
                cnt += s_c[w];
            }
            plan_frame(0, r, cnt, frames, nframes, n, offs, d_arr, min_arr, max_arr, d_one,
                       min_one, max_one, &s_bad);
        }
    } else if (per_frame <= 16) {
        // many frames, few partial boxes each: one thread per frame
        for (int f = threadIdx.x; f < nframes; f += kBlock) {
            float r[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
            uint64_t cnt = 0;
            for (int b = 0; b < per_frame; ++b) {
                const float *q = partials + ((size_t)f * per_frame + b) * 8;
                for (int a = 0; a < 3; ++a) r[a] = fminf(r[a], q[a]);
                for (int a = 3; a < 6; ++a) r[a] = fmaxf(r[a], q[a]);
                cnt += __float_as_uint(q[6]);
            }
            plan_frame(f, r, cnt, frames, nframes, n, offs, d_arr, min_arr, max_arr, d_one,
                       min_one, max_one, &s_bad);
        }
    } else
    for (int f = wave; f < nframes; f += kBlock / 64) {
        float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY;
        float hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
        uint64_t cnt = 0;
        for (int b = lane; b < per_frame; b += 64) {
            const float *q = partials + ((size_t)f * per_frame + b) * 8;
            lo0 = fminf(lo0, q[0]); lo1 = fminf(lo1, q[1]); lo2 = fminf(lo2, q[2]);
            hi0 = fmaxf(hi0, q[3]); hi1 = fmaxf(hi1, q[4]); hi2 = fmaxf(hi2, q[5]);
            cnt += __float_as_uint(q[6]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo0 = fminf(lo0, __shfl_xor(lo0, o)); lo1 = fminf(lo1, __shfl_xor(lo1, o));
            lo2 = fminf(lo2, __shfl_xor(lo2, o)); hi0 = fmaxf(hi0, __shfl_xor(hi0, o));
            hi1 = fmaxf(hi1, __shfl_xor(hi1, o)); hi2 = fmaxf(hi2, __shfl_xor(hi2, o));
            cnt += __shfl_xor(cnt, o);
        }
        if (lane != 0) continue;
        const float r[6] = {lo0, lo1, lo2, hi0, hi1, hi2};
        plan_frame(f, r, cnt, frames, nframes, n, offs, d_arr, min_arr, max_arr, d_one, min_one,
                   max_one, &s_bad);
    }
    __syncthreads();

    // x offsets: NX of every earlier frame plus a gap of two empty columns
    __shared__ unsigned long long s_ny, s_nz, s_nv;
    if (threadIdx.x == 0) s_ny = s_nz = 1, s_nv = 0;
    int64_t carry = 0;
    for (int c0 = 0; c0 < nframes; c0 += kBlock) {
        const int f = c0 + threadIdx.x;
        const bool in = f < nframes;
        const int64_t w = in ? frames[f].NX + 2 : 0;
        int64_t tot;
        const int64_t before = block_excl_scan_i64(w, s_tmp, tot);
        if (in) frames[f].xoff = carry + before;
        carry += tot;
        uint64_t ny = in ? (uint64_t)frames[f].NY : 1, nz = in ? (uint64_t)frames[f].NZ : 1;
        uint64_t nv = in ? (uint64_t)frames[f].nvalid : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t a = __shfl_xor(ny, o), b = __shfl_xor(nz, o);
            ny = a > ny ? a : ny;
            nz = b > nz ? b : nz;
            nv += __shfl_xor(nv, o);
        }
        if (lane == 0) {
            atomicMax(&s_ny, (unsigned long long)ny);
            atomicMax(&s_nz, (unsigned long long)nz);
            atomicAdd(&s_nv, (unsigned long long)nv);
        }
    }
    __syncthreads();
    const int64_t NY = (int64_t)s_ny, NZ = (int64_t)s_nz, nvalid = (int64_t)s_nv;
    if (threadIdx.x != 0) return;

    const Frame &F0 = frames[0];
    P->n = n;
    P->nframes = nframes;
    P->d = F0.d;
    P->d2 = F0.d2;
    P->min_size = F0.min_size;
    P->max_size = F0.max_size;
    P->status = s_bad ? kStatusInval : kStatusOk;
    P->nvalid = nvalid;
    P->kept = 0;
    P->M = 0;
    P->Mcol = 0;
    P->max_cell = 0;
    P->inv_s = F0.inv_s;
    P->ox = F0.ox; P->oy = F0.oy; P->oz = F0.oz;
    const int64_t NX = carry - 2;  // no gap after the last frame
    P->NX = NX; P->NY = NY; P->NZ = NZ;
    P->NYp = (NY + 31) / 32 * 32;
    P->bx = bits_for(NX);
    P->by = bits_for(NY);
    P->bz = bits_for(NZ);
    P->giant = -1;
    P->nwork = 0;
    P->nwork0 = 0;
    P->ndefer[0] = P->ndefer[1] = 0;
    P->nrunq = 0;
    P->dense_cols = ((double)NX * (double)P->NYp <= (double)colgrid_cap) ? 1 : 0;
    P->hashed_cols = 0;
    uint64_t hcap = 1;
    while (hcap * 2 <= colgrid_cap / 2) hcap *= 2;  // 8-byte slots in 4-byte entries
    P->hcap = hcap;
    P->hmask = 0;
    P->hshift = 64;
    const int B = P->bx + P->by + P->bz;
    const int kb = B + ((nvalid < n) ? 1 : 0);
    int ib = bits_for(n);
    if (ib < 1) ib = 1;
    P->key_bits = kb;
    P->idx_bits = ib;
    P->idx_mask = (1ull << ib) - 1;
    // One 64-bit word per point when key and index fit together, otherwise
    // separate key and index arrays; beyond a 64-bit key the grid is refused.
    P->pair_mode = (kb + ib > 64) ? 1 : 0;
    P->key_shift = P->pair_mode ? 0 : ib;
    if (kb > 64 && P->status == kStatusOk) P->status = kStatusRange;
    if (nframes == 1 && F0.status != kStatusOk && P->status == kStatusOk) P->status = F0.status;
    P->radix_bits = radix_bits;
    P->npasses = P->status == kStatusOk ? passes_for(radix_bits, kb) : 0;
}

// Cell key: cx, then cy, then cz.  The cells of one column (cx, cy) are
// contiguous after sorting, and so are the columns of one row cx.
__device__ __forceinline__ uint64_t make_key(uint64_t cx, uint64_t cy, uint64_t cz, int by,
                                             int bz) {
    return (((cx << by) | cy) << bz) | cz;
}

// Blocks go to the 8 XCDs round-robin by block id, and each XCD has its own
// L2.  xcd_block<C>() renumbers the blocks so that each XCD runs runs of C
// consecutive block numbers: in every whole group of 8C blocks, XCD x takes
// numbers x*C .. x*C+C-1; blocks past the last whole group keep their
// numbers.  Neighbouring work (a cell's neighbours in the next x slab, a few
// hundred cells further on) is then done by one XCD at about the same time,
// through one L2; groups keep rotating over the XCDs, so the load stays
// spread when the work varies along the cells.  A bijection on
// [0, gridDim.x); C = 1 is the identity.
constexpr uint32_t kXcds = 8;
template <uint32_t C>
__device__ __forceinline__ int64_t xcd_block() {
    const uint32_t g = gridDim.x, b = blockIdx.x, span = kXcds * C;
    const uint32_t full = g - g % span;  // blocks in whole groups
    if (C == 1 || b >= full) return b;
    const uint32_t r = b % span;
    return (int64_t)(b - r) + (r % kXcds) * C + r / kXcds;
}

// The same with C = gridDim.x / 8: each XCD runs one contiguous eighth of
// the block numbers (the last gridDim.x % 8 blocks keep theirs).  For
// kernels whose blocks all do the same work.
__device__ __forceinline__ int64_t xcd_block_eighths() {
    const uint32_t g = gridDim.x, b = blockIdx.x, C = g / kXcds;
    if (C <= 1 || b >= kXcds * C) return b;
    return (int64_t)(b % kXcds) * C + b / kXcds;
}

// ------------------------------------------------------------- 3. keys
// Packs (cell key << idx_bits) | point index, or the key alone with the
// index in vals[] in pair mode; the cell's x coordinate is offset by the
// frame's place in the stacked grid, and points of a refused frame get the
// key of non-finite points (sorted last).  Each block takes one of the
// sort's tiles of kTile points, numbered as the sort numbers them, and also
// counts the first radix pass's digits of its words, stored as the sort's
// histogram kernel stores them (th[dg * pitch + tile]): the first pass then
// needs no histogram launch, nor a second read of the words.  Frames are
// consecutive ranges of the points: a lane finds the frame of its first
// point and walks on from there.
template <int RB>
__global__ __launch_bounds__(kBlock) void k_keys(const float *__restrict__ xyz,
                                                 const Params *__restrict__ P,
                                                 const Frame *__restrict__ frames, int nframes,
                                                 int64_t n, int64_t pitch,
                                                 uint64_t *__restrict__ keys,
                                                 uint32_t *__restrict__ vals,
                                                 uint32_t *__restrict__ th) {
    constexpr int R = 1 << RB, DPT = R / kBlock;
    if (P->status != kStatusOk) return;
    __shared__ uint32_t s_cnt[kBlock / 64][R];
    const int tid = threadIdx.x, wave = tid >> 6, lane = __lane_id();
    const int64_t tile = xcd_block_eighths();
    const int64_t base = tile * kTile + (int64_t)wave * (64 * kItems);
    for (int i = tid; i < (kBlock / 64) * R; i += kBlock) (&s_cnt[0][0])[i] = 0;
    const int ks = P->key_shift;
    const bool pair = P->pair_mode != 0;
    const int by = P->by, bz = P->bz;
    const uint64_t invalid_key = 1ull << (P->bx + by + bz);
    // the lane's frame: range end, acceptance, origin, scale, extent, x offset
    int f = 0;
    if (nframes > 1 && base + lane < n) f = frame_of_point(frames, nframes, base + lane);
    int64_t hi, NX, NY, NZ, xoff;
    double ox, oy, oz, inv;
    bool accepted;
    auto load_frame = [&]() {
        const Frame *F = frames + f;
        hi = F->off1;
        accepted = F->status == kStatusOk;
        ox = F->ox;
        oy = F->oy;
        oz = F->oz;
        inv = F->inv_s;
        NX = F->NX;
        NY = F->NY;
        NZ = F->NZ;
        xoff = F->xoff;
    };
    load_frame();
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kItems; ++k) {
        const int64_t e = base + k * 64 + lane;
        if (e < n) {
            while (e >= hi && f + 1 < nframes) {
                ++f;
                load_frame();
            }
            const float x = xyz[3 * e], y = xyz[3 * e + 1], z = xyz[3 * e + 2];
            uint64_t key;
            if (accepted && finite3(x, y, z)) {
                int64_t cx = (int64_t)floor(((double)x - ox) * inv);
                int64_t cy = (int64_t)floor(((double)y - oy) * inv);
                int64_t cz = (int64_t)floor(((double)z - oz) * inv);
                cx = cx < 0 ? 0 : (cx >= NX ? NX - 1 : cx);
                cy = cy < 0 ? 0 : (cy >= NY ? NY - 1 : cy);
                cz = cz < 0 ? 0 : (cz >= NZ ? NZ - 1 : cz);
                key = make_key((uint64_t)(xoff + cx), (uint64_t)cy, (uint64_t)cz, by, bz);
            } else {
                key = invalid_key;
            }
            const uint64_t word = pair ? key : ((key << ks) | (uint64_t)e);
            keys[e] = word;
            if (pair) vals[e] = (uint32_t)e;
            atomicAdd(&s_cnt[wave][(uint32_t)(word >> ks) & (R - 1)], 1u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        const int dg = q * kBlock + tid;
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) c += s_cnt[w][dg];
        th[(int64_t)dg * pitch + tile] = c;
    }
}

// ------------------------------------------------------------- 4. sort
// Stable LSD radix sort of the packed (key, index) words, RB bits per pass
// (RB from 8 to 11, a launch-time choice: fewer passes against larger
// per-tile tables; at 9, the passes beyond a key's first 36 bits take 10,
// see pass_width), reduce-then-scan: (1) each tile of kTile words counts
// its digits (the first pass's are counted by the keys kernel), (2) one
// block per digit turns the per-tile counts
// (digit-major) into the position of every tile's run of that digit,
// counted from the digit's first word, and the digit's total, (3) each tile
// ranks its words stably, stages them in LDS in digit order and writes each
// digit's run to its position.  Tiles are independent in every step.  The
// digits' global bases come from the per-digit totals of step (2), scanned
// by every scatter block, so no earlier kernel has to count digits over the
// whole array.  A thread owns R / kBlock consecutive digits where a step
// works per digit.

// Digit and stable in-wave rank of item k of this wave (lanes with equal
// digits are "peers"; the rank counts peers on lower lanes).
template <int RB>
__device__ __forceinline__ uint64_t digit_peers(uint32_t dg, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        const bool bit = (dg >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        peers &= bit ? bb : ~bb;
    }
    return peers;
}

// Exclusive scan over R values held DPT = R / kBlock per thread (thread t
// holds digits t*DPT .. t*DPT+DPT-1): v[] becomes the exclusive prefix of
// each; returns nothing, total in `total`.
template <int DPT>
__device__ __forceinline__ void block_excl_scan_multi(uint32_t (&v)[DPT], uint32_t *s_tmp,
                                                      uint32_t &total) {
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < DPT; ++q) sum += v[q];
    uint32_t run = block_excl_scan(sum, s_tmp, total);
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        const uint32_t x = v[q];
        v[q] = run;
        run += x;
    }
}

// (1) per-tile digit counts, stored digit-major: th[dg * pitch + tile].
template <int RB>
__global__ __launch_bounds__(kBlock) void k_sort_hist(const uint64_t *__restrict__ src,
                                                      const Params *__restrict__ P, int pass,
                                                      int bit0, int64_t n, int64_t pitch,
                                                      uint32_t *__restrict__ th) {
    constexpr int R = 1 << RB, DPT = R / kBlock;
    if (pass >= P->npasses || P->status != kStatusOk) return;
    __shared__ uint32_t s_cnt[kBlock / 64][R];
    const int tid = threadIdx.x, wave = tid >> 6, lane = __lane_id();
    // tiles by XCD eighths: neighbouring tiles write neighbouring words of
    // each digit's row of counts, which their XCD's L2 then merges into
    // whole lines (4-byte writes from tiles on different XCDs would each
    // cost a partial line in memory)
    const int64_t tile = xcd_block_eighths();
    const int shift = P->key_shift + bit0;
    const int64_t base = tile * kTile + (int64_t)wave * (64 * kItems);
    // the tile's words first, their loads overlapping the counters' reset
    uint64_t v[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t e = base + k * 64 + lane;
        v[k] = e < n ? src[e] : 0ull;
    }
    for (int i = tid; i < (kBlock / 64) * R; i += kBlock) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    // counts only (no ranks): one LDS atomic add per word, into the wave's
    // own row; lanes adding to one counter are serialised by the LDS, which
    // still costs far less than the ballots of a stable rank
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const bool valid = base + k * 64 + lane < n;
        const uint32_t dg = (uint32_t)(v[k] >> shift) & (R - 1);
        if (valid) atomicAdd(&s_cnt[wave][dg], 1u);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        const int dg = q * kBlock + tid;  // coalesced rows of th per q
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) c += s_cnt[w][dg];
        th[(int64_t)dg * pitch + tile] = c;
    }
}

// (2) one block per digit: exclusive scan of the digit's per-tile counts
// (positions relative to the digit's first word) and the digit's total,
// published for the scatter blocks, which add the digits' bases themselves.
// A thread takes kScanItems consecutive counts in 16-byte loads (rows start
// on 16-byte boundaries, the table's pitch is a multiple of 4), so a round
// covers 8,192 tiles (33.5 M words) and the map's table takes one.
constexpr int kScanItems = 32;
__global__ __launch_bounds__(kBlock) void k_sort_scan(const Params *__restrict__ P, int pass,
                                                      int64_t ntiles, int64_t pitch,
                                                      uint32_t *__restrict__ th,
                                                      uint32_t *__restrict__ dtot) {
    if (pass >= P->npasses || P->status != kStatusOk) return;
    __shared__ uint32_t s_tmp[kBlock / 64];
    __shared__ uint32_t s_carry;
    const int d = blockIdx.x, tid = threadIdx.x;
    uint32_t tot;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    uint32_t *row = th + (int64_t)d * pitch;
    for (int64_t c0 = 0; c0 < ntiles; c0 += (int64_t)kBlock * kScanItems) {
        // i0 is a multiple of 4: a group of 4 that starts below ntiles ends
        // within the row's pitch; counts past ntiles are taken as 0
        const int64_t i0 = c0 + (int64_t)tid * kScanItems;
        uint32_t v[kScanItems], sum = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; k += 4) {
            uint4 q = make_uint4(0u, 0u, 0u, 0u);
            if (i0 + k < ntiles) q = *reinterpret_cast<const uint4 *>(row + i0 + k);
            v[k] = q.x;
            v[k + 1] = i0 + k + 1 < ntiles ? q.y : 0u;
            v[k + 2] = i0 + k + 2 < ntiles ? q.z : 0u;
            v[k + 3] = i0 + k + 3 < ntiles ? q.w : 0u;
            sum += v[k] + v[k + 1] + v[k + 2] + v[k + 3];
        }
        const uint32_t carry = s_carry;
        __syncthreads();
        const uint32_t before = block_excl_scan(sum, s_tmp, tot);
        uint32_t run = carry + before;
#pragma unroll
        for (int k = 0; k < kScanItems; k += 4) {
            uint4 q;
            q.x = run;
            q.y = q.x + v[k];
            q.z = q.y + v[k + 1];
            q.w = q.z + v[k + 2];
            run = q.w + v[k + 3];
            // positions past ntiles land in the row's padding, read by no one
            if (i0 + k < ntiles) *reinterpret_cast<uint4 *>(row + i0 + k) = q;
        }
        __syncthreads();
        if (tid == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (tid == 0) dtot[(int64_t)pass * kMaxRadix + d] = s_carry;
}

// (3) stable scatter of one tile.
// Waves per SIMD: as many as the LDS allows blocks per CU (four at 8 and 9
// bits, three at 10, two at 11).  The per-wave digit counters are 16-bit
// (they never exceed the tile's 4,096 words), which takes 9-bit digits to
// 38 KB of LDS per block and four blocks per CU.
constexpr int scatter_waves(int rb) { return rb <= 9 ? 4 : (rb == 10 ? 3 : 2); }

template <int RB>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(scatter_waves(RB)))) void
k_sort_scatter(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst,
               const uint32_t *__restrict__ srcv, uint32_t *__restrict__ dstv,
               const Params *__restrict__ P, int pass, int bit0, int64_t n, int64_t pitch,
               const uint32_t *__restrict__ th, const uint32_t *__restrict__ dtot) {
    constexpr int R = 1 << RB, DPT = R / kBlock;
    if (pass >= P->npasses || P->status != kStatusOk) return;
    // s_cnt: per wave and digit, the count of the wave's words, then where
    // they go in the tile's LDS buffer; s_base: where the tile's run of each
    // digit goes in the output, then that minus the run's place in the
    // buffer (so buffer slot j goes to s_base[digit] + j)
    __shared__ uint16_t s_cnt[kBlock / 64][R];
    __shared__ uint32_t s_base[R];
    __shared__ uint64_t s_buf[kTile];  // keys in digit order (values after them in pair mode)
    __shared__ uint32_t s_tmp[kBlock / 64];
    const int tid = threadIdx.x, wave = tid >> 6, lane = __lane_id();
    for (int i = tid; i < (kBlock / 64) * R; i += kBlock) (&s_cnt[0][0])[i] = 0;
    // tiles by XCD eighths: neighbouring tiles read neighbouring words of
    // each digit's row of tile positions through one L2
    const int64_t tile = xcd_block_eighths();
    // the tile's words first: their loads overlap the digit bases below
    const int shift = P->key_shift + bit0;
    const bool pair = P->pair_mode != 0;
    const int64_t base = tile * kTile + (int64_t)wave * (64 * kItems);
    uint64_t v[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t e = base + k * 64 + lane;
        v[k] = e < n ? src[e] : 0ull;
    }
    {
        // this tile's position within each digit, plus the digit's base (the
        // totals of all smaller digits); thread t owns digits t*DPT ..
        uint32_t tv[DPT];
#pragma unroll
        for (int q = 0; q < DPT; ++q) tv[q] = dtot[(int64_t)pass * kMaxRadix + tid * DPT + q];
        uint32_t tot;
        block_excl_scan_multi<DPT>(tv, s_tmp, tot);
#pragma unroll
        for (int q = 0; q < DPT; ++q)
            s_base[tid * DPT + q] = tv[q] + th[(int64_t)(tid * DPT + q) * pitch + tile];
    }
    __syncthreads();
    uint32_t rk[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const bool valid = base + k * 64 + lane < n;
        const uint32_t dg = (uint32_t)(v[k] >> shift) & (R - 1);
        const uint64_t peers = digit_peers<RB>(dg, valid);
        const uint32_t below = (uint32_t)__popcll(peers & lanemask_lt());
        const uint32_t prev = s_cnt[wave][dg];
        rk[k] = prev + below;
        if (valid && below == 0) s_cnt[wave][dg] = (uint16_t)(prev + (uint32_t)__popcll(peers));
    }
    __syncthreads();
    {
        // per digit: wave offsets inside the tile, then the tile's exclusive
        // scan over digits (where each digit's run starts in the tile),
        // folded into the wave offsets and the output base
        uint32_t tv[DPT];
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            const int dg = tid * DPT + q;
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) {
                const uint32_t c = s_cnt[w][dg];
                s_cnt[w][dg] = (uint16_t)run;
                run += c;
            }
            tv[q] = run;
        }
        uint32_t tot;
        block_excl_scan_multi<DPT>(tv, s_tmp, tot);
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            const int dg = tid * DPT + q;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) s_cnt[w][dg] = (uint16_t)(s_cnt[w][dg] + tv[q]);
            s_base[dg] -= tv[q];  // modulo 2^32; adding the slot restores it
        }
    }
    __syncthreads();
    // stage the tile in LDS in digit order, then write each digit's run
    // contiguously; in pair mode the values follow through the same buffer
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t e = base + k * 64 + lane;
        if (e < n) {
            const uint32_t dg = (uint32_t)(v[k] >> shift) & (R - 1);
            s_buf[s_cnt[wave][dg] + rk[k]] = v[k];
        }
    }
    __syncthreads();
    const int64_t rem = n - tile * kTile;
    const int tile_n = rem < kTile ? (int)rem : kTile;
    uint32_t pos[kItems];  // n < 2^31
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int j = tid + i * kBlock;
        pos[i] = 0xFFFFFFFFu;
        if (j < tile_n) {
            const uint64_t w = s_buf[j];
            const uint32_t dg = (uint32_t)(w >> shift) & (R - 1);
            const uint64_t p = (uint64_t)(uint32_t)(s_base[dg] + (uint32_t)j);
            if (p < (uint64_t)n) {
                pos[i] = (uint32_t)p;
                dst[p] = w;
            }
        }
    }
    if (pair) {
        uint32_t *s_vbuf = reinterpret_cast<uint32_t *>(s_buf);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int64_t e = base + k * 64 + lane;
            if (e < n) {
                const uint32_t dg = (uint32_t)(v[k] >> shift) & (R - 1);
                s_vbuf[s_cnt[wave][dg] + rk[k]] = srcv[e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int j = tid + i * kBlock;
            if (pos[i] != 0xFFFFFFFFu) dstv[pos[i]] = s_vbuf[j];
        }
    }
}

// ------------------------------------------------------------- 5. gather
// Sorted words: key = word >> key_shift; index = low bits (one-word mode)
// or the parallel index array (pair mode).
__device__ __forceinline__ bool cell_flag(const uint64_t *srt, int64_t e, int ks,
                                          uint64_t &key) {
    const uint64_t v = srt[e];
    key = v >> ks;
    return e == 0 || (srt[e - 1] >> ks) != key;
}

// Points in sorted order (x, y, z, original index bits), original indices,
// and per-tile counts of cell and column starts.
__global__ __launch_bounds__(kBlock) void k_gather(const float *__restrict__ xyz,
                                                   const uint64_t *__restrict__ s0,
                                                   const uint64_t *__restrict__ s1,
                                                   const uint32_t *__restrict__ v0,
                                                   const uint32_t *__restrict__ v1,
                                                   uint32_t *__restrict__ colbits,
                                                   Params *__restrict__ P,
                                                   float4 *__restrict__ spts,
                                                   uint32_t *__restrict__ sorig,
                                                   uint32_t *__restrict__ tile_cnt) {
    if (P->status != kStatusOk) return;
    const uint64_t *srt = (P->npasses & 1) ? s1 : s0;
    const uint32_t *sv = (P->npasses & 1) ? v1 : v0;
    const int64_t n = P->n, nvalid = P->nvalid;
    const int ks = P->key_shift, bz = P->bz;
    const bool pair = P->pair_mode != 0;
    const uint64_t mask = P->idx_mask;
    // each XCD gathers one contiguous eighth of the sorted order: tiles next
    // to each other share lines of the input (points of one scan line that
    // fall in neighbouring cells), which one L2 then serves (map gather
    // 0.54 -> 0.45 ms; 128-tile runs: 0.46 ms)
    const int64_t tile = xcd_block_eighths();
    const int64_t base = tile * kTile;
    if (P->dense_cols) {  // clear the column occupancy bits
        const uint64_t words = ((uint64_t)P->NX * (uint64_t)P->NYp) / 32;
        for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < words;
             i += (uint64_t)gridDim.x * kBlock)
            colbits[i] = 0;
    }
    uint32_t nc = 0, ncol = 0;
#pragma unroll 4
    for (int k = 0; k < kItems; ++k) {
        const int64_t e = base + k * kBlock + threadIdx.x;
        if (e < n) {
            const uint64_t v = srt[e];
            uint32_t i = pair ? sv[e] : (uint32_t)(v & mask);
            if (i >= (uint64_t)n) {  // cannot happen for a correct sort; never read out of range
                atomicExch(&P->status, kStatusDevice);
                i = 0;
            }
            const float x = xyz[3 * (size_t)i], y = xyz[3 * (size_t)i + 1],
                        z = xyz[3 * (size_t)i + 2];
            // streaming writes past the caches, which keep the input's
            // lines for the neighbouring tiles' reads (map gather 0.446 ->
            // 0.425 ms; the same in the sort's scatter or the key kernel
            // was slower or no faster)
            typedef float f4v __attribute__((ext_vector_type(4)));
            const f4v pv = {x, y, z, __uint_as_float(i)};
            __builtin_nontemporal_store(pv, reinterpret_cast<f4v *>(&spts[e]));
            __builtin_nontemporal_store(i, &sorig[e]);
            if (e < nvalid) {
                const uint64_t key = v >> ks;
                const uint64_t pk = e > 0 ? (srt[e - 1] >> ks) : ~0ull;
                if (e == 0 || pk != key) {
                    ++nc;
                    if (e == 0 || (pk >> bz) != (key >> bz)) ++ncol;
                }
            }
        }
    }
    __shared__ uint32_t s_tmp[kBlock / 64];
    uint32_t t1, t2;
    block_excl_scan(nc, s_tmp, t1);
    __syncthreads();
    block_excl_scan(ncol, s_tmp, t2);
    if (threadIdx.x == 0) {
        tile_cnt[2 * tile] = t1;
        tile_cnt[2 * tile + 1] = t2;
    }
}

// ------------------------------------------------------------- 6. tile scan
// Exclusive scan of the per-tile counts of cell and column starts (one
// block).
__global__ __launch_bounds__(1024) void k_tile_scan(const uint32_t *__restrict__ tile_cnt,
                                                    uint32_t *__restrict__ tile_off,
                                                    int64_t ntiles, Params *__restrict__ P) {
    if (P->status != kStatusOk) return;
    __shared__ uint32_t s_v[2][1024];
    const int tid = threadIdx.x;
    const int64_t per = (ntiles + 1023) / 1024;
    const int64_t lo = tid * per, hi = lo + per < ntiles ? lo + per : ntiles;
    uint32_t own[2] = {0, 0};
    for (int64_t t = lo; t < hi; ++t)
        for (int c = 0; c < 2; ++c) own[c] += tile_cnt[2 * t + c];
    for (int c = 0; c < 2; ++c) s_v[c][tid] = own[c];
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t x[2];
        for (int c = 0; c < 2; ++c) x[c] = tid >= o ? s_v[c][tid - o] : 0u;
        __syncthreads();
        for (int c = 0; c < 2; ++c) s_v[c][tid] += x[c];
        __syncthreads();
    }
    uint32_t run[2];
    for (int c = 0; c < 2; ++c) run[c] = s_v[c][tid] - own[c];
    for (int64_t t = lo; t < hi; ++t)
        for (int c = 0; c < 2; ++c) {
            tile_off[2 * t + c] = run[c];
            run[c] += tile_cnt[2 * t + c];
        }
    if (tid == 1023) {
        const uint32_t M = s_v[0][1023], Mc = s_v[1][1023];
        P->M = M;
        P->Mcol = Mc;
        if ((int64_t)M > P->nvalid || Mc > M) {
            P->status = kStatusDevice;  // inconsistent counts: stop before any table use
            P->M = 0;
            P->Mcol = 0;
        }
        // no dense index: hash the columns when key and cell fit one slot
        // and the table stays at most half full
        if (!P->dense_cols && P->bx + P->by <= 33) {
            uint64_t slots = 1024;
            while (slots < 4ull * Mc) slots *= 2;
            if (slots > P->hcap) slots = P->hcap;
            if (2ull * Mc <= slots) {
                int lg = 0;
                while ((1ull << lg) < slots) ++lg;
                P->hashed_cols = 1;
                P->hmask = slots - 1;
                P->hshift = 64 - lg;
            }
        }
    }
}

// Frame whose stacked x range holds cell column cx: the last frame with
// xoff <= cx (frames are stacked in order, so xoff increases).
__device__ __forceinline__ int frame_of_x(const Frame *frames, int nframes, int64_t cx) {
    int lo = 0, hi = nframes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (frames[mid].xoff <= cx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Column hash slots: column key << 31 | first cell; all ones = empty.
constexpr uint64_t kHashEmpty = ~0ull;

__device__ __forceinline__ uint64_t col_hash(uint64_t ck, int shift) {
    return (ck * 0x9E3779B97F4A7C15ull) >> shift;
}

// ------------------------------------------------------------- 7. cells
// Cell table (first sorted position and key of every occupied cell) and
// column table (key and first cell of every occupied column (cx, cy)), plus
// the per-cell union-find / size / id slots.
__global__ __launch_bounds__(kBlock) void k_cells(const uint64_t *__restrict__ s0,
                                                  const uint64_t *__restrict__ s1,
                                                  const Params *__restrict__ P,
                                                  const uint32_t *__restrict__ tile_off,
                                                  uint32_t *__restrict__ cell_start,
                                                  uint64_t *__restrict__ cell_key,
                                                  uint64_t *__restrict__ col_key,
                                                  uint32_t *__restrict__ col_cell,
                                                  int32_t *__restrict__ cpar,
                                                  uint32_t *__restrict__ csize,
                                                  uint32_t *__restrict__ ccanon,
                                                  Frame *__restrict__ frames,
                                                  uint32_t *__restrict__ cell_frame,
                                                  uint64_t *__restrict__ hslots) {
    if (P->status != kStatusOk) return;
    const uint64_t *srt = (P->npasses & 1) ? s1 : s0;
    const int64_t nvalid = P->nvalid;
    const int ks = P->key_shift, bz = P->bz, xshift = P->by + P->bz;
    const int nframes = P->nframes;
    if (P->hashed_cols) {  // empty every slot of the column hash (filled by k_colgrid)
        const uint64_t slots = P->hmask + 1;
        for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < slots;
             i += (uint64_t)gridDim.x * kBlock)
            hslots[i] = kHashEmpty;
    }
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int wave = threadIdx.x >> 6, lane = __lane_id();
    __shared__ uint32_t s_tot[2][kItems][kBlock / 64];
    uint32_t flags = 0, cflags = 0;
    for (int k = 0; k < kItems; ++k) {
        const int64_t e = base + k * kBlock + threadIdx.x;
        uint64_t key = 0;
        const bool f = e < nvalid && cell_flag(srt, e, ks, key);
        const bool cf = f && (e == 0 || ((srt[e - 1] >> ks) >> bz) != (key >> bz));
        flags |= (uint32_t)f << k;
        cflags |= (uint32_t)cf << k;
        const uint64_t m = __ballot(f), mc = __ballot(cf);
        if (lane == 0) {
            s_tot[0][k][wave] = (uint32_t)__popcll(m);
            s_tot[1][k][wave] = (uint32_t)__popcll(mc);
        }
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint32_t run = 0;
        for (int k = 0; k < kItems; ++k)
            for (int w = 0; w < kBlock / 64; ++w) {
                const uint32_t t = s_tot[threadIdx.x][k][w];
                s_tot[threadIdx.x][k][w] = run;
                run += t;
            }
    }
    __syncthreads();
    const uint32_t c0 = tile_off[2 * blockIdx.x], q0 = tile_off[2 * blockIdx.x + 1];
    const uint64_t lt = lanemask_lt();
    for (int k = 0; k < kItems; ++k) {
        const bool f = (flags >> k) & 1u, cf = (cflags >> k) & 1u;
        const uint64_t m = __ballot(f), mc = __ballot(cf);
        if (f) {
            const int64_t e = base + k * kBlock + threadIdx.x;
            const uint32_t cid = c0 + s_tot[0][k][wave] + (uint32_t)__popcll(m & lt);
            const uint32_t colx = q0 + s_tot[1][k][wave] + (uint32_t)__popcll(mc & lt);
            if ((int64_t)cid >= nvalid) continue;
            const uint64_t key = srt[e] >> ks;
            cell_start[cid] = (uint32_t)e;
            cell_key[cid] = key;
            cpar[cid] = (int32_t)cid;
            csize[cid] = 0;
            ccanon[cid] = 0xFFFFFFFFu;
            if (cf) {
                col_key[colx] = key >> bz;
                col_cell[colx] = cid;
            }
            if (nframes > 1) {  // the cell's frame; the frame's first cell
                const int64_t cx = (int64_t)(key >> xshift);
                const int fr = frame_of_x(frames, nframes, cx);
                cell_frame[cid] = (uint32_t)fr;
                if (cid == 0 || (int64_t)((srt[e - 1] >> ks) >> xshift) < frames[fr].xoff)
                    frames[fr].cell0 = cid;
            }
        }
    }
}

// Column coordinates <-> column key (see make_key).
struct Grid {
    int by, bz;
    int64_t NX, NY, NYp;
    uint64_t zmask, ymask;

    __device__ __forceinline__ uint64_t col_key(uint64_t cx, uint64_t cy) const {
        return (cx << by) | cy;
    }
    __device__ __forceinline__ void col_xy(uint64_t ck, int64_t &cx, int64_t &cy) const {
        cx = (int64_t)(ck >> by);
        cy = (int64_t)(ck & ymask);
    }
};

__device__ __forceinline__ Grid grid_of(const Params *P) {
    Grid g;
    g.by = P->by;
    g.bz = P->bz;
    g.NX = P->NX;
    g.NY = P->NY;
    g.NYp = P->NYp;
    g.zmask = (1ull << P->bz) - 1;
    g.ymask = (1ull << P->by) - 1;
    return g;
}

// Dense column index: colgrid[cx * NYp + cy] = first cell of column
// (cx, cy), valid where the occupancy bit is set (bits are cleared every
// call, the index itself is not).  Also writes the end markers of the cell and column
// tables.
__global__ __launch_bounds__(kBlock) void k_colgrid(const uint64_t *__restrict__ col_key,
                                                    uint32_t *__restrict__ col_cell,
                                                    uint32_t *__restrict__ cell_start,
                                                    uint32_t *__restrict__ colgrid,
                                                    uint32_t *__restrict__ colbits,
                                                    const Params *__restrict__ P) {
    if (P->status != kStatusOk) return;
    const int64_t Mcol = P->Mcol;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        col_cell[Mcol] = (uint32_t)P->M;
        cell_start[P->M] = (uint32_t)P->nvalid;
    }
    if (P->hashed_cols) {
        // column keys are distinct, so each insert claims one empty slot; the
        // table has more slots than columns, so every probe sequence ends
        uint64_t *hs = reinterpret_cast<uint64_t *>(colgrid);
        const uint64_t mask = P->hmask;
        const int shift = P->hshift;
        for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < Mcol;
             c += (int64_t)gridDim.x * kBlock) {
            const uint64_t ck = col_key[c];
            const uint64_t v = (ck << 31) | (uint64_t)col_cell[c];
            uint64_t h = col_hash(ck, shift);
            for (uint64_t probe = 0; probe <= mask; ++probe) {
                if (atomicCAS((unsigned long long *)(hs + h), (unsigned long long)kHashEmpty,
                              (unsigned long long)v) == kHashEmpty)
                    break;
                h = (h + 1) & mask;
            }
        }
        return;
    }
    if (!P->dense_cols) return;
    const Grid g = grid_of(P);
    const int lane = __lane_id();
    for (int64_t c0 = (int64_t)blockIdx.x * kBlock; c0 < Mcol; c0 += (int64_t)gridDim.x * kBlock) {
        const int64_t c = c0 + threadIdx.x;
        const bool valid = c < Mcol;
        uint64_t idx = 0;
        if (valid) {
            int64_t cx, cy;
            g.col_xy(col_key[c], cx, cy);
            idx = (uint64_t)(cx * g.NYp + cy);
            colgrid[idx] = col_cell[c];
        }
        // columns are sorted, so a wave's bits fall into few words: one
        // atomic OR per distinct word
        uint64_t act = __ballot(valid);
        while (act) {
            const int l = first_lane(act);
            const uint64_t w0 = __shfl(idx >> 5, l);
            const bool mine = valid && (idx >> 5) == w0;
            const uint64_t grp = __ballot(mine);
            uint32_t bits = mine ? (1u << (idx & 31)) : 0u;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) bits |= __shfl_xor(bits, o);
            if (lane == l) atomicOr(&colbits[w0], bits);
            act &= ~grp;
        }
    }
}

// Column index in use: dense table, hash table, or binary search over the
// sorted column keys.
struct ColIndex {
    int mode;  // kColDense, kColHash, kColSearch
    const uint32_t *colgrid, *colbits;
    const uint64_t *hs;
    uint64_t hmask;
    int hshift;
    const uint64_t *col_key;
    const uint32_t *col_cell;
    int64_t Mcol;
};
constexpr int kColSearch = 0, kColDense = 1, kColHash = 2;

__device__ __forceinline__ ColIndex colindex_of(const Params *P, const uint32_t *colgrid,
                                                const uint32_t *colbits,
                                                const uint64_t *col_key,
                                                const uint32_t *col_cell) {
    ColIndex c;
    c.mode = P->dense_cols ? kColDense : (P->hashed_cols ? kColHash : kColSearch);
    c.colgrid = colgrid;
    c.colbits = colbits;
    c.hs = reinterpret_cast<const uint64_t *>(colgrid);
    c.hmask = P->hmask;
    c.hshift = P->hshift;
    c.col_key = col_key;
    c.col_cell = col_cell;
    c.Mcol = P->Mcol;
    return c;
}

// Continues a hash probe sequence from slot h holding v until the column's
// slot or an empty one.
__device__ __forceinline__ bool hash_resolve(const ColIndex &ci, uint64_t want, uint64_t h,
                                             uint64_t v, uint32_t &first) {
    for (uint64_t probe = 0; probe <= ci.hmask; ++probe) {
        if (v == kHashEmpty) return false;
        if ((v >> 31) == want) {
            first = (uint32_t)(v & 0x7FFFFFFFu);
            return true;
        }
        h = (h + 1) & ci.hmask;
        v = ci.hs[h];
    }
    return false;
}

// Several column lookups with their first memory access issued together:
// has[o] / first[o] for columns (nx[o], ny[o]), o < K.
template <int K>
__device__ __forceinline__ void find_columns(const Grid &g, const ColIndex &ci,
                                             const int64_t (&nx)[K], const int64_t (&ny)[K],
                                             bool (&has)[K], uint32_t (&first)[K]) {
    bool in[K];
#pragma unroll
    for (int o = 0; o < K; ++o) in[o] = nx[o] >= 0 && nx[o] < g.NX && ny[o] >= 0 && ny[o] < g.NY;
    if (ci.mode == kColDense) {
#pragma unroll
        for (int o = 0; o < K; ++o) {
            const uint64_t idx = in[o] ? (uint64_t)(nx[o] * g.NYp + ny[o]) : 0;
            const uint32_t wd = in[o] ? ci.colbits[idx >> 5] : 0u;
            first[o] = in[o] ? ci.colgrid[idx] : 0u;
            has[o] = (wd >> (idx & 31)) & 1u;
        }
    } else if (ci.mode == kColHash) {
        uint64_t h[K], v[K], want[K];
#pragma unroll
        for (int o = 0; o < K; ++o) {
            want[o] = g.col_key((uint64_t)nx[o], (uint64_t)ny[o]);
            h[o] = col_hash(want[o], ci.hshift);
            v[o] = in[o] ? ci.hs[h[o]] : kHashEmpty;
        }
#pragma unroll
        for (int o = 0; o < K; ++o) {
            first[o] = 0;
            has[o] = in[o] && hash_resolve(ci, want[o], h[o], v[o], first[o]);
        }
    } else {
#pragma unroll
        for (int o = 0; o < K; ++o) {
            has[o] = false;
            first[o] = 0;
            if (!in[o]) continue;
            const uint64_t want = g.col_key((uint64_t)nx[o], (uint64_t)ny[o]);
            int64_t lo = 0, hi = ci.Mcol;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (ci.col_key[mid] < want) lo = mid + 1;
                else hi = mid;
            }
            if (lo < ci.Mcol && ci.col_key[lo] == want) {
                has[o] = true;
                first[o] = ci.col_cell[lo];
            }
        }
    }
}

// ------------------------------------------------------------- 8. hooking
// Run lengths C of the two hooking kernels, measured on the 27 M map against
// C = 1 (near shell 2.34 -> 2.10 ms with three cells loaded per column, far
// shell 1.04 -> 0.98 ms with groups of 8 columns; with one cell per column,
// C = 128 for the near shell measures 1.68 -> 1.63 ms against C = 64, and
// the far shell is the same for C from 8 to 64), batches of frames
// unchanged.  Whole eighths per XCD (C = gridDim.x / 8) unbalance both
// shells on batches (near 0.44 -> 0.64 ms).  The kernels over a work list
// (far shell, near shell after the sampling links) take kXcdRunFar: with
// the lists in cell order, C = 64 is best on the map (far shell 0.477 ->
// 0.460 ms against 16; 32 and 128 in between), batches unchanged.
constexpr uint32_t kXcdRunNear = 128;
constexpr uint32_t kXcdRunFar = 64;

// Union-find over cells.  Two roots are joined by hooking the one of higher
// rank under the other, rank being a fixed bijective scramble of the cell
// id: a strict total order keeps the forest acyclic under concurrent hooks,
// and a scrambled one keeps trees shallow when components are chained in
// id order (a ground strip crossing many tiles), where hooking by id builds
// one long path.  Which cell ends up the root does not matter: labels come
// from the smallest point index of each component, computed separately.
//
// Parents are read with plain (L2-cached) loads.  The L2s of the XCDs are
// not coherent with each other inside a kernel, so a read may return an
// older parent; every older parent is still an ancestor in the same
// component, which is all the algorithm needs: "same root" answers are
// always right, "different roots" answers may be stale and cost one extra
// pair test.  Only the compare-and-swap that hooks a root is coherent, and
// when it fails the parent it returns (fresh) is where the search resumes,
// so every retry moves strictly up the tree and the loop ends.
__device__ __forceinline__ int32_t uf_find(const int32_t *par, int32_t x) {
    int32_t p = par[x];
    while (p != x) {
        x = p;
        p = par[x];
    }
    return x;
}

__device__ __forceinline__ uint32_t uf_rank(int32_t x) {
    uint32_t h = (uint32_t)x * 0x9E3779B1u;  // odd multiplier, xor-shifts: bijective
    h ^= h >> 15;
    h *= 0x85EBCA77u;
    h ^= h >> 13;
    return h;
}

// Joins the components of a and b; returns a root of the union (at the
// time of the join).
__device__ __forceinline__ int32_t uf_link(int32_t *par, int32_t a, int32_t b) {
    a = uf_find(par, a);
    b = uf_find(par, b);
    while (a != b) {
        const bool ah = uf_rank(a) > uf_rank(b);
        const int32_t hi = ah ? a : b, lo = ah ? b : a;
        // hook the root of higher rank under the other
        const int32_t old = atomicCAS(par + hi, hi, lo);
        if (old == hi) return lo;
        // hi was hooked meanwhile: continue from its current parent
        if (hi == a) {
            a = uf_find(par, old);
        } else {
            b = uf_find(par, old);
        }
    }
    return a;
}

// Joins two components whose roots were just read: one CAS when both are
// still roots, the general loop otherwise.  Returns the root of the union.
__device__ __forceinline__ int32_t uf_link_roots(int32_t *par, int32_t a, int32_t b) {
    if (a == b) return a;
    const bool ah = uf_rank(a) > uf_rank(b);
    const int32_t hi = ah ? a : b, lo = ah ? b : a;
    const int32_t old = atomicCAS(par + hi, hi, lo);
    if (old == hi) return lo;
    return uf_link(par, old, lo);
}

// Is there a joined pair between the points [sA, eA) and [sB, eB)?  Stops at
// the first one.
// Point by point: for pairs of small cells that are usually joined at the
// first pair.
__device__ __forceinline__ bool any_joined_1(const float4 *__restrict__ spts, uint32_t sA,
                                             uint32_t eA, uint32_t sB, uint32_t eB, float d2) {
    for (uint32_t a = sA; a < eA; ++a) {
        const float4 pa = spts[a];
        for (uint32_t b = sB; b < eB; ++b)
            if (joined(pa.x, pa.y, pa.z, spts[b], d2)) return true;
    }
    return false;
}

// The points of B are read four at a time (independent loads in flight
// together); an index past the end re-reads B's last point, which changes
// nothing.
//
// Pairs of large cells that are not joined at once (cells across an empty
// gap, the two sides of a thin wall) would cost |A| x |B| tests in one lane.
// After two rows, the bounding box of B's points is taken, and a point a of
// A is skipped when its binary32 distance to that box already fails the
// predicate.  The box test is exact, not a heuristic: with gx = fl(lo_x -
// a_x) (or fl(a_x - hi_x), or 0 inside), every b has |fl(a_x - b_x)| >= gx,
// because rounding is monotone and lo_x, hi_x are coordinates of points of
// B; the squares and the two sums are monotone too, so every pair's computed
// s is at least the box's, and a box value >= fl(d*d) rules out every pair.
__device__ __forceinline__ bool any_joined_row(const float4 &pa, const float4 *__restrict__ spts,
                                               uint32_t sB, uint32_t eB, float d2) {
    for (uint32_t b = sB; b < eB; b += 4) {
        float4 q[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) q[j] = spts[b + j < eB ? b + j : eB - 1];
        bool hit = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) hit |= joined(pa.x, pa.y, pa.z, q[j], d2);
        if (hit) return true;
    }
    return false;
}

__device__ __forceinline__ bool any_joined(const float4 *__restrict__ spts, uint32_t sA,
                                           uint32_t eA, uint32_t sB, uint32_t eB, float d2) {
#pragma clang fp contract(off)
    const uint32_t plain = (eA - sA) * (eB - sB) <= 64 ? eA : (sA + 2 < eA ? sA + 2 : eA);
    uint32_t a = sA;
    for (; a < plain; ++a)
        if (any_joined_row(spts[a], spts, sB, eB, d2)) return true;
    if (a >= eA) return false;
    float lx = INFINITY, ly = INFINITY, lz = INFINITY;
    float hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
    for (uint32_t b = sB; b < eB; b += 4) {
        float4 q[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) q[j] = spts[b + j < eB ? b + j : eB - 1];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            lx = fminf(lx, q[j].x); ly = fminf(ly, q[j].y); lz = fminf(lz, q[j].z);
            hx = fmaxf(hx, q[j].x); hy = fmaxf(hy, q[j].y); hz = fmaxf(hz, q[j].z);
        }
    }
    for (; a < eA; ++a) {
        const float4 pa = spts[a];
        const float gx = fmaxf(fmaxf(lx - pa.x, pa.x - hx), 0.0f);
        const float gy = fmaxf(fmaxf(ly - pa.y, pa.y - hy), 0.0f);
        const float gz = fmaxf(fmaxf(lz - pa.z, pa.z - hz), 0.0f);
        float sb = gx * gx + gy * gy;
        sb = sb + gz * gz;
        if (!(sb < d2)) continue;
        if (any_joined_row(pa, spts, sB, eB, d2)) return true;
    }
    return false;
}

// A queued cell pair (A << 32 | B): joined unless already in one component,
// tested point pair by point pair.
__device__ __forceinline__ void defer_test(uint64_t e, const float4 *__restrict__ spts,
                                           const uint32_t *__restrict__ cell_start,
                                           int32_t *cpar, float d2) {
    const int32_t A = (int32_t)(e >> 32), B = (int32_t)(e & 0xFFFFFFFFu);
    const int32_t ra = uf_find(cpar, A), rb = uf_find(cpar, B);
    if (ra == rb) return;
    if (any_joined(spts, cell_start[A], cell_start[A + 1], cell_start[B], cell_start[B + 1], d2))
        uf_link(cpar, ra, rb);
}

// Runs: cell B = A + 1 (the next cell in key order) is often A's neighbour
// one step up in z, or one step along y in the next column.  Such a pair's
// first points are tested; each cell not joined to its predecessor this way
// starts a run.  Every cell of a run is connected to the run's first cell,
// which becomes its parent: a valid union-find state (parent <= cell, same
// component) reached without atomics.  A pair whose first points are not
// joined is queued and tested in full after the near shell (a full scan in
// the runs pass held up its wave, and by then most such pairs share a root).
__device__ __forceinline__ bool next_is_near(const Grid &g, uint64_t ka, uint64_t kb) {
    const uint64_t ca = ka >> g.bz, cb = kb >> g.bz;
    const int64_t za = (int64_t)(ka & g.zmask), zb = (int64_t)(kb & g.zmask);
    if (ca == cb) return zb == za + 1;
    int64_t xa, ya, xb, yb;
    g.col_xy(ca, xa, ya);
    g.col_xy(cb, xb, yb);
    return xb == xa && yb == ya + 1 && zb - za >= -1 && zb - za <= 1;
}

// Pass 1: run-start flags per cell, and the last run start of every block
// of kTile cells.
__global__ __launch_bounds__(kBlock) void k_runs1(const float4 *__restrict__ spts,
                                                  const uint32_t *__restrict__ cell_start,
                                                  const uint64_t *__restrict__ cell_key,
                                                  uint8_t *__restrict__ heads,
                                                  int32_t *__restrict__ blkhead,
                                                  uint32_t *__restrict__ runq,
                                                  const Frame *__restrict__ frames,
                                                  const uint32_t *__restrict__ cell_frame,
                                                  Params *__restrict__ P) {
    if (P->status != kStatusOk) return;
    const int64_t M = P->M;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    if (base >= M) return;
    const float d2_one = P->d2;
    const bool batched = P->nframes > 1;
    const Grid g = grid_of(P);
    int32_t last = -1;
    uint32_t qbits = 0;  // bit k: the pair ending at the thread's k-th cell is queued
    static_assert(kItems <= 32, "queue flags are 32-bit");
    // kR cells per lane at a time, their loads issued in rounds (keys; cell
    // starts and thresholds; the first point of both cells), so that a lane
    // does not wait on one chain of dependent loads per cell in turn
    constexpr int kR = 4;
    static_assert(kItems % kR == 0, "rounds cover the tile");
    for (int k0 = 0; k0 < kItems; k0 += kR) {
        int64_t A[kR];
        bool in[kR], nr[kR];
        uint64_t kp[kR], ka[kR];
        uint32_t fr[kR];
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            A[u] = base + (k0 + u) * kBlock + threadIdx.x;
            in[u] = A[u] < M;
            ka[u] = in[u] ? cell_key[A[u]] : 0ull;
            kp[u] = (in[u] && A[u] > 0) ? cell_key[A[u] - 1] : 0ull;
            fr[u] = (in[u] && batched) ? cell_frame[A[u]] : 0u;
        }
        uint32_t s0[kR], s1[kR], s2[kR];
        float d2[kR];
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            nr[u] = in[u] && A[u] > 0 && next_is_near(g, kp[u], ka[u]);  // same x: same frame
            s0[u] = nr[u] ? cell_start[A[u] - 1] : 0u;
            s1[u] = nr[u] ? cell_start[A[u]] : 0u;
            s2[u] = nr[u] ? cell_start[A[u] + 1] : 0u;
            d2[u] = (nr[u] && batched) ? frames[fr[u]].d2 : d2_one;
        }
        float4 pa[kR], pb[kR];
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            pa[u] = nr[u] ? spts[s0[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
            pb[u] = nr[u] ? spts[s1[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            if (!in[u]) continue;
            bool head = true;
            if (nr[u]) {
                head = !joined(pa[u].x, pa[u].y, pa[u].z, pb[u], d2[u]);
                if (head) qbits |= 1u << (k0 + u);
            }
            heads[A[u]] = head ? 1 : 0;
            if (head) last = (int32_t)A[u];
        }
    }
    // the queued pairs: one reservation per block
    {
        __shared__ uint32_t s_tmp[kBlock / 64];
        __shared__ uint32_t s_qbase;
        uint32_t tot;
        const uint32_t off = block_excl_scan((uint32_t)__popc(qbits), s_tmp, tot);
        if (threadIdx.x == 0) s_qbase = tot ? atomicAdd(&P->nrunq, tot) : 0u;
        __syncthreads();
        uint32_t o = s_qbase + off;
        for (uint32_t q = qbits; q; q &= q - 1u) {
            const int k = __ffs(q) - 1;
            runq[o++] = (uint32_t)(base + k * kBlock + threadIdx.x);
        }
    }
    // block max of the last run start
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t w = __shfl_xor(last, o);
        last = w > last ? w : last;
    }
    __shared__ int32_t s_w[kBlock / 64];
    if (__lane_id() == 0) s_w[threadIdx.x >> 6] = last;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t m = -1;
        for (int w = 0; w < kBlock / 64; ++w) m = s_w[w] > m ? s_w[w] : m;
        blkhead[blockIdx.x] = m;
    }
}

// Pass 2: parent of every cell = the last run start at or before it.
__global__ __launch_bounds__(kBlock) void k_runs2(const uint8_t *__restrict__ heads,
                                                  const int32_t *__restrict__ blkhead,
                                                  int32_t *__restrict__ cpar,
                                                  const Params *__restrict__ P) {
    if (P->status != kStatusOk) return;
    const int64_t M = P->M;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    if (base >= M) return;
    const int wave = threadIdx.x >> 6, lane = __lane_id();
    __shared__ int32_t s_last[kItems][kBlock / 64];
    __shared__ int32_t s_carry[kItems][kBlock / 64];
    uint32_t hf = 0;
    for (int k = 0; k < kItems; ++k) {
        const int64_t A = base + k * kBlock + threadIdx.x;
        const bool h = A < M && heads[A];
        hf |= (uint32_t)h << k;
        const uint64_t m = __ballot(h);
        if (lane == 0) s_last[k][wave] = m ? (int32_t)(base + k * kBlock + wave * 64 + 63 - __clzll(m)) : -1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // run start before this block: nearest earlier block that has one
        int32_t carry = 0;
        for (int64_t b = (int64_t)blockIdx.x - 1; b >= 0; --b) {
            const int32_t h = blkhead[b];
            if (h >= 0) {
                carry = h;
                break;
            }
        }
        for (int k = 0; k < kItems; ++k)
            for (int w = 0; w < kBlock / 64; ++w) {
                s_carry[k][w] = carry;
                if (s_last[k][w] >= 0) carry = s_last[k][w];
            }
    }
    __syncthreads();
    for (int k = 0; k < kItems; ++k) {
        const int64_t A = base + k * kBlock + threadIdx.x;
        const uint64_t m = __ballot((hf >> k) & 1u);
        if (A >= M) continue;
        const uint64_t upto = m & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
        const int32_t p = upto ? (int32_t)(base + k * kBlock + wave * 64 + 63 - __clzll(upto))
                               : s_carry[k][wave];
        cpar[A] = p;
    }
}

// Position of the first cell of column `want` with z >= zt, or of the cell
// after the column when it has none, given the column's first cell fc (its z
// is z0 < zt) and a position lo <= the answer.  The cells of a column have
// distinct, increasing z, so the answer is at most fc + (zt - z0); a column
// without gaps has it exactly there, which is tried first.  Otherwise a
// binary search over the sorted cell keys.
__device__ __forceinline__ uint32_t column_seek(const uint64_t *__restrict__ cell_key, int64_t M,
                                                int bz, uint64_t want, uint32_t fc, int64_t z0,
                                                uint32_t lo, int64_t zt) {
    int64_t hi = (int64_t)fc + (zt - z0);
    if (hi > M) hi = M;
    const uint64_t T = (want << bz) | (uint64_t)zt;
    if (hi < M && cell_key[hi] == T) return (uint32_t)hi;
    int64_t a = lo, b = hi;
    while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (cell_key[mid] < T) a = mid + 1;
        else b = mid;
    }
    return (uint32_t)a;
}

// Forward half of the 5x5x5 stencil by column offset (dx, dy): the near
// shell (max(|dx|,|dy|,|dz|) == 1) uses the first four columns with
// |dz| <= 1.  The own column's dz = +1 needs no test there: the runs pass
// has tested every cell against the next cell when that one is its own
// column's dz = +1 or column (0, +1) within dz +- 1 (next_is_near), and
// joined such pairs share a run; unjoined ones have no edge.  For the same
// reason the near shell skips column (0, +1)'s first cell when it is the
// very next cell.
// Near-shell column q (0..3): (0, +1), (1, -1), (1, 0), (1, +1).
__device__ __forceinline__ void near_col(int q, int &dx, int &dy) {
    dx = q == 0 ? 0 : 1;
    dy = q == 0 ? 1 : q - 2;
}

// Near shell: a cell pair is skipped when both cells already share a root;
// otherwise point pairs are tested until the first joined one, which joins
// the two components.
//
// On large cell tables the shell runs in two steps, after the sampling
// idea of Afforest (Sutton et al., 2018): first every cell links to the
// first cell of each forward column when their first points are joined
// (one round of loads, no further search), which joins most of the ground
// into one component; that component is found (k_giant) and only the cells
// outside it run the full near shell, on their forward pairs and on their
// backward pairs towards the giant component.  A pair with both cells in
// the giant component is already joined; any other pair has a cell outside
// it, which handles the pair.  Small cell tables run the full shell on every
// cell, one task per candidate column.
//
// The kernel is latency bound, so the loads of one cell are issued in a
// few independent rounds rather than as one long dependent chain: (1) the
// cell's own key, points, parent and the parent's parent; (2) occupancy bit
// and index entry of a group of neighbour columns (all four on large cell
// tables; on small ones one column per task); (3) the first kNearK cells
// of each of those columns; (4) the parents of every candidate cell.  Only
// then are the candidates whose component differs tested one by one.  When
// the cells loaded from a column stop below A's reach (a tall column), the
// column's cells within reach are located directly (column_seek) and tested
// after.
//
constexpr int kNearK = 1;
// Columns per group on large cell tables: all four (groups of two or one,
// with fewer registers, measured slower on the map: 1.67 -> 1.76 / 1.97 ms).
constexpr int kNearGroup = 4;

// Cell tables shorter than this give each cell four tasks, one per
// candidate column (see k_hook_far's kFarSplitBelow); longer ones take the
// sampling links and the work list.
constexpr int64_t kNearSplitBelow = 131072;

// Queued cell pairs a block of a hooking kernel holds before its flush.
constexpr uint32_t kDeferBuf = 1024;

// Cell pairs whose first points are not joined are queued in LDS, then in a
// global queue, and tested by a later kernel, once the shell's other joins
// are in: most of them then share a root and need no test.  A pair the
// block's buffer cannot take is tested where it is found.
struct DeferLds {
    uint64_t buf[kDeferBuf];  // A << 32 | B
    uint32_t n, gbase;
};

__device__ __forceinline__ bool defer_push(DeferLds &q, int32_t A, uint32_t B) {
    const uint32_t slot = atomicAdd(&q.n, 1u);
    if (slot >= kDeferBuf) return false;
    q.buf[slot] = ((uint64_t)(uint32_t)A << 32) | B;
    return true;
}

// After the block's last cell: its pairs go to the global queue (counter
// *count) as far as the queue has room; the rest are tested here.
template <int BLK>
__device__ __forceinline__ void defer_flush(DeferLds &q, uint32_t *count,
                                            uint64_t *__restrict__ defer, uint64_t cap,
                                            const float4 *__restrict__ spts,
                                            const uint32_t *__restrict__ cell_start,
                                            int32_t *cpar, const Frame *__restrict__ frames,
                                            const uint32_t *__restrict__ cell_frame, bool batched,
                                            float d2_one) {
    __syncthreads();
    const uint32_t cnt = q.n < kDeferBuf ? q.n : kDeferBuf;
    if (threadIdx.x == 0) q.gbase = cnt ? atomicAdd(count, cnt) : 0u;
    __syncthreads();
    const uint64_t gbase = q.gbase;
    const uint32_t fit =
        gbase >= cap ? 0u : (gbase + cnt <= cap ? cnt : (uint32_t)(cap - gbase));
    for (uint32_t j = threadIdx.x; j < cnt; j += BLK) {
        if (j < fit) {
            defer[gbase + j] = q.buf[j];
        } else {
            const int32_t A = (int32_t)(q.buf[j] >> 32);
            defer_test(q.buf[j], spts, cell_start, cpar,
                       batched ? frames[cell_frame[A]].d2 : d2_one);
        }
    }
}

// Is cell B in the giant component of the last k_giant_bits (bitmap)?
__device__ __forceinline__ bool is_giant(const uint64_t *__restrict__ gbits, uint32_t B) {
    return (gbits[B >> 6] >> (B & 63)) & 1ull;
}

// Occupied columns of the (2H+1)x(2H+1) neighbourhood of column (cx, cy),
// from the dense index's occupancy bits (one or two words per row): bit
// (dx + H) * (2H + 1) + (dy + H).
template <int H>
__device__ __forceinline__ uint32_t occupied_box(const Grid &g, const uint32_t *__restrict__ colbits,
                                                 int64_t cx, int64_t cy) {
    constexpr int W = 2 * H + 1;
    const int64_t y0 = cy - H < 0 ? 0 : cy - H;
    const int64_t y1 = cy + H >= g.NY ? g.NY - 1 : cy + H;
    uint32_t w0[W], w1[W];
    int64_t i0[W];
#pragma unroll
    for (int r = 0; r < W; ++r) {
        const int64_t x = cx + r - H;
        const bool in = x >= 0 && x < g.NX;
        i0[r] = in ? x * g.NYp + y0 : 0;
        const int64_t i1 = in ? x * g.NYp + y1 : 0;
        w0[r] = in ? colbits[i0[r] >> 5] : 0u;
        w1[r] = in && (i1 >> 5) != (i0[r] >> 5) ? colbits[i1 >> 5] : 0u;
    }
    const uint32_t width = (uint32_t)(y1 - y0 + 1), lo = (uint32_t)(y0 - (cy - H));
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < W; ++r) {
        const uint64_t two = ((uint64_t)w1[r] << 32) | w0[r];
        const uint32_t row = (uint32_t)(two >> (i0[r] & 31)) & ((1u << width) - 1u);
        m |= row << (r * W + lo);
    }
    return m;
}

// The 5x5 box as a 24-bit mask in the far shell's column order: bit q for
// q' = (dx + 2) * 5 + (dy + 2), q = q' below the centre (q' = 12, left out)
// and q' - 1 above.
__device__ __forceinline__ uint32_t occupied_5x5(const Grid &g, const uint32_t *__restrict__ colbits,
                                                 int64_t cx, int64_t cy) {
    const uint32_t m = occupied_box<2>(g, colbits, cx, cy);
    return (m & 0xFFFu) | ((m >> 1) & ~0xFFFu);
}

// The 3x3 box as an 8-bit mask in the near shell's column order: bits 0..3
// the forward columns (0, +1), (1, -1), (1, 0), (1, +1), bits 4..7 the
// backward ones (0, -1), (-1, +1), (-1, 0), (-1, -1).
__device__ __forceinline__ uint32_t occupied_near(const Grid &g, const uint32_t *__restrict__ colbits,
                                                  int64_t cx, int64_t cy) {
    const uint32_t m = occupied_box<1>(g, colbits, cx, cy);  // bit (dx + 1) * 3 + (dy + 1)
    auto b = [&](int dx, int dy) { return (m >> ((dx + 1) * 3 + (dy + 1))) & 1u; };
    return b(0, 1) | b(1, -1) << 1 | b(1, 0) << 2 | b(1, 1) << 3 | b(0, -1) << 4 |
           b(-1, 1) << 5 | b(-1, 0) << 6 | b(-1, -1) << 7;
}

// Forms of the near shell: every cell, one task per candidate column (small
// cell tables); every cell, one task per cell (large tables); on large
// tables of large clouds, the sampling links and then the full shell over
// the cells outside their giant component.  With the dense column index the
// one-task-per-cell forms visit the occupied columns only (kNearAllOcc,
// kNearWorkOcc: instances of their own, as for the far shell).
constexpr int kNearSplit = 0, kNearAll = 1, kNearSample = 2, kNearWork = 3, kNearWorkOcc = 4,
              kNearAllOcc = 5;
// The sampling links go to the first cells of the three columns at dx = +1
// (mask over near_col's columns): the column (0, +1) adds few links the runs
// have not made already (map: sampling 0.65 ms and near shell 0.55 ms either
// way; only (1, 0): 0.57 and 0.71 ms).  Sampling from run starts only, or
// with one compare-and-swap per link and no retry, leaves no giant component
// (with no retry a root takes at most one hook, and the trees stay small).
constexpr uint32_t kSampleCols = 0xEu;
// Clouds of at least this many points take the sampling links (unless the
// launch configuration says otherwise, see fec_tuning_set); in a batch, the
// frames' average decides (the ground of each frame is what sampling
// joins, and a batch of small frames has the small frames' thin ground).
// They pay
// where the near shell's cells in the giant component are expensive, on
// dense accumulated ground (27 M-point map: sampling, near shell, queued
// pairs and compression 1.53 -> 1.43 ms, call 4.20 -> 4.06 ms); on single
// scans the shell is cheap already and the sampling costs more than it
// saves (64-frame batch of 5.4 M points: 0.40 -> 0.50 ms).
constexpr int64_t kSampleMinPoints = 1 << 23;

template <int kMode, int BLK>
__global__ __launch_bounds__(BLK) void k_hook_near(const float4 *__restrict__ spts,
                                                      const uint32_t *__restrict__ cell_start,
                                                      const uint64_t *__restrict__ cell_key,
                                                      const uint64_t *__restrict__ col_key,
                                                      const uint32_t *__restrict__ col_cell,
                                                      const uint32_t *__restrict__ colgrid,
                                                      const uint32_t *__restrict__ colbits,
                                                      const uint64_t *__restrict__ gbits,
                                                      const uint32_t *__restrict__ work,
                                                      const Frame *__restrict__ frames,
                                                      const uint32_t *__restrict__ cell_frame,
                                                      int32_t *cpar, Params *__restrict__ P,
                                                      uint64_t *__restrict__ defer,
                                                      uint64_t defer_cap) {
    if (P->status != kStatusOk) return;
    const int64_t M = P->M;
    constexpr bool kSplit = kMode == kNearSplit;
    constexpr bool kSample = kMode == kNearSample;
    constexpr bool kWork = kMode == kNearWork || kMode == kNearWorkOcc;
    constexpr bool kOcc = kMode == kNearWorkOcc || kMode == kNearAllOcc;
    constexpr bool kAll = kMode == kNearAll || kMode == kNearAllOcc;
    if ((M < kNearSplitBelow) != kSplit) return;  // another form's case
    const ColIndex ci = colindex_of(P, colgrid, colbits, col_key, col_cell);
    // the occupancy form of the pair, or the other
    if ((kWork || kAll) && (ci.mode == kColDense) != kOcc) return;
    const float d2_one = P->d2;
    const bool batched = P->nframes > 1;
    const Grid g = grid_of(P);
    // columns: the four forward ones, and on the work list the four
    // backward ones after them
    constexpr int kC = kWork ? 8 : 4;
    // columns per group: a group's loads are issued together, the groups of
    // a cell one after the other (fewer registers, more waves)
    // (the all-cell occupancy form: two at a time, for its four columns;
    // 64-frame batch 0.245 -> 0.227 ms; the work-list form keeps four, the
    // map's near shell being 0.60 -> 0.61 ms with two)
    constexpr int kNG = kSplit ? 1 : (kMode == kNearAllOcc ? 2 : kNearGroup);
    constexpr int kGroups = kC / kNG;
    constexpr int kCand = kNG * kNearK;
    static_assert(kC % kNG == 0 && kCand <= 32, "groups cover the columns; 32-bit masks");
    // pairs whose first points are not joined: queued (see DeferLds); the
    // sampling links test first points only
    __shared__ DeferLds dq;
    if (!kSample) {
        if (threadIdx.x == 0) dq.n = 0;
        __syncthreads();
    }
    auto queue = [&](int32_t A, uint32_t B) { return defer_push(dq, A, B); };
    // kSplit: one task per (cell, group); every task loads the cell's own data
    constexpr int kTasks = kSplit ? kGroups : 1;
    const uint64_t ntask = kWork ? (uint64_t)P->nwork0 : (uint64_t)M * kTasks;
    const uint64_t t0 = kWork ? (uint64_t)xcd_block<kXcdRunFar>() * BLK + threadIdx.x
                              : (uint64_t)xcd_block<kXcdRunNear>() * BLK + threadIdx.x;
    for (uint64_t t = t0; t < ntask; t += (uint64_t)gridDim.x * BLK) {
        const int32_t A = kWork ? (int32_t)work[t] : (int32_t)(t / kTasks);
        const int task = (int)(t % kTasks);
        // round 1
        const uint64_t key = cell_key[A];
        // the sampling links come from the first (lowest) cell of each
        // column only: the cells above it mostly reach the same neighbour
        // columns' first cells, and the runs join them to it where their
        // points are joined (map: sampling 0.57 -> 0.50 ms, its work list
        // 2.30 -> 2.36 M cells, call 3.77 -> 3.74 ms)
        if (kSample && A > 0 && (cell_key[A - 1] >> g.bz) == (key >> g.bz)) continue;
        // (the sampling links test first points only: no point ranges)
        const uint32_t sA = cell_start[A], eA = kSample ? 0u : cell_start[A + 1];
        const int32_t p0 = cpar[A];
        const uint32_t fA = batched ? cell_frame[A] : 0u;
        const uint64_t ck = key >> g.bz;
        const int64_t cz = (int64_t)(key & g.zmask);
        int64_t cx, cy;
        g.col_xy(ck, cx, cy);
        const float4 pa = spts[sA];  // A's first point, for the one-pair tests
        const int32_t q0 = cpar[p0];
        const float d2 = batched ? frames[fA].d2 : d2_one;  // neighbours share A's frame
        int32_t ra = -1;  // A's root, found once the first group's loads are out
        // kOcc: the occupied columns, kNG at a time; otherwise fixed groups
        uint32_t todo = kOcc ? occupied_near(g, colbits, cx, cy) & (kWork ? 0xFFu : 0x0Fu) : 0u;
#pragma unroll 1
        for (int grp = kSplit ? task : 0;
             kOcc ? todo != 0u : grp < (kSplit ? task + 1 : kGroups); ++grp) {
            // column of each slot; backward columns (work list): only pairs
            // towards the giant component, the others are their other
            // cell's forward pairs
            int qs[kNG];
            bool back[kNG];
            // round 2: neighbour columns
            bool has[kNG];
            uint32_t fc[kNG];
            uint64_t want[kNG];
            int64_t nxs[kNG], nys[kNG];
#pragma unroll
            for (int o = 0; o < kNG; ++o) {
                const bool use = !kOcc || todo != 0u;
                qs[o] = kOcc ? (use ? __ffs(todo) - 1 : 0) : grp * kNG + o;
                if (kOcc) todo &= todo - 1u;
                back[o] = kWork && qs[o] >= 4;
                int dx, dy;
                near_col(qs[o] & 3, dx, dy);
                if (back[o]) {
                    dx = -dx;
                    dy = -dy;
                }
                nxs[o] = use ? cx + dx : -1;  // an unused slot: off the grid
                nys[o] = cy + dy;
                want[o] = g.col_key((uint64_t)(cx + dx), (uint64_t)nys[o]);
                if (kSample && !((kSampleCols >> qs[o]) & 1u)) nxs[o] = -1;  // off the grid
            }
            if (kSample && ci.mode == kColDense) {
                // the sampled columns lie in row cx + 1, at cy - 1 .. cy + 1:
                // their occupancy bits come from one or two words
                const bool rin = cx + 1 < g.NX;
                const int64_t ylo = cy > 0 ? cy - 1 : 0;
                const int64_t i0 = rin ? (cx + 1) * g.NYp + ylo : 0;
                const int64_t i1 = rin ? (cx + 1) * g.NYp + (cy + 1 < g.NY ? cy + 1 : g.NY - 1) : 0;
                const uint32_t w0 = rin ? ci.colbits[i0 >> 5] : 0u;
                const uint32_t w1 = (rin && (i1 >> 5) != (i0 >> 5)) ? ci.colbits[i1 >> 5] : 0u;
                const uint64_t two = ((uint64_t)w1 << 32) | w0;
#pragma unroll
                for (int o = 0; o < kNG; ++o) {
                    const bool in = nxs[o] >= 0 && nxs[o] < g.NX && nys[o] >= 0 && nys[o] < g.NY;
                    const int64_t idx = in ? nxs[o] * g.NYp + nys[o] : 0;
                    has[o] = in && ((two >> (idx - (i0 & ~31ll))) & 1ull);
                    fc[o] = has[o] ? ci.colgrid[idx] : 0u;
                }
            } else if (kOcc) {
                // occupied by construction: only the first cells to load
#pragma unroll
                for (int o = 0; o < kNG; ++o) {
                    has[o] = nxs[o] >= 0;
                    fc[o] = has[o] ? ci.colgrid[(uint64_t)(nxs[o] * g.NYp + nys[o])] : 0u;
                }
            } else {
                find_columns<kNG>(g, ci, nxs, nys, has, fc);
            }
            // round 3: first cells of each column
            uint64_t kk[kNG][kNearK];
#pragma unroll
            for (int o = 0; o < kNG; ++o)
#pragma unroll
                for (int j = 0; j < kNearK; ++j) {
                    const int64_t B = (int64_t)fc[o] + j;
                    kk[o][j] = (has[o] && B < M) ? cell_key[B] : ~0ull;
                }
            // candidates (existence is tracked explicitly: a key sentinel
            // could equal the wrapped key of a column off the grid)
            uint32_t cm = 0, ovf = 0;
#pragma unroll
            for (int o = 0; o < kNG; ++o) {
#pragma unroll
                for (int j = 0; j < kNearK; ++j) {
                    const bool loaded = has[o] && (int64_t)fc[o] + j < M;
                    const bool inc = loaded && (kk[o][j] >> g.bz) == want[o];
                    const int64_t dz = (int64_t)(kk[o][j] & g.zmask) - cz;
                    bool c = inc && dz >= -1 && dz <= 1;
                    if (back[o]) c = c && is_giant(gbits, fc[o] + (uint32_t)j);
                    if (c) cm |= 1u << (o * kNearK + j);
                    if (j == kNearK - 1 && inc && dz < 1) ovf |= 1u << o;
                }
            }
            // column 0 is (0, +1): its first cell, when it is the next cell,
            // was decided by the runs pass; backwards, column (0, -1)'s cell
            // A - 1 likewise (its last cell, or its first when it has one)
#pragma unroll
            for (int o = 0; o < kNG; ++o) {
                if (qs[o] == 0 && fc[o] == (uint32_t)A + 1) cm &= ~(1u << (o * kNearK));
                if (back[o] && qs[o] == 4 && fc[o] + (uint32_t)(kNearK - 1) == (uint32_t)A - 1)
                    cm &= ~(1u << (o * kNearK + kNearK - 1));
            }
            // round 4: parents and point ranges of the candidates
            int32_t rb[kCand];
            uint32_t sb[kCand], eb[kCand];
#pragma unroll
            for (int i = 0; i < kCand; ++i) {
                const uint32_t B = fc[i / kNearK] + (uint32_t)(i % kNearK);
                const bool c = (cm >> i) & 1u;
                rb[i] = c ? cpar[B] : -1;
                sb[i] = c ? cell_start[B] : 0u;
                eb[i] = (c && !kSample) ? cell_start[B + 1] : 0u;
            }
            if (ra < 0) ra = (q0 == p0) ? p0 : uf_find(cpar, q0);
            FEC_COUNT(P, 0, __popc(cm));
            // round 5: the first point of every candidate in another
            // component, tested against A's first point all at once; that
            // one pair decides most joined cell pairs, the others are
            // scanned in full below
            uint32_t need = 0, quick = 0;
#pragma unroll
            for (int i = 0; i < kCand; ++i) {
                const bool nd = ((cm >> i) & 1u) && rb[i] != ra && rb[i] != p0;
                need |= (uint32_t)nd << i;
                if (nd) quick |= (uint32_t)joined(pa.x, pa.y, pa.z, spts[sb[i]], d2) << i;
            }
            // the sampling links: joined first points only
            if (kSample) need &= quick;
            // candidates whose parent (their run's first cell) is that of a
            // candidate already joined to A's component need no search: a
            // cached read of the parent just hooked may still show it as a
            // root, and its hook would only fail
            uint32_t joinedm = 0;
#pragma unroll
            for (int i = 0; i < kCand; ++i) {
                if (!((need >> i) & 1u)) continue;
                bool dup = false;
#pragma unroll
                for (int j = 0; j < i; ++j) dup |= ((joinedm >> j) & 1u) && rb[j] == rb[i];
                if (dup) continue;
                const int32_t r = uf_find(cpar, rb[i]);
                if (r == ra) {
                    joinedm |= 1u << i;
                    continue;
                }
                FEC_COUNT(P, 1, 1);
                FEC_COUNT(P, 3, (eA - sA) * (eb[i] - sb[i]));
                if (((quick >> i) & 1u) ||
                    (!queue(A, fc[i / kNearK] + (uint32_t)(i % kNearK)) &&
                     any_joined(spts, sA, eA, sb[i], eb[i], d2))) {
                    FEC_COUNT(P, 2, 1);
                    ra = uf_link_roots(cpar, uf_find(cpar, ra), r);
                    joinedm |= 1u << i;
                }
            }
            if (kSample) continue;
            FEC_COUNT(P, 4, __popc(ovf));
            // columns with cells in reach beyond the loaded ones: at most
            // three more (z within cz +- 1, distinct), from the first one
            // not below
            if (ovf) {
                for (int o = 0; o < kNG; ++o) {
                    if (!((ovf >> o) & 1u)) continue;
                    const int64_t zl = (int64_t)(kk[o][kNearK - 1] & g.zmask);
                    const uint32_t st =
                        zl >= cz - 1 ? fc[o] + kNearK
                                     : column_seek(cell_key, M, g.bz, want[o], fc[o],
                                                   (int64_t)(kk[o][0] & g.zmask),
                                                   fc[o] + kNearK, cz - 1);
                    uint64_t kx[3];
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        kx[j] = (int64_t)st + j < M ? cell_key[st + j] : ~0ull;
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const uint32_t B = st + j;
                        if ((int64_t)B >= M || (kx[j] >> g.bz) != want[o]) break;
                        const int64_t dz = (int64_t)(kx[j] & g.zmask) - cz;
                        if (dz > 1) break;
                        if (dz < -1) continue;
                        if (back[o] && (B == (uint32_t)A - 1 || !is_giant(gbits, B))) continue;
                        const int32_t r = uf_find(cpar, (int32_t)B);
                        if (r == ra) continue;
                        const uint32_t sB = cell_start[B];
                        if (joined(pa.x, pa.y, pa.z, spts[sB], d2) ||
                            (!queue(A, B) && any_joined(spts, sA, eA, sB, cell_start[B + 1], d2)))
                            ra = uf_link(cpar, ra, r);
                    }
                }
            }
        }
    }
    if (!kSample)
        defer_flush<BLK>(dq, &P->ndefer[0], defer, defer_cap, spts, cell_start, cpar, frames,
                         cell_frame, batched, d2_one);
}

// The pairs a hooking kernel queued (the first min(count, capacity) entries
// of the queue; `which` 0: near shell, 1: far shell).
__global__ __launch_bounds__(kBlock) void k_deferred(const float4 *__restrict__ spts,
                                                     const uint32_t *__restrict__ cell_start,
                                                     const Frame *__restrict__ frames,
                                                     const uint32_t *__restrict__ cell_frame,
                                                     int32_t *cpar, const Params *__restrict__ P,
                                                     const uint64_t *__restrict__ defer,
                                                     uint64_t defer_cap,
                                                     const uint32_t *__restrict__ runq, int which) {
    if (P->status != kStatusOk) return;
    const uint64_t cnt = P->ndefer[which] < defer_cap ? P->ndefer[which] : defer_cap;
    // after the near shell, also the runs pass's pairs (cell A - 1, cell A)
    const uint64_t nq = which == 0 ? P->nrunq : 0;
    const bool batched = P->nframes > 1;
    const float d2_one = P->d2;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < cnt + nq;
         i += (uint64_t)gridDim.x * kBlock) {
        uint64_t e;
        if (i < cnt) {
            e = defer[i];
        } else {
            const uint32_t B = runq[i - cnt];
            e = ((uint64_t)(B - 1u) << 32) | B;
        }
        const int32_t A = (int32_t)(e >> 32);
        defer_test(e, spts, cell_start, cpar, batched ? frames[cell_frame[A]].d2 : d2_one);
    }
}

// Every cell points at its root afterwards.  Runs after all joins (data is
// coherent at the kernel boundary); each slot is written once, with the
// root, so concurrent finds only ever see ancestors.
// `min_cells`: cell tables shorter than this skip it (the sampling round's
// compression, for large tables only).
__global__ __launch_bounds__(kBlock) void k_compress(int32_t *cpar, const Params *__restrict__ P,
                                                     int64_t min_cells) {
    if (P->status != kStatusOk) return;
    const int64_t M = P->M;
    if (M < min_cells) return;
    for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < M;
         x += (int64_t)gridDim.x * kBlock) {
        cpar[x] = uf_find(cpar, (int32_t)x);
    }
}

// The most frequent root among up to 4096 evenly spaced cells of one frame.
// One block per frame.
constexpr int kGiantSample = 4096;
constexpr int kGiantSlots = 8192;

__global__ __launch_bounds__(1024) void k_giant(const int32_t *__restrict__ cpar,
                                                Frame *__restrict__ frames,
                                                Params *__restrict__ P, int64_t min_cells) {
    if (P->status != kStatusOk || P->M < min_cells) return;
    __shared__ int32_t t_key[kGiantSlots];
    __shared__ uint32_t t_cnt[kGiantSlots];
    __shared__ uint64_t s_best[1024 / 64];
    const int nframes = P->nframes;
    const int f = blockIdx.x;
    // the frame's cells: from its first cell to the next non-empty frame's
    int64_t c0 = 0, c1 = P->M;
    if (nframes > 1) {
        if (frames[f].nvalid == 0) {
            if (threadIdx.x == 0) frames[f].giant = -1;
            return;
        }
        c0 = frames[f].cell0;
        for (int g = f + 1; g < nframes; ++g)
            if (frames[g].nvalid > 0) {
                c1 = frames[g].cell0;
                break;
            }
    }
    const int64_t Mf = c1 - c0;
    for (int i = threadIdx.x; i < kGiantSlots; i += 1024) {
        t_key[i] = -1;
        t_cnt[i] = 0;
    }
    __syncthreads();
    const int64_t S = Mf < kGiantSample ? Mf : kGiantSample;
    for (int64_t i = threadIdx.x; i < S; i += 1024) {
        const int32_t r = cpar[c0 + i * Mf / S];
        uint32_t h = ((uint32_t)r * 2654435761u) >> (32 - 13);
        for (int probe = 0; probe < kGiantSlots; ++probe) {
            const int32_t prev = atomicCAS(&t_key[h], -1, r);
            if (prev == -1 || prev == r) {
                atomicAdd(&t_cnt[h], 1u);
                break;
            }
            h = (h + 1) & (kGiantSlots - 1);
        }
    }
    __syncthreads();
    // best = max count, then smallest root: pack (count, ~root) into 64 bits
    uint64_t best = 0;
    for (int i = threadIdx.x; i < kGiantSlots; i += 1024) {
        const int32_t r = t_key[i];
        if (r >= 0) {
            const uint64_t v = ((uint64_t)t_cnt[i] << 32) | (uint64_t)(0x7FFFFFFFu - (uint32_t)r);
            best = v > best ? v : best;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t w = __shfl_xor(best, o);
        best = w > best ? w : best;
    }
    if (__lane_id() == 0) s_best[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t b = 0;
        for (int w = 0; w < 1024 / 64; ++w) b = s_best[w] > b ? s_best[w] : b;
        const int32_t giant = b ? (int32_t)(0x7FFFFFFFu - (uint32_t)(b & 0xFFFFFFFFu)) : -1;
        frames[f].giant = giant;
        if (nframes == 1) P->giant = giant;
    }
}

// Bitmap of the cells in the giant component and the list of the others, in
// cell order: after the sampling links (`which` 0: the near-shell work list,
// large cell tables only, count in P->nwork0) and after the near shell
// (`which` 1: the far-shell work list, count in P->nwork).  Two kernels on
// the same grid of at most kListBlocks blocks, each block on one contiguous
// chunk of whole 256-cell groups: the first writes the bitmap and the
// block's count of listed cells, the second adds up the counts of the
// blocks before it and writes its cells from the bitmap.  No atomics: the
// list comes out sorted, which keeps a shell's neighbouring tasks close in
// space (with one slot reservation per block the list was a shuffle of
// chunks, and the far shell 10 % slower), and all blocks reserving at once
// on one address had queued.
__device__ __forceinline__ void list_chunk(int64_t M, int64_t &c0, int64_t &c1) {
    const int64_t groups = (M + kBlock - 1) / kBlock;
    const int64_t per = (groups + gridDim.x - 1) / gridDim.x;
    c0 = (int64_t)blockIdx.x * per * kBlock;
    c1 = c0 + per * kBlock < M ? c0 + per * kBlock : M;
}

__global__ __launch_bounds__(kBlock) void k_giant_bits(const int32_t *__restrict__ cpar,
                                                       uint64_t *__restrict__ gbits,
                                                       uint32_t *__restrict__ listcnt,
                                                       const Frame *__restrict__ frames,
                                                       const uint32_t *__restrict__ cell_frame,
                                                       const Params *__restrict__ P, int which) {
    if (P->status != kStatusOk) return;
    const int64_t M = P->M;
    if (which == 0 && M < kNearSplitBelow) return;
    const bool batched = P->nframes > 1;
    const int32_t giant_one = P->giant;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    int64_t c0, c1;
    list_chunk(M, c0, c1);
    // kNgG groups of 256 cells per round, their parents loaded at once
    constexpr int kNgG = 8;
    uint32_t mine = 0;
    for (int64_t r0 = c0; r0 < c1; r0 += (int64_t)kNgG * kBlock) {
        int32_t par[kNgG], fr[kNgG];
#pragma unroll
        for (int k = 0; k < kNgG; ++k) {
            const int64_t A = r0 + k * kBlock + threadIdx.x;
            par[k] = A < c1 ? cpar[A] : -1;
            fr[k] = (A < c1 && batched) ? (int32_t)cell_frame[A] : 0;
        }
#pragma unroll
        for (int k = 0; k < kNgG; ++k) {
            const int64_t A = r0 + k * kBlock + threadIdx.x;
            const bool valid = A < c1;
            const int32_t g = valid ? (batched ? frames[fr[k]].giant : giant_one) : -2;
            const bool gi = valid && par[k] == g;
            const uint64_t gm = __ballot(gi);
            if (lane == 0 && valid) gbits[A >> 6] = gm;  // A is 64-aligned on lane 0
            mine += (valid && !gi) ? 1u : 0u;
        }
    }
    __shared__ uint32_t s_w[kBlock / 64];
    mine = wave_sum(mine);
    if (lane == 0) s_w[wave] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < kBlock / 64; ++w) tot += s_w[w];
        listcnt[blockIdx.x] = tot;
    }
}

__global__ __launch_bounds__(kBlock) void k_work_list(const uint64_t *__restrict__ gbits,
                                                      const uint32_t *__restrict__ listcnt,
                                                      uint32_t *__restrict__ work,
                                                      Params *__restrict__ P, int which) {
    if (P->status != kStatusOk) return;
    const int64_t M = P->M;
    if (which == 0 && M < kNearSplitBelow) return;
    __shared__ uint32_t s_tmp[kBlock / 64];
    // where this block's cells go: the counts of the blocks before it (and
    // block 0 publishes the total)
    uint32_t before = 0, total = 0;
    for (uint32_t b = threadIdx.x; b < gridDim.x; b += kBlock) {
        const uint32_t c = listcnt[b];
        before += b < blockIdx.x ? c : 0u;
        total += c;
    }
    uint32_t t;
    const uint32_t bsum = block_excl_scan(before, s_tmp, t);
    (void)bsum;
    const uint32_t base = t;  // sum of `before` over the block
    __syncthreads();
    if (blockIdx.x == 0) {
        const uint32_t x = block_excl_scan(total, s_tmp, t);
        (void)x;
        if (threadIdx.x == 0) *(which == 0 ? &P->nwork0 : &P->nwork) = t;
        __syncthreads();
    }
    int64_t c0, c1;
    list_chunk(M, c0, c1);
    // one 64-cell word of the bitmap per thread and step; listed cells are
    // its zero bits below c1
    uint32_t run = base;
    for (int64_t w0 = c0 >> 6; w0 < (c1 + 63) >> 6; w0 += kBlock) {
        const int64_t w = w0 + threadIdx.x;
        uint64_t lst = 0;
        if (w < (c1 + 63) >> 6) {
            lst = ~gbits[w];
            const int64_t hi = c1 - (w << 6);  // cells of this word below c1
            if (hi < 64) lst &= (1ull << hi) - 1ull;
        }
        uint32_t tot;
        const uint32_t off = block_excl_scan((uint32_t)__popcll(lst), s_tmp, tot);
        uint32_t o = run + off;
        while (lst) {
            const int bit = __ffsll((unsigned long long)lst) - 1;
            lst &= lst - 1ull;
            work[o++] = (uint32_t)((w << 6) + bit);
        }
        run += tot;
        __syncthreads();  // s_tmp is reused by the next step
    }
}

// Far shell (max(|dx|,|dy|,|dz|) == 2) around every cell outside the giant
// component.  A cell pair is handled here when its first cell is outside
// the giant component and either the pair is "forward" (dx > 0, or dx == 0
// and dy > 0, or dx == dy == 0 and dz > 0) or the second cell is inside it.
// So every far pair with at least one cell outside the giant component is
// handled; pairs with both cells inside are already joined.

// Work lists shorter than this are cut into one task per column group
// (a small cloud leaves most of the chip idle, and each lane's chain of
// dependent loads sets the kernel's time); longer ones keep one task per
// cell (the chip is full, and the tasks' repeated set-up would cost more).
constexpr uint32_t kFarSplitBelow = 131072;

// kOcc: the large form for the dense column index, which visits only the
// occupied columns (see occupied_5x5); the other large form serves the hash
// and search indexes.  Separate instances keep each one's registers down
// (one kernel with both paths made the hash form 8 % slower on batches).
template <bool kSplit, bool kOcc, int BLK>
__global__ __launch_bounds__(BLK) void k_hook_far(const float4 *__restrict__ spts,
                                                      const uint32_t *__restrict__ cell_start,
                                                      const uint64_t *__restrict__ cell_key,
                                                      const uint64_t *__restrict__ col_key,
                                                      const uint32_t *__restrict__ col_cell,
                                                      const uint32_t *__restrict__ colgrid,
                                                      const uint32_t *__restrict__ colbits,
                                                      const uint64_t *__restrict__ gbits,
                                                      const uint32_t *__restrict__ work,
                                                      const Frame *__restrict__ frames,
                                                      const uint32_t *__restrict__ cell_frame,
                                                      int32_t *cpar, Params *__restrict__ P,
                                                      uint64_t *__restrict__ defer,
                                                      uint64_t defer_cap) {
    if (P->status != kStatusOk) return;
    const int64_t M = P->M;
    const uint32_t nwork = P->nwork;
    const ColIndex ci = colindex_of(P, colgrid, colbits, col_key, col_cell);
    const float d2_one = P->d2;
    const bool batched = P->nframes > 1;
    const Grid g = grid_of(P);
    // Columns per group (their loads issued together) and cells per column
    // loaded up front.  Small groups and one cell keep the registers low
    // (88 with groups of 3, 65 with single columns, against 163 with groups
    // of 8 and two cells), so more waves hide the loads' latency; measured
    // per call with groups of 3: map 0.97 -> 0.70 ms, 64-frame batch 0.51
    // -> 0.39 ms.  Small work lists (kSplit) give each column a task of its
    // own: 120 k frame 0.058 -> 0.046 ms.
    constexpr int kG = kSplit ? 1 : 3;
    constexpr int kK = 1;
    static_assert(kG * kK <= 32, "candidate masks are 32-bit");
    static_assert(kG <= 32 && 24 % kG == 0, "groups cover the 24 columns");
    if ((nwork < kFarSplitBelow) != kSplit) return;  // another instance's case
    static_assert(!(kSplit && kOcc), "the occupancy form is a large form");
    if (!kSplit && (ci.mode == kColDense) != kOcc) return;
    // pairs whose first points are not joined: queued (see DeferLds)
    __shared__ DeferLds dq;
    if (threadIdx.x == 0) dq.n = 0;
    __syncthreads();
    // kSplit: one task per (work cell, group of kG columns).  The groups of a
    // cell are independent; a lane that walks all of them in turn carries
    // one long chain of dependent loads (about 50 us per cell, measured).
    constexpr uint32_t kGroups = 24 / kG;
    constexpr uint32_t kTasks = kSplit ? kGroups : 1;
    const uint64_t ntask = (uint64_t)nwork * kTasks;
    for (uint64_t t = (uint64_t)xcd_block<kXcdRunFar>() * BLK + threadIdx.x; t < ntask;
         t += (uint64_t)gridDim.x * BLK) {
        const uint32_t wi = (uint32_t)(t / kTasks);
        const int task = (int)(t % kTasks);
        const int32_t A = (int32_t)work[wi];
        const uint64_t key = cell_key[A];
        const uint64_t ck = key >> g.bz;
        const int64_t cz = (int64_t)(key & g.zmask);
        int64_t cx, cy;
        g.col_xy(ck, cx, cy);
        const uint32_t sA = cell_start[A], eA = cell_start[A + 1];
        int32_t ra = uf_find(cpar, A);
        const float d2 = batched ? frames[cell_frame[A]].d2 : d2_one;
        const float4 pa = spts[sA];  // A's first point, for the one-pair tests
        auto pair = [&](uint32_t B, int32_t rb) {
            FEC_COUNT(P, 5, 1);
            if (rb == ra) return;
            rb = uf_find(cpar, rb);
            if (rb == ra) return;
            FEC_COUNT(P, 6, 1);
            FEC_COUNT(P, 7, (eA - sA) * (cell_start[B + 1] - cell_start[B]));
            const uint32_t sB = cell_start[B];
            if (joined(pa.x, pa.y, pa.z, spts[sB], d2) ||
                (!defer_push(dq, A, B) && any_joined(spts, sA, eA, sB, cell_start[B + 1], d2)))
                ra = uf_link_roots(cpar, uf_find(cpar, ra), rb);
        };
        // own column (first task of the cell): the cells two steps down (if
        // giant) and up
        for (int32_t B = A - 1; task == 0 && B >= 0 && B >= A - 2; --B) {
            const uint64_t kb = cell_key[B];
            const int64_t dz = cz - (int64_t)(kb & g.zmask);
            if ((kb >> g.bz) != ck || dz > 2) break;
            if (dz == 2 && is_giant(gbits, (uint32_t)B)) pair((uint32_t)B, cpar[B]);
        }
        for (int32_t B = A + 1; task == 0 && B < M && B <= A + 2; ++B) {
            const uint64_t kb = cell_key[B];
            const int64_t dz = (int64_t)(kb & g.zmask) - cz;
            if ((kb >> g.bz) != ck || dz > 2) break;
            if (dz == 2) pair((uint32_t)B, cpar[B]);
        }
        // the task's columns of the 24 others of the 5x5 neighbourhood, kG
        // at a time: with the dense index only the occupied ones (a third
        // of them around the map's work cells), known from the occupancy
        // bits of the five rows
        uint32_t todo = kOcc ? occupied_5x5(g, colbits, cx, cy) : 0u;
#pragma unroll 1
        for (int grp = kSplit ? task : 0;
             kOcc ? todo != 0u : grp < (kSplit ? task + 1 : (int)kGroups); ++grp) {
            int dxs[kG], dys[kG];
            bool has[kG], use[kG];
            uint32_t fc[kG];
            uint64_t want[kG];
            int64_t nxs[kG], nys[kG];
#pragma unroll
            for (int o = 0; o < kG; ++o) {
                use[o] = !kOcc || todo != 0u;
                int q = kOcc ? (use[o] ? __ffs(todo) - 1 : 0) : grp * kG + o;
                todo &= todo - 1u;
                q = q >= 12 ? q + 1 : q;  // skip (0, 0)
                dxs[o] = q / 5 - 2;
                dys[o] = q % 5 - 2;
                nxs[o] = use[o] ? cx + dxs[o] : -1;  // unused slot: off the grid
                nys[o] = cy + dys[o];
                want[o] = g.col_key((uint64_t)nxs[o], (uint64_t)nys[o]);
            }
            if (kOcc) {
                // occupied by construction: only the first cells to load
#pragma unroll
                for (int o = 0; o < kG; ++o) {
                    has[o] = use[o];
                    fc[o] = use[o] ? ci.colgrid[(uint64_t)(nxs[o] * g.NYp + nys[o])] : 0u;
                }
            } else {
                find_columns<kG>(g, ci, nxs, nys, has, fc);
            }
            uint64_t kk[kG][kK];
#pragma unroll
            for (int o = 0; o < kG; ++o)
#pragma unroll
                for (int j = 0; j < kK; ++j) {
                    const int64_t B = (int64_t)fc[o] + j;
                    kk[o][j] = (has[o] && B < M) ? cell_key[B] : 0ull;
                }
            uint32_t cm = 0, ovf = 0;
#pragma unroll
            for (int o = 0; o < kG; ++o) {
                const bool near_col = dxs[o] >= -1 && dxs[o] <= 1 && dys[o] >= -1 && dys[o] <= 1;
                const bool fwd = dxs[o] > 0 || (dxs[o] == 0 && dys[o] > 0);
#pragma unroll
                for (int j = 0; j < kK; ++j) {
                    const bool loaded = has[o] && (int64_t)fc[o] + j < M;
                    const bool inc = loaded && (kk[o][j] >> g.bz) == want[o];
                    const int64_t dz = (int64_t)(kk[o][j] & g.zmask) - cz;
                    const bool inreach = inc && dz >= -2 && dz <= 2 &&
                                         !(near_col && dz >= -1 && dz <= 1);
                    // backward pairs only towards the giant component
                    if (inreach && (fwd || is_giant(gbits, fc[o] + (uint32_t)j)))
                        cm |= 1u << (o * kK + j);
                    if (j == kK - 1 && inc && dz < 2) ovf |= 1u << o;
                }
            }
            int32_t rb[kG * kK];
#pragma unroll
            for (int i = 0; i < kG * kK; ++i)
                rb[i] = ((cm >> i) & 1u) ? cpar[fc[i / kK] + (i % kK)] : -1;
#pragma unroll
            for (int i = 0; i < kG * kK; ++i)
                if ((cm >> i) & 1u) pair(fc[i / kK] + (uint32_t)(i % kK), rb[i]);
            // columns with cells in reach beyond the loaded ones (z within
            // cz +- 2, distinct): located directly, at most five
            if (ovf) {
                for (int o = 0; o < kG; ++o) {
                    if (!((ovf >> o) & 1u)) continue;
                    const bool near_col =
                        dxs[o] >= -1 && dxs[o] <= 1 && dys[o] >= -1 && dys[o] <= 1;
                    const bool fwd = dxs[o] > 0 || (dxs[o] == 0 && dys[o] > 0);
                    const int64_t zl = (int64_t)(kk[o][kK - 1] & g.zmask);
                    const uint32_t st =
                        zl >= cz - 2 ? fc[o] + kK
                                     : column_seek(cell_key, M, g.bz, want[o], fc[o],
                                                   (int64_t)(kk[o][0] & g.zmask), fc[o] + kK,
                                                   cz - 2);
                    uint64_t kx[5];
#pragma unroll
                    for (int j = 0; j < 5; ++j)
                        kx[j] = (int64_t)st + j < M ? cell_key[st + j] : ~0ull;
#pragma unroll
                    for (int j = 0; j < 5; ++j) {
                        const uint32_t B = st + j;
                        if ((int64_t)B >= M || (kx[j] >> g.bz) != want[o]) break;
                        const int64_t dz = (int64_t)(kx[j] & g.zmask) - cz;
                        if (dz > 2) break;
                        if (dz < -2 || (near_col && dz >= -1 && dz <= 1)) continue;
                        if (fwd || is_giant(gbits, B)) pair(B, cpar[B]);
                    }
                }
            }
        }
    }
    defer_flush<BLK>(dq, &P->ndefer[1], defer, defer_cap, spts, cell_start, cpar, frames,
                     cell_frame, batched, d2_one);
}

// ------------------------------------------------------------- 9. finalize
// Cluster sizes and smallest original index per root.  Each block takes a
// contiguous run of cells and adds them into a block-local hash table of
// roots in LDS (one root of a giant component takes most cells, and global
// atomics on one address serialise), then flushes one global atomic per
// distinct root.
constexpr int kAggSlots = 4096;

__global__ __launch_bounds__(kBlock) void k_final_cells(const int32_t *__restrict__ cpar,
                                                        const uint32_t *__restrict__ cell_start,
                                                        const uint32_t *__restrict__ sorig,
                                                        uint32_t *__restrict__ csize,
                                                        uint32_t *__restrict__ ccanon,
                                                        Params *__restrict__ P) {
    if (P->status != kStatusOk) return;
    __shared__ int32_t t_key[kAggSlots];
    __shared__ uint32_t t_sum[kAggSlots], t_min[kAggSlots];
    __shared__ uint32_t s_max;
    const int64_t M = P->M;
    const int64_t per = (M + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < M ? lo + per : M;
    // the table in use: twice the block's cells (at least 64 slots, at most
    // kAggSlots), so it stays at most half full and small runs of cells
    // (batches of scans, small clouds) clear and flush few slots
    int lg = 6;
    while (lg < 12 && (1ll << lg) < 2 * per) ++lg;
    const int slots = 1 << lg;
    static_assert(kAggSlots == 1 << 12, "table sizes up to 2^12");
    for (int i = threadIdx.x; i < slots; i += kBlock) {
        t_key[i] = -1;
        t_sum[i] = 0;
        t_min[i] = 0xFFFFFFFFu;
    }
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    const int lane = __lane_id();
    uint32_t cmax = 0;

    auto add = [&](int32_t r, uint32_t c, uint32_t m) {
        uint32_t h = ((uint32_t)r * 2654435761u) >> (32 - lg);
        for (int probe = 0; probe < 64; ++probe) {
            const int32_t prev = atomicCAS(&t_key[h], -1, r);
            if (prev == -1 || prev == r) {
                atomicAdd(&t_sum[h], c);
                atomicMin(&t_min[h], m);
                return;
            }
            h = (h + 1) & (uint32_t)(slots - 1);
        }
        atomicAdd(&csize[r], c);  // table crowded: go straight to memory
        atomicMin(&ccanon[r], m);
    };

    for (int64_t b0 = lo; b0 < hi; b0 += kBlock) {
        const int64_t A = b0 + threadIdx.x;
        const bool valid = A < hi;
        int32_t r = -1;
        uint32_t cnt = 0, mn = 0xFFFFFFFFu;
        if (valid) {
            r = cpar[A];
            const uint32_t s = cell_start[A], e = cell_start[A + 1];
            cnt = e - s;
            // the radix sort is stable and its input is in index order, so
            // a cell's words keep index order: its first is its smallest
            mn = sorig[s];
            cmax = cnt > cmax ? cnt : cmax;
        }
        const uint64_t act = __ballot(valid);
        if (act == 0) continue;
        const int leader = first_lane(act);
        const int32_t r0 = __shfl(r, leader);
        if (__ballot(valid && r == r0) == act) {
            const uint32_t c = wave_sum(cnt);
            const uint32_t m = wave_min_u32(mn);
            if (lane == leader) add(r0, c, m);
        } else if (valid) {
            add(r, cnt, mn);
        }
    }
    cmax = wave_max_u32(cmax);
    if (lane == 0) atomicMax(&s_max, cmax);
    __syncthreads();
    for (int i = threadIdx.x; i < slots; i += kBlock) {
        const int32_t r = t_key[i];
        if (r >= 0) {
            atomicAdd(&csize[r], t_sum[i]);
            atomicMin(&ccanon[r], t_min[i]);
        }
    }
    if (threadIdx.x == 0) atomicMax(&P->max_cell, (int32_t)s_max);
}

// Every label -1, in one coalesced pass: the label kernel then writes only
// the points of kept clusters.  Their writes land in scattered places of the
// caller's array (the sorted order is unrelated to the input's), where each
// costs a partial line, so on clouds whose points mostly end in filtered
// clusters the pass saves most of the label traffic.
// Every label -1: the labels of the clusters the size filter drops, and on
// a refused call (a status other than ok; no later kernel changes it) all
// of them.
__global__ __launch_bounds__(kBlock) void k_labels_clear(int32_t *__restrict__ labels, int64_t n) {
    // streaming stores, past the caches (64-frame batch: labels 0.109 ->
    // 0.100 ms, map call 3.674 -> 3.657 ms)
    typedef int i4v __attribute__((ext_vector_type(4)));
    i4v *l4 = reinterpret_cast<i4v *>(labels);
    const int64_t n4 = ((uintptr_t)labels & 15) == 0 ? n / 4 : 0;
    const i4v m1 = {-1, -1, -1, -1};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * kBlock)
        __builtin_nontemporal_store(m1, &l4[i]);
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        labels[i] = -1;
}

// Clouds below this many points write all their labels in one kernel.
constexpr int64_t kLabelsAllBelow = 131072;

// Labels in the caller's order and the number of kept clusters.  With
// several frames, each cell takes its frame's size bounds, its label counts
// from the frame's first point, and kept clusters are counted per frame.
// Only kept clusters' labels are written after k_labels_clear; with
// `write_all` (small clouds, where one launch fewer matters more than the
// scattered writes of the -1 labels) every label is, -1 included, and a
// refused call fills them all with -1 here.
__global__ __launch_bounds__(kBlock) void k_final_labels(const int32_t *__restrict__ cpar,
                                                         const uint32_t *__restrict__ cell_start,
                                                         const uint32_t *__restrict__ sorig,
                                                         const uint32_t *__restrict__ csize,
                                                         const uint32_t *__restrict__ ccanon,
                                                         int32_t *__restrict__ labels,
                                                         Frame *__restrict__ frames,
                                                         const uint32_t *__restrict__ cell_frame,
                                                         Params *__restrict__ P, int write_all) {
    if (P->status != kStatusOk) {
        if (write_all)
            for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P->n;
                 i += (int64_t)gridDim.x * kBlock)
                labels[i] = -1;
        return;
    }
    const int64_t M = P->M;
    const int nframes = P->nframes;
    const bool batched = nframes > 1;
    const int lane = __lane_id();
    uint32_t kept = 0;
    const uint32_t lo_one = (uint32_t)P->min_size, hi_one = (uint32_t)P->max_size;
    for (int64_t A = (int64_t)blockIdx.x * kBlock + threadIdx.x; A < M;
         A += (int64_t)gridDim.x * kBlock) {
        uint32_t lo = lo_one, hi = hi_one;
        int32_t base = 0;
        uint32_t f = 0;
        if (batched) {
            f = cell_frame[A];
            lo = (uint32_t)frames[f].min_size;
            hi = (uint32_t)frames[f].max_size;
            base = (int32_t)frames[f].off0;
        }
        const int32_t r = cpar[A];
        const uint32_t sz = csize[r];
        const bool ok = sz >= lo && sz <= hi;
        const int32_t lab = ok ? (int32_t)ccanon[r] - base : -1;
        const bool root_kept = ok && r == (int32_t)A;
        if (!batched) {
            kept += root_kept ? 1u : 0u;
        } else {
            // one atomic per wave when the wave's kept roots share a frame
            const uint64_t km = __ballot(root_kept);
            if (km) {
                const uint32_t f0 = __shfl(f, first_lane(km));
                if (__ballot(root_kept && f == f0) == km) {
                    if (lane == first_lane(km)) atomicAdd(&frames[f0].kept, (int32_t)__popcll(km));
                } else if (root_kept) {
                    atomicAdd(&frames[f].kept, 1);
                }
            }
        }
        if (!ok && !write_all) continue;  // -1 is there already (k_labels_clear)
        const uint32_t s = cell_start[A], e = cell_start[A + 1];
        for (uint32_t p = s; p < e; p += 4) {  // four loads in flight
            uint32_t o[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) o[j] = sorig[p + j < e ? p + j : e - 1];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (p + j < e) labels[o[j]] = lab;
        }
    }
    // points sorted after every cell (non-finite, or of a refused frame):
    // singletons
    const int64_t n = P->n, nvalid = P->nvalid;
    for (int64_t p = nvalid + (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kBlock) {
        const uint32_t o = sorig[p];
        uint32_t lo = lo_one, hi = hi_one;
        int32_t base = 0;
        int f = 0;
        bool accepted = true;
        if (batched) {
            f = frame_of_point(frames, nframes, (int64_t)o);
            lo = (uint32_t)frames[f].min_size;
            hi = (uint32_t)frames[f].max_size;
            base = (int32_t)frames[f].off0;
            accepted = frames[f].status == kStatusOk;
        }
        const bool one_ok = accepted && lo <= 1u && 1u <= hi;
        if (one_ok) labels[o] = (int32_t)o - base;
        else if (write_all) labels[o] = -1;
        if (!batched) kept += one_ok ? 1u : 0u;
        else if (one_ok) atomicAdd(&frames[f].kept, 1);
    }
    if (batched) return;
    kept = wave_sum(kept);
    __shared__ uint32_t s_k;
    if (threadIdx.x == 0) s_k = 0;
    __syncthreads();
    if (lane == 0 && kept) atomicAdd(&s_k, kept);
    __syncthreads();
    if (threadIdx.x == 0 && s_k) atomicAdd(&P->kept, (int32_t)s_k);
}

// The count of an empty call (nothing else to enqueue).
__global__ void k_set_count(int32_t *__restrict__ k_out, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *k_out = v;
}

hipError_t launch_set_count(int32_t *k_out, int32_t v, hipStream_t st) {
    k_set_count<<<1, 64, 0, st>>>(k_out, v);
    return hipGetLastError();
}

// Per frame: kept clusters, or the frame's (else the call's) failure status.
__global__ __launch_bounds__(kBlock) void k_finish(const Params *__restrict__ P,
                                                   const Frame *__restrict__ frames, int nframes,
                                                   int32_t *__restrict__ k_out) {
    if (!k_out) return;
    for (int f = blockIdx.x * kBlock + threadIdx.x; f < nframes; f += gridDim.x * kBlock) {
        int32_t v;
        if (P->status != kStatusOk) v = P->status;
        else if (nframes == 1) v = P->kept;
        else v = frames[f].status != kStatusOk ? frames[f].status : frames[f].kept;
        k_out[f] = v;
    }
}

// ------------------------------------------------------------------ host side

namespace {
std::atomic<int32_t> g_cell_blocks{kDefaultCellBlocks};
std::atomic<int32_t> g_stream_blocks{kDefaultStreamBlocks};
std::atomic<int32_t> g_radix_bits{kDefaultRadixBits};
std::atomic<int32_t> g_hook_block{kDefaultHookBlock};
std::atomic<int32_t> g_near_sampling{0};
}  // namespace

Tuning tuning() {
    return Tuning{g_cell_blocks.load(std::memory_order_relaxed),
                  g_stream_blocks.load(std::memory_order_relaxed),
                  g_radix_bits.load(std::memory_order_relaxed),
                  g_hook_block.load(std::memory_order_relaxed),
                  g_near_sampling.load(std::memory_order_relaxed)};
}

void set_tuning(Tuning t) {
    g_cell_blocks.store(t.cell_blocks, std::memory_order_relaxed);
    g_stream_blocks.store(t.stream_blocks, std::memory_order_relaxed);
    g_radix_bits.store(t.radix_bits, std::memory_order_relaxed);
    g_hook_block.store(t.hook_block, std::memory_order_relaxed);
    g_near_sampling.store(t.near_sampling, std::memory_order_relaxed);
}

const char *stage_name(int s) {
    static const char *names[kNumStages] = {
        "bbox",       "plan",      "keys",       "sort_hist",   "sort_scan",    "sort_scatter",
        "gather",     "tile_scan", "cells",      "colgrid",     "runs",         "sample",
        "giant_0",    "hook_near",
        "deferred",   "compress_1", "giant",     "work_list",  "hook_far",    "compress_2",
        "final_cells", "final_labels", "finish"};
    return (s >= 0 && s < kNumStages) ? names[s] : "";
}

// One radix pass of W-bit digits over key bits [bit0, bit0 + W): counts (the
// first pass's come from the keys kernel), per-digit scans, scatter.
template <int W>
static hipError_t launch_pass(int pass, int bit0, const uint64_t *src, uint64_t *dst,
                              const uint32_t *srcv, uint32_t *dstv, const Params *P, int64_t n,
                              int64_t ntiles, int64_t pitch, uint32_t *th, uint32_t *dtot,
                              hipStream_t st, Timer *timer) {
    hipError_t e;
    if (pass > 0) {
        if (timer) timer->begin(kStSortHist, st);
        k_sort_hist<W><<<(unsigned)ntiles, kBlock, 0, st>>>(src, P, pass, bit0, n, pitch, th);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (timer) timer->end(kStSortHist, st);
    }
    if (timer) timer->begin(kStSortScan, st);
    k_sort_scan<<<1u << W, kBlock, 0, st>>>(P, pass, ntiles, pitch, th, dtot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (timer) timer->end(kStSortScan, st);
    if (timer) timer->begin(kStSort, st);
    k_sort_scatter<W><<<(unsigned)ntiles, kBlock, 0, st>>>(src, dst, srcv, dstv, P, pass, bit0, n,
                                                         pitch, th, dtot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (timer) timer->end(kStSort, st);
    return hipSuccess;
}

// The radix passes of the schedule for RB-bit digits (pass_width /
// pass_bit0), enough for a 64-bit key (the pair-mode fallback can need one);
// passes beyond the device-side count return at once.
template <int RB>
static hipError_t launch_sort(uint64_t *keys0, uint64_t *keys1, uint32_t *vals0, uint32_t *vals1,
                              const Params *P, int64_t n, int64_t ntiles, uint32_t *th,
                              uint32_t *dtot, hipStream_t st, Timer *timer) {
    constexpr int kPasses = passes_for(RB, 64);
    const int64_t pitch = tile_pitch(ntiles);
    for (int pass = 0; pass < kPasses; ++pass) {
        const uint64_t *src = (pass & 1) ? keys1 : keys0;
        uint64_t *dst = (pass & 1) ? keys0 : keys1;
        const uint32_t *srcv = (pass & 1) ? vals1 : vals0;
        uint32_t *dstv = (pass & 1) ? vals0 : vals1;
        const int bit0 = pass_bit0(RB, pass);
        hipError_t e;
        if (pass_width(RB, pass) == RB)
            e = launch_pass<RB>(pass, bit0, src, dst, srcv, dstv, P, n, ntiles, pitch, th, dtot,
                                st, timer);
        else  // the 10-bit passes after the first four at 9 bits
            e = launch_pass<10>(pass, bit0, src, dst, srcv, dstv, P, n, ntiles, pitch, th, dtot,
                                st, timer);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_pipeline(const CallArgs &args, void *ws, const Layout &L, hipStream_t st,
                           Timer *timer) {
    const float *xyz = args.xyz;
    const int64_t n = args.n;
    const int nframes = args.nframes;
    int32_t *labels_out = args.labels_out;
    char *w = static_cast<char *>(ws);
    Params *P = reinterpret_cast<Params *>(w + L.params);
    Frame *frames = reinterpret_cast<Frame *>(w + L.frames);
    float *partials = reinterpret_cast<float *>(w + L.partials);
    uint32_t *tile_cnt = reinterpret_cast<uint32_t *>(w + L.tile_cnt);
    uint32_t *tile_off = reinterpret_cast<uint32_t *>(w + L.tile_off);
    uint64_t *keys0 = reinterpret_cast<uint64_t *>(w + L.keys0);
    uint64_t *keys1 = reinterpret_cast<uint64_t *>(w + L.keys1);
    uint32_t *vals0 = reinterpret_cast<uint32_t *>(w + L.vals0);
    uint32_t *vals1 = reinterpret_cast<uint32_t *>(w + L.vals1);
    uint32_t *th = reinterpret_cast<uint32_t *>(w + L.th);
    uint32_t *dtot = reinterpret_cast<uint32_t *>(w + L.dtot);
    float4 *spts = reinterpret_cast<float4 *>(w + L.spts);
    uint32_t *sorig = reinterpret_cast<uint32_t *>(w + L.sorig);
    uint32_t *cell_start = reinterpret_cast<uint32_t *>(w + L.cell_start);
    uint64_t *cell_key = reinterpret_cast<uint64_t *>(w + L.cell_key);
    int32_t *cpar = reinterpret_cast<int32_t *>(w + L.cpar);
    uint32_t *csize = reinterpret_cast<uint32_t *>(w + L.csize);
    uint32_t *ccanon = reinterpret_cast<uint32_t *>(w + L.ccanon);
    uint64_t *col_key = reinterpret_cast<uint64_t *>(w + L.col_key);
    uint32_t *col_cell = reinterpret_cast<uint32_t *>(w + L.col_cell);
    uint32_t *colgrid = reinterpret_cast<uint32_t *>(w + L.colgrid);
    uint32_t *colbits = reinterpret_cast<uint32_t *>(w + L.colbits);
    uint8_t *heads = reinterpret_cast<uint8_t *>(w + L.heads);
    int32_t *blkhead = reinterpret_cast<int32_t *>(w + L.blkhead);
    uint64_t *gbits = reinterpret_cast<uint64_t *>(w + L.gbits);
    uint32_t *listcnt = reinterpret_cast<uint32_t *>(w + L.listcnt);
    uint32_t *work = reinterpret_cast<uint32_t *>(w + L.work);
    uint64_t *defer = reinterpret_cast<uint64_t *>(w + L.defer);
    uint32_t *runq = reinterpret_cast<uint32_t *>(w + L.runq);
    uint32_t *cell_frame = nframes > 1 ? reinterpret_cast<uint32_t *>(w + L.cell_frame) : nullptr;

    const int64_t ntiles = L.ntiles;
    const int bbox_pf = L.bbox_per_frame;
    int64_t nb_pts = (n + kBlock - 1) / kBlock;
    const Tuning tn = tuning();
    const int nb_stream =
        (int)(nb_pts > tn.stream_blocks ? tn.stream_blocks : (nb_pts < 1 ? 1 : nb_pts));
    const int nb_cells =
        (int)(nb_pts > tn.cell_blocks ? tn.cell_blocks : (nb_pts < 1 ? 1 : nb_pts));
    const int nb_finish = (nframes + kBlock - 1) / kBlock;
    const int nb_list = nb_cells < kListBlocks ? nb_cells : kListBlocks;
    const int radix_bits = tn.radix_bits < kMinRadixBits
                               ? kMinRadixBits
                               : (tn.radix_bits > kMaxRadixBits ? kMaxRadixBits : tn.radix_bits);
    const int hook_block = tn.hook_block == 64 || tn.hook_block == 128 ? tn.hook_block : 256;

#define FEC_LAUNCH(stage, ...)                         \
    do {                                               \
        if (timer) timer->begin(stage, st);            \
        __VA_ARGS__;                                   \
        hipError_t e_ = hipGetLastError();             \
        if (e_ != hipSuccess) return e_;               \
        if (timer) timer->end(stage, st);              \
    } while (0)

    FEC_LAUNCH(kStBbox, k_bbox<<<(unsigned)(nframes * bbox_pf), kBlock, 0, st>>>(
                            xyz, n, args.offsets, bbox_pf, partials));
    FEC_LAUNCH(kStPlan, k_plan<<<1, kBlock, 0, st>>>(partials, bbox_pf, P, frames, nframes, n,
                                                      args.offsets, args.d_arr, args.min_arr,
                                                      args.max_arr, args.d, args.min_size,
                                                      args.max_size, L.colgrid_cap, radix_bits));
    {
        hipError_t e = hipSuccess;
        const int64_t pitch = tile_pitch(ntiles);
#define FEC_KEYS_SORT(RB)                                                                     \
    FEC_LAUNCH(kStKeys, k_keys<RB><<<(unsigned)ntiles, kBlock, 0, st>>>(                      \
                            xyz, P, frames, nframes, n, pitch, keys0, vals0, th));            \
    e = launch_sort<RB>(keys0, keys1, vals0, vals1, P, n, ntiles, th, dtot, st, timer)
        switch (radix_bits) {
            case 8: FEC_KEYS_SORT(8); break;
            case 9: FEC_KEYS_SORT(9); break;
            case 10: FEC_KEYS_SORT(10); break;
            default: FEC_KEYS_SORT(11); break;
        }
#undef FEC_KEYS_SORT
        if (e != hipSuccess) return e;
    }
    FEC_LAUNCH(kStGather, k_gather<<<(unsigned)ntiles, kBlock, 0, st>>>(
                              xyz, keys0, keys1, vals0, vals1, colbits, P, spts, sorig,
                              tile_cnt));
    FEC_LAUNCH(kStTileScan, k_tile_scan<<<1, 1024, 0, st>>>(tile_cnt, tile_off, ntiles, P));
    FEC_LAUNCH(kStCells, k_cells<<<(unsigned)ntiles, kBlock, 0, st>>>(
                             keys0, keys1, P, tile_off, cell_start, cell_key, col_key, col_cell,
                             cpar, csize, ccanon, frames, cell_frame,
                             reinterpret_cast<uint64_t *>(colgrid)));
    FEC_LAUNCH(kStColGrid, k_colgrid<<<nb_cells, kBlock, 0, st>>>(col_key, col_cell, cell_start,
                                                                   colgrid, colbits, P));
    // runs, near shell, giant component, far shell
    FEC_LAUNCH(kStRuns, k_runs1<<<(unsigned)ntiles, kBlock, 0, st>>>(
                            spts, cell_start, cell_key, heads, blkhead, runq, frames, cell_frame,
                            P));
    FEC_LAUNCH(kStRuns, k_runs2<<<(unsigned)ntiles, kBlock, 0, st>>>(heads, blkhead, cpar, P));
    // Each shell has large-table and small-table forms; which one a call
    // needs is known on the device only, so both are launched and the other
    // returns at once.  Cells and work cells never outnumber points, so below
    // the thresholds in points the large forms cannot be meant and are not
    // launched (two launches fewer on small clouds).  Whether the near shell
    // takes the sampling links is decided here, by the number of points.
#define FEC_HOOK_NEAR(MODE, BLK, GRID)                                                     \
    FEC_LAUNCH(MODE == kNearSample ? kStSample : kStHookNear,                               \
               k_hook_near<MODE, BLK><<<GRID, BLK, 0, st>>>(                                \
                   spts, cell_start, cell_key, col_key, col_cell, colgrid, colbits, gbits,  \
                   work, frames, cell_frame, cpar, P, defer, L.defer_cap))
#define FEC_HOOK_NEAR_ALL(MODE, GRID)                                                      \
    do {                                                                                   \
        if (hook_block == 64) FEC_HOOK_NEAR(MODE, 64, GRID);                               \
        else if (hook_block == 128) FEC_HOOK_NEAR(MODE, 128, GRID);                        \
        else FEC_HOOK_NEAR(MODE, 256, GRID);                                               \
    } while (0)
#define FEC_HOOK_FAR(SPLIT, OCC, BLK)                                                      \
    FEC_LAUNCH(kStHookFar, k_hook_far<SPLIT, OCC, BLK><<<nb_cells, BLK, 0, st>>>(            \
                               spts, cell_start, cell_key, col_key, col_cell, colgrid,       \
                               colbits, gbits, work, frames, cell_frame, cpar, P, defer,     \
                               L.defer_cap))
    const bool sampled =
        n >= kNearSplitBelow &&
        (tn.near_sampling == 1 || (tn.near_sampling == 0 && n / nframes >= kSampleMinPoints));
    if (n >= kNearSplitBelow && !sampled) {
        FEC_HOOK_NEAR_ALL(kNearAllOcc, nb_cells);
        FEC_HOOK_NEAR_ALL(kNearAll, nb_cells);
    }
    if (sampled) {
        // sampling links, their giant component and work list, then the near
        // shell on that list
        FEC_HOOK_NEAR_ALL(kNearSample, nb_cells);
        FEC_LAUNCH(kStGiant0, k_compress<<<nb_cells, kBlock, 0, st>>>(cpar, P, kNearSplitBelow));
        FEC_LAUNCH(kStGiant0, k_giant<<<(unsigned)nframes, 1024, 0, st>>>(cpar, frames, P,
                                                                          kNearSplitBelow));
        FEC_LAUNCH(kStGiant0, k_giant_bits<<<nb_list, kBlock, 0, st>>>(cpar, gbits, listcnt, frames,
                                                                        cell_frame, P, 0));
        FEC_LAUNCH(kStGiant0, k_work_list<<<nb_list, kBlock, 0, st>>>(gbits, listcnt, work, P, 0));
        FEC_HOOK_NEAR_ALL(kNearWorkOcc, nb_cells);
        FEC_HOOK_NEAR_ALL(kNearWork, nb_cells);
    }
    FEC_HOOK_NEAR_ALL(kNearSplit, nb_cells);
    FEC_LAUNCH(kStDeferred, k_deferred<<<nb_cells, kBlock, 0, st>>>(
                                spts, cell_start, frames, cell_frame, cpar, P, defer,
                                L.defer_cap, runq, 0));
    FEC_LAUNCH(kStCompress1, k_compress<<<nb_cells, kBlock, 0, st>>>(cpar, P, 0));
    FEC_LAUNCH(kStGiant, k_giant<<<(unsigned)nframes, 1024, 0, st>>>(cpar, frames, P, 0));
    FEC_LAUNCH(kStWorkList, k_giant_bits<<<nb_list, kBlock, 0, st>>>(cpar, gbits, listcnt, frames,
                                                                      cell_frame, P, 1));
    FEC_LAUNCH(kStWorkList, k_work_list<<<nb_list, kBlock, 0, st>>>(gbits, listcnt, work, P, 1));
    if (n >= (int64_t)kFarSplitBelow) {
        if (hook_block == 64) {
            FEC_HOOK_FAR(false, true, 64);
            FEC_HOOK_FAR(false, false, 64);
        } else if (hook_block == 128) {
            FEC_HOOK_FAR(false, true, 128);
            FEC_HOOK_FAR(false, false, 128);
        } else {
            FEC_HOOK_FAR(false, true, 256);
            FEC_HOOK_FAR(false, false, 256);
        }
    }
    if (hook_block == 64) FEC_HOOK_FAR(true, false, 64);
    else if (hook_block == 128) FEC_HOOK_FAR(true, false, 128);
    else FEC_HOOK_FAR(true, false, 256);
#undef FEC_HOOK_NEAR
#undef FEC_HOOK_NEAR_ALL
#undef FEC_HOOK_FAR
    FEC_LAUNCH(kStDeferred, k_deferred<<<nb_cells, kBlock, 0, st>>>(
                                spts, cell_start, frames, cell_frame, cpar, P, defer,
                                L.defer_cap, runq, 1));
    FEC_LAUNCH(kStCompress2, k_compress<<<nb_cells, kBlock, 0, st>>>(cpar, P, 0));
    FEC_LAUNCH(kStFinalCells, k_final_cells<<<nb_cells, kBlock, 0, st>>>(
                                  cpar, cell_start, sorig, csize, ccanon, P));
    // small clouds: one label kernel that writes every label
    const int labels_all = n < kLabelsAllBelow ? 1 : 0;
    if (!labels_all)
        FEC_LAUNCH(kStFinalLabels, k_labels_clear<<<nb_stream, kBlock, 0, st>>>(labels_out, n));
    FEC_LAUNCH(kStFinalLabels, k_final_labels<<<nb_cells, kBlock, 0, st>>>(
                                   cpar, cell_start, sorig, csize, ccanon, labels_out, frames,
                                   cell_frame, P, labels_all));
    FEC_LAUNCH(kStFinish, k_finish<<<(unsigned)nb_finish, kBlock, 0, st>>>(P, frames, nframes,
                                                                           args.k_out));
#undef FEC_LAUNCH
    return hipSuccess;
}

}  // namespace fec
