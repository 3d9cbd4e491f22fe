// Fixed-radius Euclidean clustering on gfx950: the device pipeline.
//
// The result is the clustering of Sec. 2.2 (Eq. (1), Alg. 1): connected
// components of the graph that joins points closer than d, then the inclusive
// min/max size filter, labels = smallest member index.  The paper's serial
// point-wise loop is replaced by a grid-based design:
//
//   bbox -> plan -> keys(+digit histograms) -> radix sort passes -> gather
//   -> cell table -> column hash -> hook (near shell) -> compress
//   -> hook (far shell) -> compress -> cluster sizes/ids -> labels
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
// compression most of a dense surface is one component and the far shell
// (offsets of 2) is mostly skipped by the root comparison.
//
// Determinism.  The union-find always hooks the larger root under the
// smaller; the partition it reaches is the unique set of components, and the
// labels (smallest original index per component) do not depend on timing.

#include "fec_internal.h"

#include <float.h>
#include <math.h>

namespace fec {

// ------------------------------------------------------------------ helpers

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

template <class T>
__device__ __forceinline__ T ld_relaxed(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ void st_relaxed(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
// Per-block min/max of the finite points and their count.
__global__ __launch_bounds__(kBlock) void k_bbox(const float *__restrict__ xyz, int64_t n,
                                                 float *__restrict__ partials) {
    float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY;
    float hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    uint32_t cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (finite3(x, y, z)) {
            lo0 = fminf(lo0, x); lo1 = fminf(lo1, y); lo2 = fminf(lo2, z);
            hi0 = fmaxf(hi0, x); hi1 = fmaxf(hi1, y); hi2 = fmaxf(hi2, z);
            ++cnt;
        }
    }
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
// Reduces the partial boxes and fixes the grid, the key layout and the
// number of radix passes.  One block.
__global__ __launch_bounds__(kBlock) void k_plan(const float *__restrict__ partials, int nparts,
                                                 Params *__restrict__ P, int64_t n, float d,
                                                 int32_t min_size, int32_t max_size) {
    float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY;
    float hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    uint64_t cnt = 0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) {
        const float *q = partials + (size_t)b * 8;
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
    __shared__ float s[kBlock / 64][6];
    __shared__ uint64_t sc[kBlock / 64];
    const int wave = threadIdx.x >> 6;
    if (__lane_id() == 0) {
        s[wave][0] = lo0; s[wave][1] = lo1; s[wave][2] = lo2;
        s[wave][3] = hi0; s[wave][4] = hi1; s[wave][5] = hi2;
        sc[wave] = cnt;
    }
    for (int i = threadIdx.x; i < kMaxPasses * kRadix; i += kBlock) (&P->hist[0][0])[i] = 0;
    if (threadIdx.x < kMaxPasses) P->ticket[threadIdx.x] = 0;
    __syncthreads();
    if (threadIdx.x != 0) return;

    float r[6] = {s[0][0], s[0][1], s[0][2], s[0][3], s[0][4], s[0][5]};
    uint64_t c = sc[0];
    for (int w = 1; w < kBlock / 64; ++w) {
        for (int a = 0; a < 3; ++a) r[a] = fminf(r[a], s[w][a]);
        for (int a = 3; a < 6; ++a) r[a] = fmaxf(r[a], s[w][a]);
        c += sc[w];
    }
    P->n = n;
    P->d = d;
    P->d2 = __fmul_rn(d, d);
    P->min_size = min_size < 1 ? 1 : min_size;
    P->max_size = max_size;
    P->status = kStatusOk;
    P->nvalid = (int64_t)c;
    P->kept = 0;
    P->M = 0;
    P->Mcol = 0;
    P->max_cell = 0;

    const double side = (double)d * (1.0 - 0x1p-10) / sqrt(3.0);
    const double inv = 1.0 / side;
    P->inv_s = inv;
    int64_t N3[3] = {1, 1, 1};
    double o3[3] = {0.0, 0.0, 0.0};
    if (c > 0) {
        for (int a = 0; a < 3; ++a) {
            o3[a] = (double)r[a];
            const double ext = ((double)r[a + 3] - (double)r[a]) * inv;
            if (!(ext < 0x1p31)) {
                P->status = kStatusRange;
            } else {
                N3[a] = (int64_t)floor(ext) + 1;
            }
        }
    }
    P->ox = o3[0]; P->oy = o3[1]; P->oz = o3[2];
    P->NX = N3[0]; P->NY = N3[1]; P->NZ = N3[2];
    P->bx = bits_for(N3[0]);
    P->by = bits_for(N3[1]);
    P->bz = bits_for(N3[2]);
    const int B = P->bx + P->by + P->bz;
    const int kb = B + (((int64_t)c < n) ? 1 : 0);
    int ib = bits_for(n);
    if (ib < 1) ib = 1;
    P->key_bits = kb;
    P->idx_bits = ib;
    P->idx_mask = (1ull << ib) - 1;
    // One 64-bit word per point when key and index fit together, otherwise
    // separate key and index arrays; beyond a 64-bit key the grid is refused.
    P->pair_mode = (kb + ib > 64) ? 1 : 0;
    P->key_shift = P->pair_mode ? 0 : ib;
    if (kb > 64) P->status = kStatusRange;
    P->npasses = P->status == kStatusOk ? (kb + kRadixBits - 1) / kRadixBits : 0;
}

// ------------------------------------------------------------- 3. keys
// Packs (cell key << idx_bits) | point index, counts the radix digits of
// every pass, and clears the first look-back buffer.
__global__ __launch_bounds__(kBlock) void k_keys(const float *__restrict__ xyz,
                                                 Params *__restrict__ P,
                                                 uint64_t *__restrict__ keys,
                                                 uint32_t *__restrict__ vals,
                                                 uint64_t *__restrict__ lb0, int64_t lb_words) {
    __shared__ uint32_t sh[kMaxPasses][kRadix];
    if (P->status != kStatusOk) return;
    for (int i = threadIdx.x; i < kMaxPasses * kRadix; i += kBlock) (&sh[0][0])[i] = 0;
    __syncthreads();
    const int64_t n = P->n;
    const int np = P->npasses;
    const int ks = P->key_shift;
    const bool pair = P->pair_mode != 0;
    const double ox = P->ox, oy = P->oy, oz = P->oz, inv = P->inv_s;
    const int64_t NX = P->NX, NY = P->NY, NZ = P->NZ;
    const int by = P->by, bz = P->bz;
    const uint64_t invalid_key = 1ull << (P->bx + by + bz);
    const int lane = __lane_id();
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        uint64_t key;
        if (finite3(x, y, z)) {
            int64_t cx = (int64_t)floor(((double)x - ox) * inv);
            int64_t cy = (int64_t)floor(((double)y - oy) * inv);
            int64_t cz = (int64_t)floor(((double)z - oz) * inv);
            cx = cx < 0 ? 0 : (cx >= NX ? NX - 1 : cx);
            cy = cy < 0 ? 0 : (cy >= NY ? NY - 1 : cy);
            cz = cz < 0 ? 0 : (cz >= NZ ? NZ - 1 : cz);
            key = ((uint64_t)cx << (by + bz)) | ((uint64_t)cy << bz) | (uint64_t)cz;
        } else {
            key = invalid_key;
        }
        const uint64_t e = pair ? key : ((key << ks) | (uint64_t)i);
        keys[i] = e;
        if (pair) vals[i] = (uint32_t)i;
        const uint64_t act = __ballot(1);
        const int leader = first_lane(act);
        for (int p = 0; p < np; ++p) {
            const uint32_t dg = (uint32_t)(e >> (ks + p * kRadixBits)) & (kRadix - 1);
            const uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
            if (__ballot(dg == d0) == act) {
                if (lane == leader) atomicAdd(&sh[p][d0], (uint32_t)__popcll(act));
            } else {
                atomicAdd(&sh[p][dg], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np * kRadix; i += kBlock) {
        const uint32_t v = (&sh[0][0])[i];
        if (v) atomicAdd(&(&P->hist[0][0])[i], v);
    }
    for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < lb_words;
         w += (int64_t)gridDim.x * kBlock)
        lb0[w] = 0;
}

// ------------------------------------------------------------- 4. sort
// One stable LSD radix pass over the packed (key, index) words with a
// decoupled look-back across tiles.  Tiles are claimed in launch order from
// a counter, so every tile a block waits for belongs to a block that is
// already running.  The wait is bounded; on timeout the call fails with a
// device status instead of hanging.
constexpr uint32_t kSpinLimit = 1u << 22;

__global__ __launch_bounds__(kBlock) void k_sort_pass(const uint64_t *__restrict__ src,
                                                      uint64_t *__restrict__ dst,
                                                      const uint32_t *__restrict__ srcv,
                                                      uint32_t *__restrict__ dstv,
                                                      Params *__restrict__ P,
                                                      uint64_t *__restrict__ lb_cur,
                                                      uint64_t *__restrict__ lb_next, int pass,
                                                      int64_t n, int64_t ntiles) {
    if (pass >= P->npasses || P->status != kStatusOk) return;
    __shared__ uint32_t s_cnt[kBlock / 64][kRadix];
    __shared__ uint32_t s_base[kRadix];
    __shared__ uint32_t s_tmp[kBlock / 64];
    __shared__ uint32_t s_tile;
    __shared__ int s_fail;
    const int tid = threadIdx.x, wave = tid >> 6, lane = __lane_id();

    for (int64_t w = (int64_t)blockIdx.x * kBlock + tid; w < ntiles * kRadix;
         w += (int64_t)gridDim.x * kBlock)
        lb_next[w] = 0;
    for (int i = tid; i < (kBlock / 64) * kRadix; i += kBlock) (&s_cnt[0][0])[i] = 0;
    if (tid == 0) {
        s_tile = atomicAdd(&P->ticket[pass], 1u);
        s_fail = 0;
    }
    __syncthreads();
    const int64_t tile = s_tile;
    const int shift = P->key_shift + pass * kRadixBits;
    const bool pair = P->pair_mode != 0;
    const int64_t base = tile * kTile + (int64_t)wave * (64 * kItems);

    uint64_t v[kItems];
    uint32_t rk[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t e = base + k * 64 + lane;
        v[k] = e < n ? src[e] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const bool valid = base + k * 64 + lane < n;
        const uint32_t dg = (uint32_t)(v[k] >> shift) & (kRadix - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lanemask_lt());
        const uint32_t prev = s_cnt[wave][dg];
        rk[k] = prev + below;
        if (valid && below == 0) s_cnt[wave][dg] = prev + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    // per digit (thread = digit): wave offsets inside the tile, tile count
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const uint32_t c = s_cnt[w][tid];
        s_cnt[w][tid] = run;
        run += c;
    }
    const uint32_t tcount = run;
    uint64_t *mine = lb_cur + tile * kRadix + tid;
    uint64_t excl = 0;
    if (tile == 0) {
        st_relaxed(mine, kLbInclusive | (uint64_t)tcount);
    } else {
        st_relaxed(mine, kLbAggregate | (uint64_t)tcount);
        int64_t j = tile - 1;
        uint32_t spins = 0;
        while (true) {
            const uint64_t w = ld_relaxed(lb_cur + j * kRadix + tid);
            const uint64_t f = w & ~kLbValue;
            if (f == 0) {
                if (++spins > kSpinLimit) {
                    s_fail = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += w & kLbValue;
            if (f == kLbInclusive) break;
            if (--j < 0) {
                s_fail = 1;
                break;
            }
        }
        st_relaxed(mine, kLbInclusive | (excl + tcount));
    }
    // global digit base: exclusive scan of the pass histogram
    uint32_t tot;
    const uint32_t hb = block_excl_scan(P->hist[pass][tid], s_tmp, tot);
    s_base[tid] = hb + (uint32_t)excl;
    __syncthreads();
    if (s_fail) {
        if (tid == 0) atomicExch(&P->status, kStatusDevice);
        return;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t e = base + k * 64 + lane;
        if (e < n) {
            const uint32_t dg = (uint32_t)(v[k] >> shift) & (kRadix - 1);
            const uint64_t pos = (uint64_t)s_base[dg] + s_cnt[wave][dg] + rk[k];
            if (pos < (uint64_t)n) {
                dst[pos] = v[k];
                if (pair) dstv[pos] = srcv[e];
            }
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
    const int64_t base = (int64_t)blockIdx.x * kTile;
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
            spts[e] = make_float4(x, y, z, __uint_as_float(i));
            sorig[e] = i;
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
        tile_cnt[2 * blockIdx.x] = t1;
        tile_cnt[2 * blockIdx.x + 1] = t2;
    }
}

// ------------------------------------------------------------- 6. tile scan
// Exclusive scan of the per-tile cell / column counts (one block).
__global__ __launch_bounds__(1024) void k_tile_scan(const uint32_t *__restrict__ tile_cnt,
                                                    uint32_t *__restrict__ tile_off,
                                                    int64_t ntiles, Params *__restrict__ P) {
    if (P->status != kStatusOk) return;
    __shared__ uint32_t s_a[1024], s_b[1024];
    const int tid = threadIdx.x;
    const int64_t per = (ntiles + 1023) / 1024;
    const int64_t lo = tid * per, hi = lo + per < ntiles ? lo + per : ntiles;
    uint32_t sa = 0, sb = 0;
    for (int64_t t = lo; t < hi; ++t) {
        sa += tile_cnt[2 * t];
        sb += tile_cnt[2 * t + 1];
    }
    s_a[tid] = sa;
    s_b[tid] = sb;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t xa = tid >= o ? s_a[tid - o] : 0u, xb = tid >= o ? s_b[tid - o] : 0u;
        __syncthreads();
        s_a[tid] += xa;
        s_b[tid] += xb;
        __syncthreads();
    }
    uint32_t ra = s_a[tid] - sa, rb = s_b[tid] - sb;
    for (int64_t t = lo; t < hi; ++t) {
        tile_off[2 * t] = ra;
        tile_off[2 * t + 1] = rb;
        ra += tile_cnt[2 * t];
        rb += tile_cnt[2 * t + 1];
    }
    if (tid == 1023) {
        P->M = s_a[1023];
        P->Mcol = s_b[1023];
        if ((int64_t)s_a[1023] > P->nvalid || s_b[1023] > s_a[1023]) {
            P->status = kStatusDevice;  // inconsistent counts: stop before any table use
            P->M = 0;
            P->Mcol = 0;
        }
    }
}

// ------------------------------------------------------------- 7. cells
// Cell table (first sorted position and key of every occupied cell, and
// its column) and column table (key (cx, cy) and first cell of every
// occupied column), plus the per-cell union-find / size / id slots.
__global__ __launch_bounds__(kBlock) void k_cells(const uint64_t *__restrict__ s0,
                                                  const uint64_t *__restrict__ s1,
                                                  const Params *__restrict__ P,
                                                  const uint32_t *__restrict__ tile_off,
                                                  uint32_t *__restrict__ cell_start,
                                                  uint64_t *__restrict__ cell_key,
                                                  uint32_t *__restrict__ cell_col,
                                                  uint64_t *__restrict__ col_key,
                                                  uint32_t *__restrict__ col_cell,
                                                  int32_t *__restrict__ cpar,
                                                  uint32_t *__restrict__ csize,
                                                  uint32_t *__restrict__ ccanon) {
    if (P->status != kStatusOk) return;
    const uint64_t *srt = (P->npasses & 1) ? s1 : s0;
    const int64_t nvalid = P->nvalid;
    const int ks = P->key_shift, bz = P->bz;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int wave = threadIdx.x >> 6, lane = __lane_id();
    __shared__ uint32_t s_tot[kItems][kBlock / 64];
    __shared__ uint32_t s_ctot[kItems][kBlock / 64];
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
            s_tot[k][wave] = (uint32_t)__popcll(m);
            s_ctot[k][wave] = (uint32_t)__popcll(mc);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0, crun = 0;
        for (int k = 0; k < kItems; ++k)
            for (int w = 0; w < kBlock / 64; ++w) {
                const uint32_t t = s_tot[k][w], c = s_ctot[k][w];
                s_tot[k][w] = run;
                s_ctot[k][w] = crun;
                run += t;
                crun += c;
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
            const uint32_t cid = c0 + s_tot[k][wave] + (uint32_t)__popcll(m & lt);
            const uint32_t colx = q0 + s_ctot[k][wave] + (uint32_t)__popcll(mc & lt);
            if ((int64_t)cid >= nvalid) continue;
            const uint64_t key = srt[e] >> ks;
            cell_start[cid] = (uint32_t)e;
            cell_key[cid] = key;
            cell_col[cid] = cf ? colx : colx - 1;
            cpar[cid] = (int32_t)cid;
            csize[cid] = 0;
            ccanon[cid] = 0xFFFFFFFFu;
            if (cf) {
                col_key[colx] = key >> bz;
                col_cell[colx] = cid;
            }
        }
    }
}

// ------------------------------------------------------------- 8. column rows
// For every column (cx, cy), the first column of rows cx+1 and cx+2 whose
// cy' >= cy - 2 (columns are sorted by (cx, cy), so the columns of the
// stencil in one row are consecutive from there).
__global__ __launch_bounds__(kBlock) void k_colrows(const uint64_t *__restrict__ col_key,
                                                    uint32_t *__restrict__ col_cell,
                                                    uint32_t *__restrict__ cell_start,
                                                    uint32_t *__restrict__ row_start,
                                                    const Params *__restrict__ P) {
    if (P->status != kStatusOk) return;
    const int64_t Mcol = P->Mcol;
    const int by = P->by;
    const uint64_t ymask = (1ull << by) - 1;
    const int64_t NX = P->NX;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        col_cell[Mcol] = (uint32_t)P->M;
        cell_start[P->M] = (uint32_t)P->nvalid;
    }
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < Mcol;
         c += (int64_t)gridDim.x * kBlock) {
        const uint64_t ck = col_key[c];
        const uint64_t cx = ck >> by, cy = ck & ymask;
        for (int dx = 1; dx <= 2; ++dx) {
            uint32_t rs = (uint32_t)Mcol;
            if ((int64_t)(cx + dx) < NX) {
                const uint64_t target = ((cx + dx) << by) | (cy >= 2 ? cy - 2 : 0);
                uint32_t lo = (uint32_t)c + 1, hi = (uint32_t)Mcol;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (col_key[mid] < target) lo = mid + 1;
                    else hi = mid;
                }
                rs = lo;
            }
            row_start[2 * c + dx - 1] = rs;
        }
    }
}

// ------------------------------------------------------------- 9. hooking
// Union-find over cells; parent[x] <= x always, roots are the smallest cell
// of their component.
__device__ __forceinline__ int32_t uf_find(int32_t *par, int32_t x) {
    int32_t p = ld_relaxed(par + x);
    while (p != x) {
        const int32_t gp = ld_relaxed(par + p);
        if (gp != p) st_relaxed(par + x, gp);  // path halving; any ancestor is valid
        x = gp;
        p = ld_relaxed(par + x);
    }
    return x;
}

__device__ __forceinline__ int32_t uf_find_ro(const int32_t *par, int32_t x) {
    int32_t p = ld_relaxed(par + x);
    while (p != x) {
        x = p;
        p = ld_relaxed(par + x);
    }
    return x;
}

__device__ __forceinline__ void uf_link(int32_t *par, int32_t a, int32_t b) {
    while (true) {
        a = uf_find(par, a);
        b = uf_find(par, b);
        if (a == b) return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        // hook the larger root a under the smaller root b
        if (atomicCAS(par + a, a, b) == a) return;
    }
}

// Tests the cell pair (A, B) point pair by point pair until the first
// joined pair; joins their components when one is found.  Skips pairs that
// already share a root.
__device__ __forceinline__ void hook_pair(int32_t A, int32_t B, uint32_t sA, uint32_t eA,
                                          const float4 *__restrict__ spts,
                                          const uint32_t *__restrict__ cell_start,
                                          int32_t *cpar, float d2) {
    const int32_t ra = uf_find(cpar, A);
    const int32_t rb = uf_find(cpar, B);
    if (ra == rb) return;
    const uint32_t sB = cell_start[B], eB = cell_start[B + 1];
    for (uint32_t a = sA; a < eA; ++a) {
        const float4 pa = spts[a];
        for (uint32_t b = sB; b < eB; ++b) {
            if (joined(pa.x, pa.y, pa.z, spts[b], d2)) {
                uf_link(cpar, ra, rb);
                return;
            }
        }
    }
}

// One shell of the forward half of the 5x5x5 stencil around every cell.
// ROUND 0 (near): offsets with max(|dx|,|dy|,|dz|) = 1.
// ROUND 1 (far):  offsets with max(|dx|,|dy|,|dz|) = 2.
// Forward: dx > 0, or dx == 0 and dy > 0, or dx == dy == 0 and dz > 0.
template <int ROUND>
__global__ __launch_bounds__(kBlock) void k_hook(const float4 *__restrict__ spts,
                                                 const uint32_t *__restrict__ cell_start,
                                                 const uint64_t *__restrict__ cell_key,
                                                 const uint32_t *__restrict__ cell_col,
                                                 const uint64_t *__restrict__ col_key,
                                                 const uint32_t *__restrict__ col_cell,
                                                 const uint32_t *__restrict__ row_start,
                                                 int32_t *cpar, const Params *__restrict__ P) {
    if (P->status != kStatusOk) return;
    const int64_t M = P->M, Mcol = P->Mcol;
    const float d2 = P->d2;
    const int by = P->by, bz = P->bz;
    const uint64_t zmask = (1ull << bz) - 1, ymask = (1ull << by) - 1;
    constexpr int zr = ROUND == 0 ? 1 : 2;
    for (int64_t Ai = (int64_t)blockIdx.x * kBlock + threadIdx.x; Ai < M;
         Ai += (int64_t)gridDim.x * kBlock) {
        const int32_t A = (int32_t)Ai;
        const uint64_t key = cell_key[A];
        const int64_t cz = (int64_t)(key & zmask);
        const uint64_t ck = key >> bz;
        const int64_t cx = (int64_t)(ck >> by), cy = (int64_t)(ck & ymask);
        const uint32_t col = cell_col[A];
        const uint32_t sA = cell_start[A], eA = cell_start[A + 1];

        auto scan_column = [&](uint32_t c2, int64_t dx, int64_t dy) {
            const bool near_col = dx <= 1 && dy <= 1 && dy >= -1;
            const uint32_t b0 = col_cell[c2], b1 = col_cell[c2 + 1];
            uint32_t lo = b0, hi = b1;
            if (b1 - b0 > 8) {  // first cell with cz' >= cz - zr
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if ((int64_t)(cell_key[mid] & zmask) < cz - zr) lo = mid + 1;
                    else hi = mid;
                }
            }
            for (uint32_t B = lo; B < b1; ++B) {
                const int64_t dz = (int64_t)(cell_key[B] & zmask) - cz;
                if (dz < -zr) continue;
                if (dz > zr) break;
                if (ROUND == 1 && near_col && dz >= -1 && dz <= 1) continue;
                hook_pair(A, (int32_t)B, sA, eA, spts, cell_start, cpar, d2);
            }
        };

        // own column, cells above: dz = +zr
        for (int32_t B = A + 1; B < M && B <= A + 2; ++B) {
            const uint64_t kb = cell_key[B];
            if ((kb >> bz) != ck) break;
            const int64_t dz = (int64_t)(kb & zmask) - cz;
            if (dz > zr) break;
            if (dz == zr) hook_pair(A, B, sA, eA, spts, cell_start, cpar, d2);
        }
        // row dx = 0: columns cy+1 .. cy+zr follow this column directly
        for (uint32_t c2 = col + 1; c2 <= col + zr && (int64_t)c2 < Mcol; ++c2) {
            const uint64_t k2 = col_key[c2];
            if ((int64_t)(k2 >> by) != cx) break;
            const int64_t dy = (int64_t)(k2 & ymask) - cy;
            if (dy > zr) break;
            scan_column(c2, 0, dy);
        }
        // rows dx = 1 (and 2 in the far shell)
        for (int dx = 1; dx <= zr; ++dx) {
            for (uint32_t c2 = row_start[2 * col + dx - 1]; (int64_t)c2 < Mcol; ++c2) {
                const uint64_t k2 = col_key[c2];
                if ((int64_t)(k2 >> by) != cx + dx) break;
                const int64_t dy = (int64_t)(k2 & ymask) - cy;
                if (dy > zr) break;
                if (dy < -zr) continue;
                scan_column(c2, dx, dy);
            }
        }
    }
}

// Every cell points at its root afterwards.  Read-only finds, one writer per
// slot, so no slot is overwritten with a stale ancestor.
__global__ __launch_bounds__(kBlock) void k_compress(int32_t *cpar, const Params *__restrict__ P) {
    if (P->status != kStatusOk) return;
    const int64_t M = P->M;
    for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < M;
         x += (int64_t)gridDim.x * kBlock) {
        const int32_t r = uf_find_ro(cpar, (int32_t)x);
        st_relaxed(cpar + x, r);
    }
}

// ------------------------------------------------------------- 10. finalize
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
    for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
        t_key[i] = -1;
        t_sum[i] = 0;
        t_min[i] = 0xFFFFFFFFu;
    }
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    const int64_t M = P->M;
    const int64_t per = (M + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < M ? lo + per : M;
    const int lane = __lane_id();
    uint32_t cmax = 0;

    auto add = [&](int32_t r, uint32_t c, uint32_t m) {
        uint32_t h = ((uint32_t)r * 2654435761u) >> (32 - 12);
        for (int probe = 0; probe < 64; ++probe) {
            const int32_t prev = atomicCAS(&t_key[h], -1, r);
            if (prev == -1 || prev == r) {
                atomicAdd(&t_sum[h], c);
                atomicMin(&t_min[h], m);
                return;
            }
            h = (h + 1) & (kAggSlots - 1);
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
            for (uint32_t p = s; p < e; ++p) {
                const uint32_t o = sorig[p];
                mn = o < mn ? o : mn;
            }
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
    for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
        const int32_t r = t_key[i];
        if (r >= 0) {
            atomicAdd(&csize[r], t_sum[i]);
            atomicMin(&ccanon[r], t_min[i]);
        }
    }
    if (threadIdx.x == 0) atomicMax(&P->max_cell, (int32_t)s_max);
}

// Labels in the caller's order and the number of kept clusters.
__global__ __launch_bounds__(kBlock) void k_final_labels(const int32_t *__restrict__ cpar,
                                                         const uint32_t *__restrict__ cell_start,
                                                         const uint32_t *__restrict__ sorig,
                                                         const uint32_t *__restrict__ csize,
                                                         const uint32_t *__restrict__ ccanon,
                                                         int32_t *__restrict__ labels,
                                                         Params *__restrict__ P) {
    if (P->status != kStatusOk) return;
    const int64_t M = P->M;
    const uint32_t lo = (uint32_t)P->min_size, hi = (uint32_t)P->max_size;
    uint32_t kept = 0;
    for (int64_t A = (int64_t)blockIdx.x * kBlock + threadIdx.x; A < M;
         A += (int64_t)gridDim.x * kBlock) {
        const int32_t r = cpar[A];
        const uint32_t sz = csize[r];
        const bool ok = sz >= lo && sz <= hi;
        const int32_t lab = ok ? (int32_t)ccanon[r] : -1;
        kept += (ok && r == (int32_t)A) ? 1u : 0u;
        const uint32_t s = cell_start[A], e = cell_start[A + 1];
        for (uint32_t p = s; p < e; ++p) labels[sorig[p]] = lab;
    }
    // non-finite points (sorted after every finite one): singletons
    const int64_t n = P->n, nvalid = P->nvalid;
    const bool one_ok = lo <= 1u && 1u <= hi;
    for (int64_t p = nvalid + (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kBlock) {
        const uint32_t o = sorig[p];
        labels[o] = one_ok ? (int32_t)o : -1;
        kept += one_ok ? 1u : 0u;
    }
    kept = wave_sum(kept);
    __shared__ uint32_t s_k;
    if (threadIdx.x == 0) s_k = 0;
    __syncthreads();
    if (__lane_id() == 0 && kept) atomicAdd(&s_k, kept);
    __syncthreads();
    if (threadIdx.x == 0 && s_k) atomicAdd(&P->kept, (int32_t)s_k);
}

// On a device-side failure every label is -1.
__global__ __launch_bounds__(kBlock) void k_error_fill(int32_t *__restrict__ labels, int64_t n,
                                                       const Params *__restrict__ P) {
    if (P->status == kStatusOk) return;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        labels[i] = -1;
}

__global__ void k_finish(const Params *__restrict__ P, int32_t *__restrict__ k_out) {
    if (k_out) *k_out = P->status != kStatusOk ? P->status : P->kept;
}

// ------------------------------------------------------------------ host side

const char *stage_name(int s) {
    static const char *names[kNumStages] = {
        "bbox",      "plan",       "keys",        "sort_pass",    "gather",
        "tile_scan", "cells",      "column_rows", "hook_near",    "compress_1",
        "hook_far",  "compress_2", "final_cells", "final_labels", "finish"};
    return (s >= 0 && s < kNumStages) ? names[s] : "";
}

hipError_t launch_pipeline(const float *xyz, int64_t n, float d, int32_t min_size,
                           int32_t max_size, int32_t *labels_out, int32_t *k_out, void *ws,
                           const Layout &L, hipStream_t st, Timer *timer) {
    char *w = static_cast<char *>(ws);
    Params *P = reinterpret_cast<Params *>(w + L.params);
    float *partials = reinterpret_cast<float *>(w + L.partials);
    uint32_t *tile_cnt = reinterpret_cast<uint32_t *>(w + L.tile_cnt);
    uint32_t *tile_off = reinterpret_cast<uint32_t *>(w + L.tile_off);
    uint64_t *keys0 = reinterpret_cast<uint64_t *>(w + L.keys0);
    uint64_t *keys1 = reinterpret_cast<uint64_t *>(w + L.keys1);
    uint32_t *vals0 = reinterpret_cast<uint32_t *>(w + L.vals0);
    uint32_t *vals1 = reinterpret_cast<uint32_t *>(w + L.vals1);
    uint64_t *lb0 = reinterpret_cast<uint64_t *>(w + L.lb0);
    uint64_t *lb1 = reinterpret_cast<uint64_t *>(w + L.lb1);
    float4 *spts = reinterpret_cast<float4 *>(w + L.spts);
    uint32_t *sorig = reinterpret_cast<uint32_t *>(w + L.sorig);
    uint32_t *cell_start = reinterpret_cast<uint32_t *>(w + L.cell_start);
    uint64_t *cell_key = reinterpret_cast<uint64_t *>(w + L.cell_key);
    int32_t *cpar = reinterpret_cast<int32_t *>(w + L.cpar);
    uint32_t *csize = reinterpret_cast<uint32_t *>(w + L.csize);
    uint32_t *ccanon = reinterpret_cast<uint32_t *>(w + L.ccanon);
    uint32_t *cell_col = reinterpret_cast<uint32_t *>(w + L.cell_col);
    uint64_t *col_key = reinterpret_cast<uint64_t *>(w + L.col_key);
    uint32_t *col_cell = reinterpret_cast<uint32_t *>(w + L.col_cell);
    uint32_t *row_start = reinterpret_cast<uint32_t *>(w + L.row_start);

    const int64_t ntiles = L.ntiles;
    int nb_bbox = (int)((n + kBlock * 4 - 1) / (kBlock * 4));
    nb_bbox = nb_bbox < 1 ? 1 : (nb_bbox > kBboxBlocks ? kBboxBlocks : nb_bbox);
    int64_t nb_pts = (n + kBlock - 1) / kBlock;
    const int nb_stream = (int)(nb_pts > 8192 ? 8192 : (nb_pts < 1 ? 1 : nb_pts));
    const int nb_cells = (int)(nb_pts > kCellBlocks ? kCellBlocks : (nb_pts < 1 ? 1 : nb_pts));
    // Passes beyond the device-side count return at once; the pair-mode
    // fallback can need up to a full 64-bit key.
    const int max_passes = kMaxPasses;

#define FEC_LAUNCH(stage, ...)                         \
    do {                                               \
        if (timer) timer->begin(stage, st);            \
        __VA_ARGS__;                                   \
        hipError_t e_ = hipGetLastError();             \
        if (e_ != hipSuccess) return e_;               \
        if (timer) timer->end(stage, st);              \
    } while (0)

    FEC_LAUNCH(kStBbox, k_bbox<<<nb_bbox, kBlock, 0, st>>>(xyz, n, partials));
    FEC_LAUNCH(kStPlan, k_plan<<<1, kBlock, 0, st>>>(partials, nb_bbox, P, n, d, min_size,
                                                      max_size));
    FEC_LAUNCH(kStKeys, k_keys<<<nb_stream, kBlock, 0, st>>>(xyz, P, keys0, vals0, lb0,
                                                              ntiles * kRadix));
    for (int pass = 0; pass < max_passes; ++pass) {
        const uint64_t *src = (pass & 1) ? keys1 : keys0;
        uint64_t *dst = (pass & 1) ? keys0 : keys1;
        const uint32_t *srcv = (pass & 1) ? vals1 : vals0;
        uint32_t *dstv = (pass & 1) ? vals0 : vals1;
        uint64_t *cur = (pass & 1) ? lb1 : lb0;
        uint64_t *nxt = (pass & 1) ? lb0 : lb1;
        FEC_LAUNCH(kStSort, k_sort_pass<<<(unsigned)ntiles, kBlock, 0, st>>>(
                                src, dst, srcv, dstv, P, cur, nxt, pass, n, ntiles));
    }
    FEC_LAUNCH(kStGather, k_gather<<<(unsigned)ntiles, kBlock, 0, st>>>(
                              xyz, keys0, keys1, vals0, vals1, P, spts, sorig, tile_cnt));
    FEC_LAUNCH(kStTileScan, k_tile_scan<<<1, 1024, 0, st>>>(tile_cnt, tile_off, ntiles, P));
    FEC_LAUNCH(kStCells, k_cells<<<(unsigned)ntiles, kBlock, 0, st>>>(
                             keys0, keys1, P, tile_off, cell_start, cell_key, cell_col, col_key,
                             col_cell, cpar, csize, ccanon));
    FEC_LAUNCH(kStColumnRows, k_colrows<<<nb_cells, kBlock, 0, st>>>(col_key, col_cell,
                                                                      cell_start, row_start, P));
    FEC_LAUNCH(kStHookNear, k_hook<0><<<nb_cells, kBlock, 0, st>>>(
                                spts, cell_start, cell_key, cell_col, col_key, col_cell,
                                row_start, cpar, P));
    FEC_LAUNCH(kStCompress1, k_compress<<<nb_cells, kBlock, 0, st>>>(cpar, P));
    FEC_LAUNCH(kStHookFar, k_hook<1><<<nb_cells, kBlock, 0, st>>>(
                               spts, cell_start, cell_key, cell_col, col_key, col_cell,
                               row_start, cpar, P));
    FEC_LAUNCH(kStCompress2, k_compress<<<nb_cells, kBlock, 0, st>>>(cpar, P));
    FEC_LAUNCH(kStFinalCells, k_final_cells<<<nb_cells, kBlock, 0, st>>>(
                                  cpar, cell_start, sorig, csize, ccanon, P));
    FEC_LAUNCH(kStFinalLabels, k_final_labels<<<nb_cells, kBlock, 0, st>>>(
                                   cpar, cell_start, sorig, csize, ccanon, labels_out, P));
    FEC_LAUNCH(kStFinish, k_error_fill<<<nb_stream, kBlock, 0, st>>>(labels_out, n, P));
    FEC_LAUNCH(kStFinish, k_finish<<<1, 1, 0, st>>>(P, k_out));
#undef FEC_LAUNCH
    return hipSuccess;
}

}  // namespace fec
