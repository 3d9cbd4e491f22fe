/*
 * fec.h -- C ABI of the MI355X (gfx950) fixed-radius Euclidean clustering
 * library (the clustering of "FEC: Fast Euclidean Clustering for Point Cloud
 * Segmentation", arXiv 2208.07678).
 *
 * What is computed (Sec. 2.2, Eq. (1) and Alg. 1 of the paper):
 *   Two points p_i, p_j are joined when they are closer than d.  The test is
 *   Eq. (1)'s strict inequality evaluated in IEEE binary32, round to nearest,
 *   with no contraction and no flush-to-zero, in the fixed order
 *       dx = x_i - x_j, dy = y_i - y_j, dz = z_i - z_j,
 *       s  = (dx*dx + dy*dy) + dz*dz,        joined  <=>  s < d*d
 *   (d*d rounded to binary32).  Clusters are the connected components of
 *   the graph of joined pairs, which is the set of segments Alg. 1's
 *   point-wise loop arrives at when every point is visited and the neighbour
 *   cap Th_max is unlimited.  A point with a non-finite coordinate is joined
 *   to nothing.
 *
 * Output convention (fixed by this library; the paper labels segments in
 * discovery order 1, 2, ...):
 *   labels_out[i] = the smallest index j in i's cluster, when the cluster
 *                   size |C| satisfies min_size <= |C| <= max_size
 *                   (inclusive; min_size <= 0 acts as 1),
 *                 = -1 otherwise.
 *   The return value / *k_out is the number of clusters kept.
 *   Labels are deterministic: they do not depend on scheduling.
 *
 * Memory: every buffer argument is a DEVICE pointer on the current HIP
 * device, owned by the caller; the library never frees caller memory.
 *   xyz        float32, array-of-structures [n][3] (x, y, z), contiguous,
 *              4-byte aligned.  Read only.
 *   labels_out int32 [n].  Written.
 *
 * Status codes (negative values are errors; no kernel is launched and no
 * output is written when the host-side checks fail):
 */
#ifndef FEC_H
#define FEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FEC_OK 0
#define FEC_EINVAL (-1)  /* bad argument (checked on the host, before any launch)   */
#define FEC_ERANGE (-2)  /* the point cloud's extent needs a grid key of more than  */
                         /* 64 bits together with the point index (found on the    */
                         /* device; labels_out is then filled with -1)              */
#define FEC_ENOMEM (-3)  /* workspace allocation failed (blocking form only)        */
#define FEC_EDEVICE (-4) /* a HIP runtime call failed, or a device-side consistency */
                         /* check failed; see fec_last_error()                       */

/*
 * Blocking form.  Clusters n points with threshold d (Eq. (1)), applies the
 * inclusive [min_size, max_size] size filter and writes labels_out.
 * Runs on the stream set by fec_set_stream (default: the null stream) with a
 * workspace the library allocates on first use and keeps (grown when a
 * larger n arrives) until fec_release().  Waits for completion.
 * Returns the number of kept clusters (>= 0) or a negative FEC_* status.
 * Host-side checks (FEC_EINVAL): n < 0 or n > 2^31 - 1; d not finite, d <= 0,
 * or d*d not a normal binary32 number; min_size > max_size; xyz or
 * labels_out null while n > 0.  n == 0 returns 0 and touches nothing.
 * Not safe to call concurrently from several host threads.
 */
int32_t fec_cluster(const float *xyz, int64_t n, float d, int32_t min_size, int32_t max_size,
                    int32_t *labels_out);

/*
 * Workspace bytes fec_cluster_async needs for n points (0 for n <= 0).
 * Linear in n (about 100-140 bytes per point).
 */
size_t fec_workspace_bytes(int64_t n);

/*
 * Asynchronous form: same computation, enqueued on `stream` (a hipStream_t,
 * NULL for the null stream) with a caller-provided device workspace of at
 * least fec_workspace_bytes(n) bytes (256-byte aligned).  Returns FEC_OK once
 * the work is enqueued, or a negative status (host-side checks as for
 * fec_cluster, plus FEC_EINVAL for a null or too small workspace; FEC_EDEVICE
 * when a launch fails).  When the work completes, *k_out (a DEVICE int32, may
 * be NULL) holds the number of kept clusters or FEC_ERANGE / FEC_EDEVICE.
 * The workspace and outputs must not be used by other work until then; calls
 * on distinct workspaces may run concurrently on distinct streams.
 */
int32_t fec_cluster_async(const float *xyz, int64_t n, float d, int32_t min_size,
                          int32_t max_size, int32_t *labels_out, int32_t *k_out, void *workspace,
                          size_t workspace_bytes, void *stream);

/*
 * No-allocation form, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same computation as fec_cluster_async, enqueued on
 * `stream`, but its workspace is the library's own static device array of
 * FEC_NOALLOC_SCRATCH_BYTES bytes (one per GPU, held until the process
 * ends), so the call allocates nothing; the caller passes only the inputs
 * and outputs (DEVICE pointers as above; k_out may be NULL).
 *   n          at most FEC_NOALLOC_MAX_POINTS; larger n returns FEC_EINVAL
 *              (with the host-side checks of fec_cluster), nothing launched.
 * Returns FEC_OK once enqueued, FEC_EDEVICE when the scratch array's device
 * address cannot be obtained or a launch fails.  Every call on one GPU
 * shares that GPU's array, and each call overwrites what the previous left
 * there: calls that overlap on one GPU (on different streams, or from
 * several host threads) race and give wrong results.  Order them on one
 * stream, or synchronise between them.
 */
#define FEC_NOALLOC_MAX_POINTS 524288
#define FEC_NOALLOC_SCRATCH_BYTES (64u << 20)
int32_t fec_cluster_noalloc(const float *xyz, int64_t n, float d, int32_t min_size,
                            int32_t max_size, int32_t *labels_out, int32_t *k_out,
                            void *stream);

/*
 * Batched form: many independent clouds ("frames") in one call, each with its
 * own threshold and size bounds -- the result for every frame is exactly what
 * fec_cluster_async returns for that frame alone (same Sec. 2.2 / Eq. (1) /
 * Alg. 1 computation), but the whole batch shares one sort and one launch
 * sequence.
 *
 *   xyz        float32 [n_total][3], the frames' points one frame after the
 *              other (DEVICE, read only).
 *   offsets    int64 [nframes + 1] (DEVICE): frame f holds the points
 *              offsets[f] .. offsets[f+1]-1; offsets[0] == 0,
 *              offsets[nframes] == n_total, non-decreasing (empty frames are
 *              allowed).
 *   d          float32 [nframes] (DEVICE): the frame's threshold.
 *   min_size, max_size  int32 [nframes] (DEVICE): the frame's inclusive size
 *              bounds (min_size <= 0 acts as 1).
 *   labels_out int32 [n_total] (DEVICE, written): FRAME-LOCAL labels -- for a
 *              point of frame f, the smallest index in its cluster counted
 *              from offsets[f] (i.e. the label fec_cluster gives on that frame
 *              alone), or -1.
 *   k_out      int32 [nframes] (DEVICE, written): per frame, the number of
 *              kept clusters, or FEC_EINVAL when that frame's d / bounds fail
 *              the checks fec_cluster applies on the host (d finite, > 0,
 *              d*d a normal binary32 number, min_size <= max_size), or
 *              FEC_ERANGE when its extent needs a grid coordinate of 2^31 or
 *              more cells.  Such a frame's labels are all -1; other frames are
 *              unaffected.  When the offsets are not a partition of
 *              [0, n_total) every k_out entry is FEC_EINVAL and every label
 *              -1; when the stacked grid of all frames needs a key of more
 *              than 64 bits every entry is FEC_ERANGE.
 *   workspace  DEVICE, >= fec_batch_workspace_bytes(n_total, nframes) bytes,
 *              256-byte aligned.
 * Host-side checks (FEC_EINVAL, nothing launched): n_total outside
 * [0, 2^31 - 1]; nframes outside [1, 65536]; a null offsets, d, min_size,
 * max_size or k_out; null xyz or labels_out with n_total > 0; workspace null,
 * too small or misaligned.  Returns FEC_OK once enqueued, FEC_EDEVICE when a
 * launch fails.  Same stream / workspace rules as fec_cluster_async.
 */
int32_t fec_cluster_batch_async(const float *xyz, int64_t n_total, int32_t nframes,
                                const int64_t *offsets, const float *d, const int32_t *min_size,
                                const int32_t *max_size, int32_t *labels_out, int32_t *k_out,
                                void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes of fec_cluster_batch_async (0 for invalid sizes). */
size_t fec_batch_workspace_bytes(int64_t n_total, int32_t nframes);

/*
 * Serving engine: continuous batching of independent requests (one cloud
 * each, with its own d and size bounds; the same computation as
 * fec_cluster_async on that cloud alone, so each request's labels and count
 * equal its single-call result whatever it was batched with).
 *
 * The engine owns nslots batch slots on the current device, each with its
 * own stream, batched-form workspace and buffers.  Admission is by HBM
 * footprint: a slot holds at most fec_server_slot_points() points (the most
 * whose slot footprint, fec_server_slot_bytes(), fits hbm_budget / nslots)
 * in at most slot_frames requests.  Requests queue in submission order;
 * fec_server_pump() retires finished batches and launches the head of the
 * queue into every free slot at once (no waiting for a batch to fill), so
 * batches overlap on the device.  One host thread drives a server.
 */
typedef struct fec_server fec_server;

/* HBM bytes of one slot for slot_points points in slot_frames requests (0 if invalid). */
size_t fec_server_slot_bytes(int64_t slot_points, int32_t slot_frames);

/*
 * Creates a server: nslots in [1, 64], slot_frames in [1, 1024].  Returns
 * FEC_OK and *out, FEC_EINVAL for bad arguments, FEC_ENOMEM when the budget
 * holds no point per slot or an allocation fails.
 */
int32_t fec_server_create(size_t hbm_budget, int32_t nslots, int32_t slot_frames,
                          fec_server **out);

/* Points one slot admits. */
int64_t fec_server_slot_points(const fec_server *server);

/*
 * Queues one request.  xyz (float32 [n][3]) and labels_out (int32 [n]) are
 * DEVICE pointers (pinned host memory also works, over PCIe) that must stay
 * valid, and unused by other work, until the request completes; labels_out
 * then holds the request's labels (as fec_cluster gives them).  Returns
 * FEC_OK and *ticket (0, 1, 2, ... in submission order); FEC_EINVAL for the
 * argument checks of fec_cluster; FEC_ENOMEM when n exceeds a slot.
 */
int32_t fec_server_submit(fec_server *server, const float *xyz, int64_t n, float d,
                          int32_t min_size, int32_t max_size, int32_t *labels_out,
                          int64_t *ticket);

/*
 * Retires finished batches, then launches queued requests into free slots.
 * With wait != 0 and nothing retired or launched, blocks until the oldest
 * batch in flight finishes (returns at once when none is).  Returns the
 * number of requests completed by this call, or a negative status.
 */
int32_t fec_server_pump(fec_server *server, int32_t wait);

/*
 * fec_server_pump without waiting, then, when it completed nothing, watches
 * the batches in flight for up to max_wait_us microseconds and retires the
 * first that finishes (launching queued requests into the slots it frees).
 * A caller that must also admit new requests at known times passes the time
 * left until the next one.  Returns the number of requests completed, or a
 * negative status (FEC_EINVAL for max_wait_us < 0).
 */
int32_t fec_server_pump_for(fec_server *server, int64_t max_wait_us);

/*
 * Takes up to max completed requests, oldest first: ticket, k (kept
 * clusters, or a negative FEC_* status) and latency in milliseconds from
 * submission to retirement by fec_server_pump.  Returns the number taken.
 */
int32_t fec_server_poll(fec_server *server, int64_t *tickets, int32_t *k, double *latency_ms,
                        int32_t max);

/*
 * out[0] requests submitted, out[1] completed, out[2] batches launched,
 * out[3] queued now, out[4] slots busy now, out[5] most requests in one
 * batch, out[6] most batches in flight at once, out[7] points per slot,
 * out[8] bytes per slot, out[9] requests re-queued to run alone (their
 * batch's stacked grid needed a key wider than 64 bits, so the whole batch
 * was refused; alone each gets its own result).  Returns the number of
 * values written (<= 10).
 */
int32_t fec_server_stats(const fec_server *server, int64_t *out, int32_t max_out);

/* Waits for the server's work and frees it. */
void fec_server_destroy(fec_server *server);

/* Stream used by fec_cluster (a hipStream_t; NULL = null stream).  Returns FEC_OK. */
int32_t fec_set_stream(void *stream);

/* Frees the workspace cached by fec_cluster. */
void fec_release(void);

/* Message for the last non-OK status returned on this host thread ("" if none). */
const char *fec_last_error(void);

/* Library version string. */
const char *fec_version(void);

/*
 * Diagnostics of the last call that used `workspace` (waits for `stream`):
 * out[0] n, out[1] finite points, out[2] occupied grid cells, out[3] occupied
 * grid columns, out[4] grid key bits, out[5] radix passes, out[6..8] grid
 * cells along x, y, z, out[9] largest points per cell, out[10] status,
 * out[11] cells left outside the largest component after the near shell,
 * out[12] that component's root cell, out[13..20] diagnostic event counts
 * (zero unless the library was built with FEC_COUNTERS defined), out[21]
 * the column index used (0 binary search, 1 dense table, 2 hash table),
 * out[22] cells left outside the largest component after the sampling links
 * (the cells the near shell visits; 0 when the cloud has fewer than 131,072
 * cells, where the near shell visits every cell).
 * For a batched call the grid fields describe the frames' stacked grid,
 * out[11] and out[22] count the cells outside each frame's largest component
 * and out[12] is -1.
 * Writes min(max_out, 23) values; returns that count or a negative status.
 */
int32_t fec_workspace_stats(const void *workspace, void *stream, int64_t *out, int32_t max_out);

/*
 * Kernel timing with HIP events recorded on the launch stream around the
 * kernels of the stages selected by `stage_mask` (bit i = stage i; 0 turns
 * timing off).  fec_profile_read waits for the recorded events, adds their
 * durations to per-stage totals and writes, for i < max_stages, the total
 * milliseconds and the number of timed launches of stage i; it returns the
 * number of stages.  fec_profile_reset clears the totals.
 */
int32_t fec_profile_enable(uint64_t stage_mask);
int32_t fec_profile_read(double *ms_total, int64_t *launches, int32_t max_stages);
void fec_profile_reset(void);
int32_t fec_stage_count(void);

/*
 * Launch configuration (the autotuner's knobs; process-wide, applies to
 * calls enqueued afterwards):
 *   cell_blocks    the most blocks of the per-cell grid-stride kernels
 *                  (default 4096), in [0, 2^20];
 *   stream_blocks  the most blocks of the per-point streaming kernel that
 *                  sets every label to -1 before the kept clusters' labels
 *                  (default 4096), in [0, 2^20];
 *   radix_bits     bits per radix-sort pass: 8, 9, 10 or 11 (default 9);
 *                  wider digits take fewer passes over larger tables (at
 *                  9, the passes beyond a key's first 36 bits take 10);
 *   hook_block     threads per block of the hooking kernels: 64, 128 or
 *                  256 (default 256);
 *   near_sampling  whether clouds of at least 131,072 cells first link each
 *                  cell to the first cells of its dx = +1 neighbour columns
 *                  and run the near shell only outside the largest component
 *                  so formed: 0 when the cloud (in a batch, the average
 *                  frame) has at least 2^23 points (default), 1 always,
 *                  2 never.
 * 0 restores a knob's default.  Labels and counts do not depend on any of
 * them.  Returns FEC_OK, or FEC_EINVAL for a value outside its set.
 */
int32_t fec_tuning_set(int32_t cell_blocks, int32_t stream_blocks, int32_t radix_bits,
                       int32_t hook_block, int32_t near_sampling);
int32_t fec_tuning_get(int32_t *cell_blocks, int32_t *stream_blocks, int32_t *radix_bits,
                       int32_t *hook_block, int32_t *near_sampling);
const char *fec_stage_name(int32_t stage);

#ifdef __cplusplus
}
#endif

#endif /* FEC_H */
