/*
 * cox.h -- C ABI of libcox.so, an MI355X (gfx950) library of kernels built on
 * CUDA's 32-lane warp-level functions with their exact semantics.
 *
 * The paper this library follows (COX, "CUDA on X86 by Exposing Warp-Level
 * Functions to CPUs") runs CUDA kernels that use warp shuffles, warp votes
 * and cooperative-group tiles (its Sec. 2.2 and Table 1) on CPUs.  This
 * library runs the same kind of kernels on AMD wave64 hardware: every
 * 64-lane wavefront carries two logical 32-lane warps; a logical warp's
 * ballot is one half of the wave's 64-bit lane mask.
 *
 * Conventions for every entry point below:
 *  - Pointers named as device buffers point to GPU memory (hipMalloc or a
 *    torch CUDA tensor); the caller owns all of them.  The library never
 *    allocates on these calls.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on that stream; results are ready when the
 *    stream is synchronized.
 *  - Arguments are validated before anything is enqueued; on an error
 *    nothing is launched and the status says why.  A failed HIP launch
 *    returns COX_ERR_HIP (its hipError_t via cox_last_hip_error()).
 *  - n = 0 is valid everywhere: totals become the identity (0 or -0.0),
 *    counts 0, nothing else is written.
 *  - Workspaces (`ws`, `ws_bytes`) are device buffers sized by
 *    cox_workspace_bytes().  A fresh workspace must be zero-filled once
 *    (cox_workspace_init); every call leaves it ready for the next call of
 *    the same operation kind.  Calls that share a workspace must be ordered
 *    on one stream; a workspace used for a different operation kind must be
 *    re-initialised.
 *  - Vector loads need 16-byte aligned data pointers for the reduce, dot,
 *    scan, compaction and sort entry points (COX_ERR_ALIGN otherwise).
 */
#ifndef COX_H
#define COX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  COX_OK = 0,
  COX_ERR_INVALID = 1,     /* bad size, width, offset, tile or schedule */
  COX_ERR_DTYPE = 2,       /* dtype / accumulation not offered by this entry */
  COX_ERR_ALIGN = 3,       /* data pointer not 16-byte aligned */
  COX_ERR_HIP = 4,         /* a HIP call failed; see cox_last_hip_error() */
  COX_ERR_WORKSPACE = 5,   /* workspace missing or smaller than required */
  COX_ERR_UNSUPPORTED = 6, /* schedule outside the compiled set */
  COX_ERR_TIMEOUT = 7      /* a bounded cross-block wait gave up */
} cox_status;

typedef enum { COX_I32 = 0, COX_U32 = 1, COX_F32 = 2, COX_BF16 = 3 } cox_dtype;

/* accumulation of floating-point reductions: plain binary32 adds, or the
 * compensated TwoSum / TwoProduct variant (Ogita, Rump and Oishi's Sum2 /
 * Dot2 carried through the warp tree) */
typedef enum { COX_ACC_PLAIN = 0, COX_ACC_TWOSUM = 1 } cox_acc;

/* warp shuffle variants (CUDA __shfl_sync, __shfl_up_sync,
 * __shfl_down_sync, __shfl_xor_sync) */
typedef enum { COX_SHFL_IDX = 0, COX_SHFL_UP = 1, COX_SHFL_DOWN = 2, COX_SHFL_XOR = 3 } cox_shfl_op;

/* operation kinds for cox_workspace_bytes */
typedef enum {
  COX_OP_REDUCE = 0,
  COX_OP_DOT = 1,
  COX_OP_SCAN = 2,
  COX_OP_COMPACT = 3,
  COX_OP_SEGMENTED = 4,
  COX_OP_CG = 5,           /* n = rows; cfg: items_per_lane = rows per lane R */
  COX_OP_GRID_EXCHANGE = 6, /* n = grid blocks */
  COX_OP_INTEGRAL_IMAGE = 7 /* n = image height, nseg = image width */
} cox_op;

/* Schedule sigma of the chunked kernels.  A chunk is the tile of one
 * thread block: S = 32 * warps_per_block * items_per_lane elements.
 * Thread (w, l) of the block owns, for row i in [0, items/V) and vector slot
 * v in [0, V) (V = min(items, 16 bytes / element size)), chunk offset
 *     w * 32 * items + (i * 32 + l) * V + v
 * and accumulates its elements in (i, v) order; the warp combines lanes with
 * the shfl_down tree (offsets 16, 8, 4, 2, 1), lane 0 of every warp puts the
 * warp value in shared memory, and warp 0 runs the same tree over those
 * values.  Floating-point results depend on (items_per_lane,
 * warps_per_block) only, never on grid_blocks or on the order in which
 * blocks run.  Zero fields select the operation's default.
 *   items_per_lane  : 1, 2, 4, 8, 16 or 32
 *   warps_per_block : 1, 2, 4, 8, 16 or 32
 *   grid_blocks     : persistent grid size (0 = fill the device)
 */
typedef struct {
  int32_t items_per_lane;
  int32_t warps_per_block;
  int32_t grid_blocks;
  int32_t reserved;
} cox_cfg;

/* ---------------------------------------------------------------------
 * Library plumbing (status text, versions, schedules, workspaces): no
 * passage of the paper defines these.
 * ------------------------------------------------------------------- */
const char *cox_status_string(cox_status s);
/* hipError_t of the most recent COX_ERR_HIP on the calling thread */
int cox_last_hip_error(void);
/* library ABI version (major * 100 + minor) */
int cox_version(void);
/* default schedule the library uses for `op` / `dtype` when cfg is NULL or
 * has zero fields; writes *out */
cox_status cox_default_cfg(cox_op op, cox_dtype dtype, cox_cfg *out);

/* Bytes of workspace that `op` needs for n elements (nseg segments for
 * COX_OP_SEGMENTED) under cfg (NULL = defaults). */
size_t cox_workspace_bytes(cox_op op, cox_dtype dtype, int64_t n, int64_t nseg, const cox_cfg *cfg);
/* Zero-fills a workspace on `stream` (with a kernel, so it may be captured
 * in a graph). */
cox_status cox_workspace_init(void *ws, size_t ws_bytes, void *stream);
/* Synchronises `stream`, then reports COX_ERR_TIMEOUT if a bounded
 * cross-block wait of a call that used this workspace gave up since the
 * previous check (the results of that call are invalid), or
 * COX_ERR_INVALID if a segmented call's offsets overlapped so that their
 * chunks outnumbered the workspace's capacity (those results are invalid
 * too), and clears the flag.  COX_OK otherwise. */
cox_status cox_workspace_status(void *ws, void *stream);

/* ---------------------------------------------------------------------
 * Warp functions applied to arrays (the paper's warp builtins operating
 * on per-warp arrays, Sec. 3.2; semantics per the CUDA Programming Guide
 * that the paper refers to in Sec. 2.2.1).
 * ------------------------------------------------------------------- */

/* For every 32-element warp g (n % 32 == 0): the lanes l set in mask[g]
 * (mask == NULL: all 32) execute
 *     out[32g + l] = shfl_op(v, arg_l, width)
 * with arg_l = argv[32g + l] when argv != NULL, else arg, and the CUDA
 * rules: b = l & ~(width-1); IDX reads b + (arg & (width-1)); UP reads
 * l - arg if l - b >= arg else keeps v[l]; DOWN reads l + arg if
 * l - b + arg < width else keeps v[l]; XOR reads j = l ^ arg if
 * j < b + width (an earlier segment is readable) else keeps v[l].
 * Lanes outside the mask copy v.  width is 1, 2, 4, 8, 16 or 32; arg of
 * UP / DOWN / XOR is in [0, 31].  A source lane outside the mask is
 * undefined in CUDA; here it reads that lane's input.
 * v, out, argv, mask: device buffers (int32[n], int32[n], int32[n],
 * uint32[n/32]). */
cox_status cox_warp_shfl(const int32_t *v, int32_t *out, int64_t n, int op, int32_t arg,
                         const int32_t *argv, int width, const uint32_t *mask, void *stream);

/* For every warp g (n % 32 == 0) the lanes of m = mask[g] (NULL: all)
 * execute b = __ballot_sync(m, pred), a = __any_sync(m, pred),
 * t = __all_sync(m, pred) (pred nonzero = true); the lowest lane of m
 * stores ballot[g] = b, anyall[g] = a | t << 1 (zeros for an empty mask).
 * Code 4 of the paper (VoteAll) is the case pred = tx % 2, full mask.
 * pred: int32[n]; mask: uint32[n/32] or NULL; ballot: uint32[n/32];
 * anyall: int32[n/32]; all device buffers. */
cox_status cox_warp_vote(const int32_t *pred, const uint32_t *mask, int64_t n, uint32_t *ballot,
                         int32_t *anyall, void *stream);

/* Tile-scoped votes of cooperative groups' thread_block_tile<T> (the
 * static groups of Sec. 2.2.2 with the votes of Sec. 2.2.1): every warp
 * (n % 32 == 0) is 32/T tiles of T consecutive lanes, T in {1, 2, 4, 8,
 * 16, 32}, each a whole group.  For tile g (elements gT .. gT + T - 1):
 *     ballot[g] = sum over i < T of (pred[gT + i] != 0) << i   (T bits)
 *     anyall[g] = tile.any(pred) | tile.all(pred) << 1
 * written by the tile's rank-0 lane.  A lane's thread_rank() in its tile
 * is e mod T, and its tile's rank among the tiles of its warp is
 * (e mod 32) / T (meta_group_rank() of a partition of a 32-thread tile).
 * pred: int32[n]; ballot: uint32[n / T]; anyall: int32[n / T]; device
 * buffers. */
cox_status cox_tile_vote(const int32_t *pred, int64_t n, int tile, uint32_t *ballot, int32_t *anyall,
                         void *stream);

/* ---------------------------------------------------------------------
 * Block reduction with warp shuffles (Sec. 2.3 Code 1 generalised to a
 * 256-thread block, the SDK reduction kernels of Table 1).
 * ------------------------------------------------------------------- */

/* 256-thread blocks of 8 logical warps, one element per thread:
 *   block_sums[b] = wrap32 sum of x[256b .. 256b+255] (shfl_down tree per
 *                   warp, shared-memory combine of the 8 warp values);
 *   warp_pos_count[g] = popc(__ballot_sync(FULL, x > 0)) over
 *                   x[32g .. 32g+31].
 * Elements past n count as 0 and as not positive.
 * x: int32[n]; block_sums: int32[ceil(n/256)];
 * warp_pos_count: int32[ceil(n/32)]; device buffers. */
cox_status cox_warp_reduce_blocks_i32(const int32_t *x, int64_t n, int32_t *block_sums,
                                      int32_t *warp_pos_count, void *stream);

/* Chunked sum of x under schedule cfg (see cox_cfg): the warp-shuffle
 * reduction of Code 1 (Sec. 2.3) inside every block, as in the SDK
 * reduction kernels reduce4-6 / reduce / reduceFinal of Table 1, with the
 * compensated variant and the FP64 final combine of this library (the
 * paper does not discuss floating-point accuracy).
 * dtype COX_I32 (acc must be PLAIN): lanes, warps and blocks add with
 *   two's-complement wrap (CUDA int); chunk partials are int32;
 *   *total (int64) = sum of the chunk partials as int64, which equals the
 *   exact sum whenever no chunk partial overflows.
 * dtype COX_F32 / COX_BF16 (bfloat16 bits as uint16, widened exactly):
 *   binary32 lane accumulation and tree (TwoSum-compensated pairs (s, c)
 *   for COX_ACC_TWOSUM), chunk partials float32 (float32 pairs for
 *   TWOSUM), and *total (double) = FP64 final combine: a fixed tree shaped
 *   like a 256-thread block (thread j adds chunks j, j+256, ... serially
 *   from -0.0, an FP64 shfl_down tree per warp, then over the 8 warp
 *   values); for TWOSUM each chunk enters as (double)s + (double)c.
 * Elements past n are padding equal to -0.0 (0 for int32).
 * x: device buffer of n elements; chunk_partials: device buffer of
 * nchunks (x2 for TWOSUM) entries or NULL; total: device int64 / double;
 * ws: workspace of cox_workspace_bytes(COX_OP_REDUCE, ...). */
cox_status cox_warp_reduce(const void *x, cox_dtype dtype, int64_t n, cox_acc acc,
                           const cox_cfg *cfg, void *chunk_partials, void *total, void *ws,
                           size_t ws_bytes, void *stream);

/* Chunked dot product sum_i a_i * b_i (dtype COX_F32 or COX_BF16), the
 * gpuDotProduct kernel of Table 1 (a warp cooperative-group reduction,
 * Sec. 2.2.2), with the schedule of cox_warp_reduce.  PLAIN: s = fmaf(a_i, b_i, s) per element.
 * TWOSUM (Dot2): (p, pe) = TwoProduct(a_i, b_i) = (a*b, fmaf(a, b, -p)),
 * (s, q) = TwoSum(s, p), c = c + (pe + q).  Padding: a = -0.0, b = +0.0.
 * Result in *total (device double); partials as for cox_warp_reduce. */
cox_status cox_warp_dot(const void *a, const void *b, cox_dtype dtype, int64_t n, cox_acc acc,
                        const cox_cfg *cfg, void *chunk_partials, double *total, void *ws,
                        size_t ws_bytes, void *stream);

/* Inclusive int32 scan (the shuffle scan of the CUDA sample whose
 * shfl_scan_test and uniform_add kernels Table 1 lists; shfl_up is one of
 * the warp shuffles of Sec. 2.2.1), y_i = (x_0 + ... + x_i) mod 2^32, in
 * one pass: warp scans with shfl_up (Kogge-Stone), warp totals combined in
 * shared memory (the block-level carry that uniform_add applies), chunks chained by decoupled look-back (status words published
 * with device-scope atomics; chunk order from a ticket counter so that a
 * chunk only waits for chunks already being processed).  x, y: int32[n]
 * device buffers (may not overlap); ws: cox_workspace_bytes(COX_OP_SCAN). */
cox_status cox_warp_scan(const int32_t *x, int32_t *y, int64_t n, const cox_cfg *cfg, void *ws,
                         size_t ws_bytes, void *stream);

/* Size of the device scratch that cox_warp_scan_noalloc uses (1 MiB). */
#define COX_NOALLOC_SCRATCH_BYTES ((size_t)1 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * cox_warp_scan with the same arguments, result and kernels, but without a
 * workspace argument.  The look-back header and status words live in a
 * library-owned device array of COX_NOALLOC_SCRATCH_BYTES, one per device,
 * held until the process ends; the call allocates nothing (no hipMalloc,
 * no allocating library routine).  The first call on a device looks the
 * array up and zeroes it on `stream`, ahead of its own kernels.  Its
 * status words are packed 8 bytes apart (a workspace spaces them 128
 * bytes apart, which makes cox_warp_scan about 4 % faster).
 * Limit: 256 + 8 * (chunks + 1) bytes, chunks = ceil(n / (32 k W)), must
 * not exceed COX_NOALLOC_SCRATCH_BYTES (the default schedule covers every
 * n the scan accepts; the smallest schedule, 32 elements per chunk, about
 * 4.2M elements), else COX_ERR_WORKSPACE before anything is enqueued.
 * err_out: NULL, or a device uint32 that receives 0, or nonzero if a
 * bounded cross-block wait of this call (or an earlier one on this device
 * whose status was not taken) gave up; the scratch's record is then cleared.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (other streams, other threads) race and must be serialised
 * by the caller. */
cox_status cox_warp_scan_noalloc(const int32_t *x, int32_t *y, int64_t n, const cox_cfg *cfg,
                                 uint32_t *err_out, void *stream);

/* Stable ballot compaction (warp votes, Sec. 2.2.1; the filtering that
 * the filter_arr kernel of Table 1 performs, here with a static full mask
 * and ballot ranks instead of its dynamic group), keeping x_i > 0:
 * out[0 .. *count) = the kept elements in input order; *count (device int64) = their number.  Per warp and row
 * the ranks come from ballots: rank = popc(ballot & lanemask_lt) summed
 * over the lane's vector slots; warp counts are scanned in shared memory
 * and chunk offsets chained by decoupled look-back.  x: int32[n]; out:
 * int32[n] capacity; ws: cox_workspace_bytes(COX_OP_COMPACT). */
cox_status cox_ballot_compact(const int32_t *x, int64_t n, int32_t *out, int64_t *count,
                              const cox_cfg *cfg, void *ws, size_t ws_bytes, void *stream);

/* Tile sort, a workload built from the warp shuffles of Sec. 2.2.1
 * (__shfl_xor_sync exchanges) over thread-block tiles of Sec. 2.2.2:
 * sorts every group of `tile` consecutive keys ascending (unsigned) with a
 * bitonic network.  tile = 32: the cross-lane steps are __shfl_xor_sync
 * exchanges inside the group, cfg->items_per_lane keys per lane (1, 2, 4,
 * 8 or 16; 0 = 4).  tile = 64 .. 1024 (a power of two): the group spans
 * both halves of a wave (exchanges across them by v_permlane32_swap) or
 * several waves (exchanges through shared memory); items_per_lane 4
 * (0 = 4) for tile <= 1024, or 1 for tile <= 256 (tile 64 with 1 key per
 * lane is the full-wave 64-key sort).  Other combinations give
 * COX_ERR_UNSUPPORTED.  A partial last group is sorted among its valid
 * keys.  keys, out: uint32[n] device buffers (may be the same buffer). */
cox_status cox_tile_sort(const uint32_t *keys, uint32_t *out, int64_t n, int tile,
                         const cox_cfg *cfg, void *stream);

/* Key-value form (a workload built from the same shuffle network: warp
 * shuffles, Sec. 2.2.1, over 32-lane tiles, Sec. 2.2.2): every group of 32
 * consecutive pairs (keys[i], vals[i]) ordered by unsigned key,
 * pairs with equal keys in their original order (a stable sort, so the
 * result is unique).  The network sorts (key, position in the group);
 * each output then takes the value at its position.  A partial last group
 * is sorted among its valid pairs.  keys, out_keys: uint32[n], 16-byte
 * aligned (may be the same buffer); vals: uint32[n] payloads of any 4-byte
 * type; out_vals: uint32[n], 16-byte aligned, not overlapping vals
 * (COX_ERR_INVALID if it is vals).  cfg->items_per_lane: pairs per lane,
 * 1, 2, 4 or 8 (0 = 4). */
cox_status cox_tile_sort_kv(const uint32_t *keys, const uint32_t *vals, uint32_t *out_keys, uint32_t *out_vals,
                            int64_t n, int tile, const cox_cfg *cfg, void *stream);

/* thread_block_tile<T> reduction (static cooperative groups, section
 * 2.2.2; warp-function support, section 3.2): out[g] = wrap32 sum of
 * x[gT .. gT+T-1], the value tile.shfl_down(v, o), o = T/2 .. 1, leaves in
 * the tile's first lane; T in {2, 4, 8, 16, 32}; elements past n count as
 * 0.  Sums modulo 2^32 do not depend on the order of the additions, so
 * each lane adds 4 consecutive elements (one 16-byte load) and the T/4
 * lanes of a tile finish with xor exchanges.  x: int32[n] (4-byte
 * aligned); out: int32[ceil(n/T)]; device buffers. */
cox_status cox_tile_reduce(const int32_t *x, int64_t n, int tile, int32_t *out, void *stream);

/* Masked (divergent) warp operations with predicate-derived masks (the
 * mask argument of the warp shuffles and votes, Sec. 2.2.1; COX itself
 * supports only static full masks, Sec. 2.2.3), n % 32 == 0.  Lane l of warp g, x = x[32g + l]:
 *   p = ((uint32)x & 1023) < density;  m = __ballot_sync(FULL, p);
 *   if (p) { b = __ballot_sync(m, x > 0); A = __any_sync(m, ((x >> 10) & 31) == 0);
 *            L = __all_sync(m, ((x >> 15) & 31) != 0);
 *            s = __shfl_sync(m, x, next lane of m above l, wrapping);
 *            bc = __shfl_sync(m, x, ffs(m) - 1);  out = s;
 *            lane ffs(m)-1 stores rec[g] = {m, b, A | L << 1, bc}; }
 *   else out = INT32_MIN;   (m == 0: lane 0 stores rec[g] = {0, 0, 0, 0})
 * density in [0, 1024].  x, out: int32[n]; rec: uint32[4 * n/32]. */
cox_status cox_warp_masked(const int32_t *x, int64_t n, int density, int32_t *out, uint32_t *rec,
                           void *stream);

/* Dynamic groups (the dynamic cooperative group of the filter kernel that
 * COX does not support, Table 1; cooperative groups, section 2.2.2;
 * static-only limitation, section 2.2.3), n % 32 == 0.  Lane l of warp g,
 * x = x[32g + l]:
 *   p = ((uint32)x & 1023) < density;
 *   if (p) { grp = coalesced_threads();  m = __activemask();
 *            rank[e] = grp.thread_rank();  key = ((uint32)x >> 10) & 7;
 *            match_any[e] = __match_any_sync(m, key);
 *            ma = __match_all_sync(m, key, &pred);
 *            add = __reduce_add_sync(m, x & 0xffff);  min / max =
 *            __reduce_min_sync / __reduce_max_sync(m, x) (signed);
 *            and / or / xor = __reduce_{and,or,xor}_sync(m, (unsigned) x);
 *            the rank-0 member appends grp.size() slots to filtered[] and
 *            shares the base (grp.shfl); filtered[base + rank] = x;
 *            the rank-0 member stores rec[g] = {m, ma, add, min, max, and,
 *            or, xor} }
 *   else { match_any[e] = 0; rank[e] = 0xffffffff; }
 *   (m == 0: rec[g] = 8 zeros).
 * *filtered_count (device int64) = number of members.  Every warp's
 * members occupy consecutive slots of filtered[] in rank order; the order
 * of the warps' runs is the order their appends happen to take (not
 * deterministic).  x, match_any, rank: [n]; rec: uint32[8 * n/32], 16-byte
 * aligned; filtered: int32[n] capacity. */
cox_status cox_warp_dynamic(const int32_t *x, int64_t n, int density, uint32_t *match_any, uint32_t *rank,
                            uint32_t *rec, int32_t *filtered, int64_t *filtered_count, void *stream);

/* ---------------------------------------------------------------------
 * Segmented batching: thousands of uneven CSR segments in one persistent
 * launch.  The paper runs one CUDA block per CPU thread through pthread
 * fork/join per kernel launch (Sec. 4) and names a reusable thread pool
 * as the better runtime; here every chunk of every segment is a ticket of
 * one queue drained by a persistent grid, and a plan captures the whole
 * call (setup kernels + fused kernel) in a hipGraph.
 *
 * Segment s = x[offsets[s], offsets[s+1]) (offsets: device int64[nseg+1],
 * non-decreasing, within [0, n]; x: device int32 or float32 [n], 16-byte
 * aligned).  Offsets cannot be checked before launch; the kernels clamp
 * every segment to [0, n] (a reversed segment is empty), so bad offsets
 * give meaningless results but no access outside x, y, out_compact or the
 * workspace.  Offsets that go down and up again make overlapping
 * segments; when their chunks outnumber the workspace's capacity
 * (n / S + nseg + 1), the chunks past it are dropped and
 * cox_workspace_status reports COX_ERR_INVALID.  Chunks of
 * S = 32 * warps_per_block * items_per_lane elements start at each
 * segment's first element (items_per_lane <= 32).
 *   seg_total[s] : device int64 (int32 input) = sum of the int32-wrapped
 *                  chunk partials as int64; device double (float input) =
 *                  FP64 sum, from -0.0 in chunk order, of the chunk
 *                  partials (each the sigma reduce tree of cox_cfg);
 *   y            : inclusive scan restarting at every segment, at the
 *                  positions of x; int32 wraps; float: chunk-local scan
 *                  q by the documented shuffle tree, then
 *                  (float)(C_j + (double)q) with C_j the FP64 sum from
 *                  -0.0 in chunk order of the earlier chunks' totals;
 *   out_compact  : the elements > 0 of segment s, in order, written at
 *                  out_compact[offsets[s] ...]; seg_count[s] (device
 *                  int64) their number.
 * An empty segment gets total 0 / -0.0 and count 0.  `which` selects the
 * outputs: 1 = totals, 2 = scan, 4 = compaction (or any sum).  Workspace:
 * cox_workspace_bytes(COX_OP_SEGMENTED, dtype, n, nseg, cfg).
 * ------------------------------------------------------------------- */
cox_status cox_segmented(const void *x, cox_dtype dtype, const int64_t *offsets, int64_t nseg, int64_t n,
                         void *seg_total, void *y, void *out_compact, int64_t *seg_count, int which,
                         const cox_cfg *cfg, void *ws, size_t ws_bytes, void *stream);
cox_status cox_segmented_reduce(const void *x, cox_dtype dtype, const int64_t *offsets, int64_t nseg, int64_t n,
                                void *seg_total, const cox_cfg *cfg, void *ws, size_t ws_bytes, void *stream);
cox_status cox_segmented_scan(const void *x, cox_dtype dtype, const int64_t *offsets, int64_t nseg, int64_t n,
                              void *y, const cox_cfg *cfg, void *ws, size_t ws_bytes, void *stream);
cox_status cox_segmented_compact(const void *x, cox_dtype dtype, const int64_t *offsets, int64_t nseg, int64_t n,
                                 void *out_compact, int64_t *seg_count, const cox_cfg *cfg, void *ws,
                                 size_t ws_bytes, void *stream);
/* all three outputs in one fused launch (which = 7) */
cox_status cox_segmented_fused(const void *x, cox_dtype dtype, const int64_t *offsets, int64_t nseg, int64_t n,
                               void *seg_total, void *y, void *out_compact, int64_t *seg_count, const cox_cfg *cfg,
                               void *ws, size_t ws_bytes, void *stream);
/* The per-segment baseline: the same fused kernel launched once per
 * segment (offsets_host: host copy of offsets, used for grid sizes). */
cox_status cox_segmented_per_segment(const void *x, cox_dtype dtype, const int64_t *offsets,
                                     const int64_t *offsets_host, int64_t nseg, int64_t n, void *seg_total, void *y,
                                     void *out_compact, int64_t *seg_count, const cox_cfg *cfg, void *ws,
                                     size_t ws_bytes, void *stream);

/* A plan: one segmented call bound to its buffers and captured in a
 * hipGraph on a stream of the plan's own (the batched form of the
 * per-launch fork/join that Sec. 4 describes; this is the plan that a
 * general cox_plan_create(op, ...) would build for the segmented
 * operations, the only ones that need one).  The schedule, when the
 * caller gives none (cfg NULL or items/warps zero), is, in this order:
 *  - COX_FORCE_CFG="k,W" or "k,W,G" from the environment, if it is valid;
 *  - with autotune != 0 and COX_TUNE_CACHE naming a file: the last entry
 *    of that file for this call shape (operation, dtype, n, nseg, outputs,
 *    device architecture and compute units);
 *  - with autotune != 0: the fastest of a set of candidate
 *    (items_per_lane, warps_per_block, grid), each timed on the caller's
 *    buffers; the choice is appended to COX_TUNE_CACHE when it is set;
 *  - otherwise the default schedule.
 * The chosen schedule (which fixes the float results) is reported by
 * cox_plan_get_cfg.  Creation replays the captured graph once, so the
 * outputs hold the call's results, and synchronises; ws must be large
 * enough for every candidate tried (candidates that do not fit are
 * skipped).  cox_plan_execute replays the graph on `stream`; a plan must
 * not run concurrently with itself or with another call on the same
 * workspace. */
typedef struct cox_plan_s *cox_plan;
cox_status cox_plan_segmented(const void *x, cox_dtype dtype, const int64_t *offsets, int64_t nseg, int64_t n,
                              void *seg_total, void *y, void *out_compact, int64_t *seg_count, int which,
                              const cox_cfg *cfg, int autotune, void *ws, size_t ws_bytes, void *stream,
                              cox_plan *plan);
cox_status cox_plan_execute(cox_plan plan, void *stream);
cox_status cox_plan_get_cfg(cox_plan plan, cox_cfg *cfg);
cox_status cox_plan_destroy(cox_plan plan);

/* Integral image (summed-area table), the application of the warp
 * shuffle scans that Table 1 lists (the row pass and the vertical pass of
 * the CUDA scan sample):
 *     sat[y][x] = sum of img[y'][x'] over y' <= y and x' <= x   (mod 2^32)
 * img: device uint8[height][width], row-major; sat: device
 * uint32[height][width].  Tiles of 64 rows x 1024 columns are reduced
 * (column sums, row sums, tile totals), the column sums are scanned down
 * the bands, and every tile is then scanned row by row (a 32-lane shuffle
 * scan per row) with its carries from above and from the left: three
 * launches, about 6.1 bytes per pixel.  The result is exact (uint32
 * arithmetic).  A width that is a multiple of 4 with img 4-byte and sat
 * 16-byte aligned uses 4-pixel loads and 16-byte stores; any other shape
 * works element by element.  ws: cox_workspace_bytes(COX_OP_INTEGRAL_IMAGE,
 * COX_U32, height, width, NULL). */
cox_status cox_integral_image(const uint8_t *img, int64_t height, int64_t width, uint32_t *sat, void *ws,
                              size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Grid-wide synchronisation (cooperative groups' this_grid().sync(),
 * Sec. 2.2.2), which COX could not run (Sec. 5.1, Table 1: the
 * conjugate-gradient sample).  The kernels below run on a cooperative
 * launch, every block resident at once, and meet at a grid barrier: block
 * arrivals are counted in eight groups (blocks b mod 8), the last arrival
 * advances a generation word the other blocks wait for, and the writes of
 * every block before the barrier are visible to every block after it.
 * Waits are bounded: a barrier that does not complete within about a
 * second ends the kernel early and sets the workspace's timeout flag
 * (cox_workspace_status then reports COX_ERR_TIMEOUT; outputs are
 * invalid).  The barrier words live in the workspace and are reset by
 * every call.
 * ------------------------------------------------------------------- */

/* Largest grid (blocks of 1024 threads) a cooperative launch of the
 * exchange kernel can hold on the current device. */
cox_status cox_grid_capacity(int32_t *max_blocks);

/* Exchange kernel (a check and a clock for the barrier): grid_blocks
 * blocks of 1024 threads run `rounds` rounds; in round r thread t of block
 * b writes fmix32(r << 20 ^ b << 10 ^ t) (MurmurHash3's 32-bit finaliser)
 * to its slot, all blocks meet at a grid barrier, thread t adds (mod 2^32)
 * the slot of thread t of block (b + r + 1) mod grid_blocks, and all
 * blocks meet again.  out (device uint32[grid_blocks * 1024]) receives the
 * sums.  1 <= grid_blocks <= cox_grid_capacity (COX_ERR_INVALID
 * otherwise); ws: cox_workspace_bytes(COX_OP_GRID_EXCHANGE, COX_U32,
 * grid_blocks, 0, NULL). */
cox_status cox_grid_exchange(int32_t grid_blocks, int32_t rounds, uint32_t *out, void *ws, size_t ws_bytes,
                             void *stream);
/* Check of the barrier's failure handling: the exchange kernel with block
 * absent_block (0 <= absent_block < grid_blocks) leaving before the first
 * barrier, and every wait bounded by spin_limit polls (1 .. 2^20) instead
 * of the usual bound.  The other blocks' waits give up, every block
 * finishes, and cox_workspace_status then reports COX_ERR_TIMEOUT; out is
 * meaningless.  The next call on the workspace starts clean. */
cox_status cox_grid_exchange_absent(int32_t grid_blocks, int32_t rounds, int32_t absent_block, uint32_t spin_limit,
                                    uint32_t *out, void *ws, size_t ws_bytes, void *stream);

/* Conjugate gradient (Hestenes and Stiefel) for A x = b, A symmetric
 * positive definite in CSR form, in ONE cooperative launch: the iteration
 * loop runs inside the kernel with two grid barriers per iteration.
 *   row_ptr : device int32[n + 1], row_ptr[0] = 0, nondecreasing,
 *             row_ptr[n] = nnz;  col_idx : device int32[nnz] in [0, n);
 *   val     : device float[nnz];  b : device float[n];
 *   x       : device float[n], the start x_0 on entry, the result on exit;
 *   result  : device int32[2] = {iterations k, reason}: 0 converged
 *             (rr_k <= tol^2), 1 max_iter reached, 2 breakdown (<p, A p>
 *             not positive), 3 a barrier wait gave up;
 *   rr_hist : device double[max_iter + 1] (nullable): rr_0 .. rr_k.
 * Arithmetic (binary32 vectors, binary64 scalars):
 *   r = b - A x; rr_0 = <r, r>; iteration k (while rr_k > tol^2 and
 *   k < max_iter): p = r (k = 0) or fmaf(beta, p, r) with
 *   beta = (float)(rr_k / rr_{k-1}); q = A p; stop if not <p, q> > 0;
 *   alpha = (float)(rr_k / <p, q>); x = fmaf(alpha, p, x);
 *   r = fmaf(-alpha, q, r); rr_{k+1} = <r, r>.
 *   (A v)_i: the row's entries in storage order, from +0.0f, with
 *   acc = fmaf(a_ij, v_j, acc).
 *   <u, v>: chunks of S = 32 * warps_per_block * items_per_lane rows; thread
 *   (w, l) adds the exact products (double)u_i * (double)v_i of rows
 *   cS + 32 W q + 32 w + l, q = 0 .. R-1, in FP64 from -0.0; the shfl_down
 *   tree per warp, then over the W warp values (-0.0 beyond W); the chunk
 *   values combined by the FP64 final tree of the reductions above.
 * Results depend on (items_per_lane, warps_per_block) only, never on the
 * grid, nor on where the kernel keeps its data.  With at most one chunk
 * per block, x, r, p and q stay in registers for the whole solve, and a
 * block whose rows fit in what shared memory the grid leaves (at most
 * 65535 entries) reads its rows of row_ptr, col_idx and val once; if every
 * such block's columns lie within 64 rows of its chunk, the blocks exchange
 * only those halo rows of r and p through memory.
 * cfg: items_per_lane 1, 2, 4 or 8, warps_per_block 8, 16 or 32
 * (COX_ERR_UNSUPPORTED otherwise), grid_blocks 0 = one block per compute
 * unit.  Malformed CSR (indices out of range) gives meaningless results
 * but no access outside the arrays.  n < 2^31 - 2^13, nnz < 2^31.
 * ws: cox_workspace_bytes(COX_OP_CG, COX_F32, n, 0, cfg). */
cox_status cox_cg_solve(const int32_t *row_ptr, const int32_t *col_idx, const float *val, int64_t n, int64_t nnz,
                        const float *b, float *x, int32_t max_iter, double tol, int32_t *result, double *rr_hist,
                        const cox_cfg *cfg, void *ws, size_t ws_bytes, void *stream);
/* The same solve as one launch per phase (2 per iteration, max_iter
 * enqueued; the launches after a stop return at once): the baseline
 * without grid barriers.  Identical results. */
cox_status cox_cg_solve_per_phase(const int32_t *row_ptr, const int32_t *col_idx, const float *val, int64_t n,
                                  int64_t nnz, const float *b, float *x, int32_t max_iter, double tol,
                                  int32_t *result, double *rr_hist, const cox_cfg *cfg, void *ws, size_t ws_bytes,
                                  void *stream);

/* ---------------------------------------------------------------------
 * Bandwidth reference kernels (measurement plumbing, not part of the
 * method, so no passage of the paper defines them): a plain read and
 * a plain copy with 16-byte accesses.  They give the achievable HBM
 * ceiling and the known-size reference for hardware byte counters.
 * bytes % 16 == 0; pointers 16-byte aligned; grid_blocks 0 = fill the
 * device.  cox_stream_read xors every word into *sink (device uint32).
 * ------------------------------------------------------------------- */
cox_status cox_stream_read(const void *x, size_t bytes, uint32_t *sink, int32_t grid_blocks, void *stream);
cox_status cox_stream_copy(const void *src, void *dst, size_t bytes, int32_t grid_blocks, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* COX_H */
