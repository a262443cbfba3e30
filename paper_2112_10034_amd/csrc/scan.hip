// Single-pass int32 inclusive scan and ballot compaction.
//
// Chunk layout (schedule sigma = (k, W)): warp w of the block owns the 32k
// consecutive elements [c*S + 32kw, c*S + 32k(w+1)); in row i lane l holds
// the V consecutive elements at offset (32i + l) * V of that range, loaded
// as one 16-byte vector.
//
// Scan: per row, a lane-serial prefix over its V elements, a Kogge-Stone
// shfl_up scan of the lane totals (DPP row_shr:1,2,4,8 inside each 16-lane
// row, then row_bcast:15 carries row 0's total into row 1 -- never across
// lanes 31 -> 32), and the row total from logical lane 31; warp totals meet
// in shared memory, warp 0 scans them, and the chunk's exclusive prefix
// comes from a decoupled look-back (Merrill and Garland) over status words
// [tag | flag | value] published with device-scope atomics.
//
// Compaction: p = (x > 0); per row and vector slot v a ballot B_v; the
// rank of (l, v) inside the row is sum_v' popc(B_v' & lanemask_lt) plus the
// lane's own earlier slots (mbcnt over the wave's 64-bit ballots).  Kept
// elements are staged in the warp's own shared-memory region at their rank
// (the others in a trash slot, without branches), warp counts are scanned
// in shared memory, chunk offsets chained by the same look-back, and each
// warp then
// writes its run in 16-byte vectors aligned in global memory (the run's
// ragged first and last vectors element by element).
//
// Chunks are claimed from a ticket counter, so a chunk only ever waits for
// chunks that running blocks already hold.  Every block finally draws one
// ticket past the end; the block drawing the very last one (all others
// have finished) resets the counter and advances the epoch whose tag marks
// this call's status words, so the workspace needs no clearing between
// calls.  Every wait is bounded (MAX_SPIN); running out sets HDR_ERR.
#include <mutex>

#include "cox_internal.hpp"

namespace cox {

// 16-byte vectors at 4-byte aligned addresses (one dwordx4 access each)
typedef uint32_t u32x4u __attribute__((ext_vector_type(4), aligned(4)));

// inclusive scan of v over the 32 lanes of the logical warp (integers)
__device__ __forceinline__ uint32_t warp_incl_scan_u32(uint32_t v) {
  v += (uint32_t)dpp<DPP_ROW_SHR1>(0, (int)v);
  v += (uint32_t)dpp<DPP_ROW_SHR2>(0, (int)v);
  v += (uint32_t)dpp<DPP_ROW_SHR4>(0, (int)v);
  v += (uint32_t)dpp<DPP_ROW_SHR8>(0, (int)v);
  v += (uint32_t)dpp<DPP_ROW_BCAST15, 0xa>(0, (int)v);
  return v;
}

__device__ __forceinline__ uint32_t warp_sum_u32(uint32_t v) {
  v += (uint32_t)xor_lane<16>((int)v);
  v += (uint32_t)xor_lane<8>((int)v);
  v += (uint32_t)xor_lane<4>((int)v);
  v += (uint32_t)xor_lane<2>((int)v);
  v += (uint32_t)xor_lane<1>((int)v);
  return v;
}

// Decoupled look-back, run by the 32 lanes of logical warp 0, in two
// halves so that other loads can be issued in between: lookback_begin
// publishes the chunk's aggregate and requests the first window of
// predecessor status words (lane l reads chunk c - 1 - l); lookback_end
// waits for them, walks further back 32 chunks at a time until a lane
// finds an inclusive prefix, and publishes the chunk's inclusive prefix.
// Returns the exclusive prefix (same in every lane).
__device__ __forceinline__ uint64_t lookback_begin(int64_t c, uint32_t agg, uint64_t *__restrict__ status,
                                                   int64_t sst, uint32_t tag) {
  const int l = llane();
  if (c == 0) {
    if (l == 0) st_dev(&status[0], st_pack(tag, ST_PREFIX, agg));
    return 0;
  }
  if (l == 0) st_dev(&status[c * sst], st_pack(tag, ST_AGG, agg));
  const int64_t idx = c - 1 - l;
  return idx >= 0 ? ld_dev(&status[idx * sst]) : st_pack(tag, ST_PREFIX, 0u);
}

__device__ uint32_t lookback_end(int64_t c, uint32_t agg, uint64_t first, uint64_t *__restrict__ status,
                                 int64_t sst, uint32_t tag, uint32_t *__restrict__ hdr) {
  const int l = llane();
  if (c == 0) return 0u;
  uint32_t run = 0u;
  int64_t top = c - 1;
  uint64_t s = first;
  for (;;) {
    const int64_t idx = top - l;
    if (idx >= 0) {
      uint32_t spins = 0;
      while (st_tag(s) != tag || st_flag(s) == 0u) {
        if (++spins >= MAX_SPIN || ((spins & 1023u) == 0u && ld_dev32(&hdr[HDR_ERR]) == tag)) {
          st_dev32(&hdr[HDR_ERR], tag);  // give up: result invalid, kernel still ends
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        s = ld_dev(&status[idx * sst]);
      }
    }
    const uint32_t flag = st_flag(s), val = st_val(s);
    const uint32_t pm = ballot(flag == ST_PREFIX);
    if (pm) {
      const int p = __builtin_ctz(pm);
      run += warp_sum_u32(l <= p ? val : 0u);
      break;
    }
    run += warp_sum_u32(val);
    top -= 32;
    s = top - l >= 0 ? ld_dev(&status[(top - l) * sst]) : st_pack(tag, ST_PREFIX, 0u);
  }
  if (l == 0) st_dev(&status[c * sst], st_pack(tag, ST_PREFIX, agg + run));
  return run;
}

// last exit ticket: reset the ticket counter, advance the epoch
__device__ __forceinline__ void finish_call(uint32_t *hdr, uint32_t ticket, uint32_t last, uint32_t epoch) {
  if (ticket == last) {
    st_dev32(&hdr[HDR_TICKET], 0u);
    st_dev32(&hdr[HDR_EPOCH], epoch + 1u);
  }
}

enum { MODE_SCAN = 0, MODE_COMPACT = 1 };

// One kernel for both look-back operations.  Per block: draw a ticket,
// then for every full chunk c: (1) row work on c's registers (scan: lane
// prefixes, warp scans, warp carry; compaction: ballots, ranks, warp
// count), (2) draw the next ticket and request its vectors into the other
// register buffer (a ticket past the full chunks reloads c, which is
// always valid, so the loads are unconditional), (3) warp 0 scans the warp
// values and runs the look-back, (4) outputs of c.  The partial last chunk
// is handled after the loop with element-wise bounds.
template <int K, int MODE>
__global__ __launch_bounds__(1024) void k_lookback(const int32_t *__restrict__ x, int32_t *__restrict__ out,
                                                   long long *__restrict__ count, int64_t n, int64_t nch,
                                                   uint64_t *__restrict__ status, int64_t sst,
                                                   uint32_t *__restrict__ hdr) {
  constexpr int V = K < 4 ? K : 4;
  constexpr int R = K / V;
  __shared__ uint32_t s_epoch, s_tk[2];
  __shared__ uint32_t s_w[32];
  extern __shared__ int32_t s_stage[];  // compaction: 32K elements per warp
  const int W = blockDim.x >> 5;
  const int w = threadIdx.x >> 5, l = threadIdx.x & 31;
  const int64_t S = (int64_t)blockDim.x * K;
  const int64_t nfull = n / S;
  if (threadIdx.x == 0) {
    s_epoch = ld_epoch(hdr);
    s_tk[0] = add_dev32(&hdr[HDR_TICKET], 1u);
  }
  __syncthreads();
  const uint32_t epoch = s_epoch;
  const uint32_t tag = tag_of_epoch(epoch);
  const bool hi_half = lhalf() != 0;

  // vectors of chunk c; with dummy set every lane reads the array's first
  // vector instead (a ticket past the full chunks: keeps the loads
  // unconditional while fetching a single line)
  auto load_full = [&](int64_t c, uint32_t (&v)[R][V], bool dummy) {
    // one base pointer and one row stride per lane (not a select per load)
    const int32_t *src = x + (dummy ? 0 : c * S + (int64_t)w * 32 * K + l * V);
    const int rstride = dummy ? 0 : 32 * V;
#pragma unroll
    for (int i = 0; i < R; i++) {
      const int32_t *p = src + i * rstride;
      if constexpr (V == 4) {
        const u32x4 q = ld_stream4(p);
        v[i][0] = q.x; v[i][1] = q.y; v[i][2] = q.z; v[i][3] = q.w;
      } else if constexpr (V == 2) {
        const u32x2 q = ld_stream2(p);
        v[i][0] = q.x; v[i][1] = q.y;
      } else {
        v[i][0] = ld_stream1(p);
      }
    }
  };
  auto load_tail = [&](int64_t c, uint32_t (&v)[R][V]) {
    const int64_t wbase = c * S + (int64_t)w * 32 * K;
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
      for (int j = 0; j < V; j++) {
        const int64_t e = wbase + (int64_t)(i * 32 + l) * V + j;
        v[i][j] = e < n ? ld_stream1(x + e) : 0u;
      }
  };

  // process chunk c held in cur; when `full`, prefetch the next ticket's
  // chunk into nxt.  Returns the next ticket.
  auto process = [&](int64_t c, uint32_t (&cur)[R][V], uint32_t (&nxt)[R][V], bool full) -> int64_t {
    uint32_t wval = 0u;  // warp carry (scan) or warp count (compaction)
    if constexpr (MODE == MODE_SCAN) {
#pragma unroll
      for (int i = 0; i < R; i++) {
#pragma unroll
        for (int j = 1; j < V; j++) cur[i][j] += cur[i][j - 1];
        const uint32_t r = cur[i][V - 1];
        const uint32_t incl = warp_incl_scan_u32(r);
        const uint32_t add = wval + (incl - r);
#pragma unroll
        for (int j = 0; j < V; j++) cur[i][j] += add;
        wval += (uint32_t)bcast31((int)incl);
      }
    } else {
      // ranks inside the warp from ballots: the wave's 64-bit ballot, lanes
      // below counted by mbcnt (an upper-half lane also counts the whole
      // lower half, subtracted once per row); kept elements go to the
      // warp's own shared-memory region at their rank, the others to the
      // lane's trash slot past the region (no branches).  The region is
      // written and later read by the same warp: no block barrier.
      int32_t *region = s_stage + w * (32 * K + 32);
      const uint32_t trash = 32 * K + l;
#pragma unroll
      for (int i = 0; i < R; i++) {
        uint32_t base = 0u, lo_cnt = 0u, hi_cnt = 0u;
#pragma unroll
        for (int j = 0; j < V; j++) {
          const uint64_t B = __builtin_amdgcn_ballot_w64((int32_t)cur[i][j] > 0);
          base = __builtin_amdgcn_mbcnt_hi((uint32_t)(B >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)B, base));
          lo_cnt += __builtin_popcount((uint32_t)B);
          hi_cnt += __builtin_popcount((uint32_t)(B >> 32));
        }
        if (hi_half) base -= lo_cnt;
        uint32_t pos = wval + base;
#pragma unroll
        for (int j = 0; j < V; j++) {
          const bool k = (int32_t)cur[i][j] > 0;
          region[k ? pos : trash] = (int32_t)cur[i][j];
          pos += k ? 1u : 0u;
        }
        wval += hi_half ? hi_cnt : lo_cnt;
      }
    }
    if (l == 0) s_w[w] = wval;
    if (threadIdx.x == 0) s_tk[1] = add_dev32(&hdr[HDR_TICKET], 1u);
    __syncthreads();
    const int64_t cn = s_tk[1];
    // warp 0: scan of the warp values, aggregate published, first window
    // of predecessor words requested -- before this block's prefetch, so
    // that waiting for the window does not also wait for the prefetch
    uint32_t wa = 0u, wincl = 0u, agg = 0u;
    uint64_t first = 0;
    if (w == 0) {
      wa = l < W ? s_w[l] : 0u;
      wincl = warp_incl_scan_u32(wa);
      agg = (uint32_t)bcast31((int)wincl);
      first = lookback_begin(c, agg, status, sst, tag);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (full) load_full(cn, nxt, cn >= nfull);
    __builtin_amdgcn_sched_barrier(0);
    if (w == 0) {
      const uint32_t pre = lookback_end(c, agg, first, status, sst, tag, hdr);
      if (l < W) s_w[l] = pre + (wincl - wa);
      if constexpr (MODE == MODE_COMPACT)
        if (c == nch - 1 && l == 0) *count = (long long)pre + (long long)agg;
    }
    __syncthreads();
    const uint32_t off = s_w[w];
    const int64_t wbase = c * S + (int64_t)w * 32 * K;
    if constexpr (MODE == MODE_SCAN) {
      if (full) {
#pragma unroll
        for (int i = 0; i < R; i++) {
          const int64_t e = wbase + (int64_t)(i * 32 + l) * V;
          if constexpr (V == 4) {
            st_stream4(out + e, cur[i][0] + off, cur[i][1] + off, cur[i][2] + off, cur[i][3] + off);
          } else if constexpr (V == 2) {
            st_stream2(out + e, cur[i][0] + off, cur[i][1] + off);
          } else {
            st_stream1(out + e, cur[i][0] + off);
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < R; i++)
#pragma unroll
          for (int j = 0; j < V; j++) {
            const int64_t e = wbase + (int64_t)(i * 32 + l) * V + j;
            if (e < n) out[e] = (int32_t)(cur[i][j] + off);
          }
      }
    } else {
      // the warp writes its kept run [off, off + wval) from its region in
      // 16-byte vectors aligned in global memory: lane j takes positions
      // [A + 4j, A + 4j + 4) of each 128-position step, A = off rounded down
      // to a multiple of 4; the run's partial first and last vectors are
      // written element by element.  Offsets below are relative to A.
      const int32_t *region = s_stage + w * (32 * K + 32);
      const uint64_t A = (uint64_t)off & ~(uint64_t)3;
      const uint32_t head = (uint32_t)((uint64_t)off - A);  // 0..3 positions before the run
      uint32_t span = head + wval;
      // the bound on n only matters if a look-back wait gave up
      if (A + span > (uint64_t)n) span = A < (uint64_t)n ? (uint32_t)((uint64_t)n - A) : 0u;
      int32_t *dst = out + A;
      for (uint32_t t = 4u * (uint32_t)l; t < span; t += 128u) {
        if (t >= head && t + 4u <= span) {
          const u32x4u v = *(const u32x4u *)(region + (t - head));
          *(u32x4u *)(dst + t) = v;
        } else {
#pragma unroll
          for (uint32_t j = 0; j < 4u; j++)
            if (t + j >= head && t + j < span) dst[t + j] = region[t + j - head];
        }
      }
    }
    return cn;
  };

  int64_t c = s_tk[0];
  uint32_t A[R][V], B[R][V];
  if (c < nfull) {
    load_full(c, A, false);
    for (;;) {
      c = process(c, A, B, true);
      if (c >= nfull) break;
      c = process(c, B, A, true);
      if (c >= nfull) break;
    }
  }
  if (c < nch) {  // the partial last chunk
    load_tail(c, A);
    c = process(c, A, B, false);
  }
  if (threadIdx.x == 0) {
    if constexpr (MODE == MODE_COMPACT)
      if (nch == 0 && c == (int64_t)gridDim.x - 1) *count = 0;
    finish_call(hdr, (uint32_t)c, (uint32_t)(nch + gridDim.x - 1), epoch);
  }
}

using lb_fn = void (*)(const int32_t *, int32_t *, long long *, int64_t, int64_t, uint64_t *, int64_t,
                       uint32_t *);

template <int MODE>
static lb_fn pick_lb(int k) {
  switch (k) {
  case 1: return k_lookback<1, MODE>;
  case 2: return k_lookback<2, MODE>;
  case 4: return k_lookback<4, MODE>;
  case 8: return k_lookback<8, MODE>;
  case 16: return k_lookback<16, MODE>;
  case 32: return k_lookback<32, MODE>;
  }
  return nullptr;
}

static cox_status check_lookback_args(cox_op op, int64_t n, const void *x, const cox_cfg *cfg, Sigma *sg,
                                      int64_t *nch) {
  if (n < 0) return COX_ERR_INVALID;
  cox_status st = resolve_cfg(op, COX_I32, cfg, sg);
  if (st != COX_OK) return st;
  if (n > 0 && !x) return COX_ERR_INVALID;
  if (n > 0 && !aligned16(x)) return COX_ERR_ALIGN;
  const int64_t S = (int64_t)32 * sg->W * sg->k;
  *nch = (n + S - 1) / S;
  // tickets and counts are 32-bit
  if (*nch > (int64_t)0x7fffffff - 65536 || n > (int64_t)0xffffffffLL) return COX_ERR_INVALID;
  return COX_OK;
}

static cox_status check_lookback_call(cox_op op, int64_t n, const void *x, const cox_cfg *cfg, void *ws,
                                      size_t ws_bytes, Sigma *sg, int64_t *nch) {
  const cox_status st = check_lookback_args(op, n, x, cfg, sg, nch);
  if (st != COX_OK) return st;
  if (!ws || ws_bytes < cox_workspace_bytes(op, COX_I32, n, 0, cfg)) return COX_ERR_WORKSPACE;
  return COX_OK;
}

// ------------------------------------------------ allocation-free variant
// The look-back header and status words of cox_warp_scan_noalloc live in a
// file-scope device array.  Each device that runs the library holds its own
// copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns on that device.
constexpr size_t SCRATCH_BYTES = COX_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];

__global__ void k_scratch_clear(uint32_t *p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// hands the call's bounded-wait status to the caller and clears it
__global__ void k_scratch_status(uint32_t *hdr, uint32_t *err_out) {
  if (threadIdx.x == 0) {
    *err_out = hdr[HDR_ERR];
    hdr[HDR_ERR] = 0u;
  }
}

// Device address of this device's scratch.  The first call on a device
// looks it up and zeroes it on `st`, ahead of that call's kernels.
static cox_status scratch_for_device(hipStream_t st, void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_hip_error(e);
    return COX_ERR_HIP;
  }
  if (dev < 0 || dev >= MAX_DEVICES) return COX_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
      return COX_ERR_HIP;
    }
    const int64_t words = (int64_t)(SCRATCH_BYTES / 4);
    hipLaunchKernelGGL(k_scratch_clear, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st, (uint32_t *)ptr,
                       words);
    const cox_status ls = launch_status();
    if (ls != COX_OK) return ls;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return COX_OK;
}

}  // namespace cox

using namespace cox;

extern "C" {

cox_status cox_warp_scan(const int32_t *x, int32_t *y, int64_t n, const cox_cfg *cfg, void *ws,
                         size_t ws_bytes, void *stream) {
  Sigma sg;
  int64_t nch;
  cox_status st = check_lookback_call(COX_OP_SCAN, n, x, cfg, ws, ws_bytes, &sg, &nch);
  if (st != COX_OK) return st;
  if (n == 0) return COX_OK;
  if (!y) return COX_ERR_INVALID;
  if (!aligned16(y)) return COX_ERR_ALIGN;
  lb_fn fn = pick_lb<MODE_SCAN>(sg.k);
  if (!fn) return COX_ERR_UNSUPPORTED;
  const int block = 32 * sg.W;
  const int grid = persistent_grid((const void *)fn, block, nch, sg.G);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(block), 0, (hipStream_t)stream, x, y, (long long *)nullptr, n, nch,
                     (uint64_t *)((char *)ws + WS_HEADER), (int64_t)ST_STRIDE, (uint32_t *)ws);
  return launch_status();
}

cox_status cox_warp_scan_noalloc(const int32_t *x, int32_t *y, int64_t n, const cox_cfg *cfg, uint32_t *err_out,
                                 void *stream) {
  Sigma sg;
  int64_t nch;
  cox_status st = check_lookback_args(COX_OP_SCAN, n, x, cfg, &sg, &nch);
  if (st != COX_OK) return st;
  // status words packed 8 bytes apart (a workspace spaces them ST_STRIDE
  // words apart), so that 1 MiB covers every n the default schedule takes
  if (WS_HEADER + 8 * (size_t)(nch + 1) > SCRATCH_BYTES) return COX_ERR_WORKSPACE;
  if (n > 0 && !y) return COX_ERR_INVALID;
  if (n > 0 && !aligned16(y)) return COX_ERR_ALIGN;
  lb_fn fn = pick_lb<MODE_SCAN>(sg.k);
  if (!fn) return COX_ERR_UNSUPPORTED;
  const hipStream_t hs = (hipStream_t)stream;
  void *ws = nullptr;
  st = scratch_for_device(hs, &ws);
  if (st != COX_OK) return st;
  if (n > 0) {
    const int block = 32 * sg.W;
    const int grid = persistent_grid((const void *)fn, block, nch, sg.G);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(block), 0, hs, x, y, (long long *)nullptr, n, nch,
                       (uint64_t *)((char *)ws + WS_HEADER), (int64_t)1, (uint32_t *)ws);
    st = launch_status();
    if (st != COX_OK) return st;
  }
  if (err_out) {
    hipLaunchKernelGGL(k_scratch_status, dim3(1), dim3(64), 0, hs, (uint32_t *)ws, err_out);
    st = launch_status();
  }
  return st;
}

cox_status cox_ballot_compact(const int32_t *x, int64_t n, int32_t *out, int64_t *count,
                              const cox_cfg *cfg, void *ws, size_t ws_bytes, void *stream) {
  Sigma sg;
  int64_t nch;
  cox_status st = check_lookback_call(COX_OP_COMPACT, n, x, cfg, ws, ws_bytes, &sg, &nch);
  if (st != COX_OK) return st;
  if (!count || (n > 0 && !out)) return COX_ERR_INVALID;
  lb_fn fn = pick_lb<MODE_COMPACT>(sg.k);
  if (!fn) return COX_ERR_UNSUPPORTED;
  const int block = 32 * sg.W;
  const size_t lds = (size_t)sg.W * (32 * sg.k + 32) * sizeof(int32_t) + 256;  // staging (+ trash) + static
  if (lds > device_max_lds()) return COX_ERR_UNSUPPORTED;
  if (lds - 256 > 64 * 1024 &&
      hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(lds - 256)) != hipSuccess)
    return COX_ERR_UNSUPPORTED;
  const int grid = persistent_grid((const void *)fn, block, nch > 0 ? nch : 1, sg.G, lds);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(block), lds - 256, (hipStream_t)stream, x, out, (long long *)count, n,
                     nch, (uint64_t *)((char *)ws + WS_HEADER), (int64_t)ST_STRIDE, (uint32_t *)ws);
  return launch_status();
}

}  // extern "C"
