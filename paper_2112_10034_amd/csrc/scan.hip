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
// lane's own earlier slots; warp counts are scanned in shared memory and
// chunk offsets chained by the same look-back.
//
// Chunks are claimed from a ticket counter, so a chunk only ever waits for
// chunks that running blocks already hold.  Every block finally draws one
// ticket past the end; the block drawing the very last one (all others
// have finished) resets the counter and advances the epoch whose tag marks
// this call's status words, so the workspace needs no clearing between
// calls.  Every wait is bounded (MAX_SPIN); running out sets HDR_ERR.
#include "cox_internal.hpp"

namespace cox {

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

// Decoupled look-back, run by the 32 lanes of logical warp 0.  Publishes
// the chunk's aggregate, walks back over predecessor status words 32 at a
// time, and publishes the inclusive prefix.  Returns the exclusive prefix
// (same in every lane).
__device__ uint32_t lookback(int64_t c, uint32_t agg, uint64_t *__restrict__ status, uint32_t tag,
                             uint32_t *__restrict__ hdr) {
  const int l = llane();
  if (c == 0) {
    if (l == 0) st_dev(&status[0], st_pack(tag, ST_PREFIX, agg));
    return 0u;
  }
  if (l == 0) st_dev(&status[c], st_pack(tag, ST_AGG, agg));
  uint32_t run = 0u;
  int64_t top = c - 1;
  for (;;) {
    const int64_t idx = top - l;
    uint32_t flag = ST_PREFIX, val = 0u;
    if (idx >= 0) {
      uint64_t s = ld_dev(&status[idx]);
      uint32_t spins = 0;
      while (st_tag(s) != tag || st_flag(s) == 0u) {
        if (++spins >= MAX_SPIN || ((spins & 1023u) == 0u && ld_dev32(&hdr[HDR_ERR]) == tag)) {
          st_dev32(&hdr[HDR_ERR], tag);  // give up: result invalid, kernel still ends
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        s = ld_dev(&status[idx]);
      }
      flag = st_flag(s);
      val = st_val(s);
    }
    const uint32_t pm = ballot(flag == ST_PREFIX);
    if (pm) {
      const int p = __builtin_ctz(pm);
      run += warp_sum_u32(l <= p ? val : 0u);
      break;
    }
    run += warp_sum_u32(val);
    top -= 32;
  }
  if (l == 0) st_dev(&status[c], st_pack(tag, ST_PREFIX, agg + run));
  return run;
}

// last exit ticket: reset the ticket counter, advance the epoch
__device__ __forceinline__ void finish_call(uint32_t *hdr, uint32_t ticket, uint32_t last, uint32_t epoch) {
  if (ticket == last) {
    st_dev32(&hdr[HDR_TICKET], 0u);
    st_dev32(&hdr[HDR_EPOCH], epoch + 1u);
  }
}

template <int K>
__global__ __launch_bounds__(1024) void k_scan_i32(const int32_t *__restrict__ x, int32_t *__restrict__ y,
                                                   int64_t n, int64_t nch, uint64_t *__restrict__ status,
                                                   uint32_t *__restrict__ hdr) {
  constexpr int V = K < 4 ? K : 4;
  constexpr int R = K / V;
  __shared__ uint32_t s_epoch, s_ticket;
  __shared__ uint32_t s_w[32];
  const int W = blockDim.x >> 5;
  const int w = threadIdx.x >> 5, l = threadIdx.x & 31;
  const int64_t S = (int64_t)blockDim.x * K;
  if (threadIdx.x == 0) s_epoch = ld_epoch(hdr);

  for (;;) {
    if (threadIdx.x == 0) s_ticket = add_dev32(&hdr[HDR_TICKET], 1u);
    __syncthreads();
    const int64_t c = s_ticket;
    if (c >= nch) break;
    const uint32_t tag = tag_of_epoch(s_epoch);
    const int64_t wbase = c * S + (int64_t)w * 32 * K;
    const bool full = (c + 1) * S <= n;
    uint32_t v[R][V];
    if (full) {
#pragma unroll
      for (int i = 0; i < R; i++) {
        const int64_t e = wbase + (int64_t)(i * 32 + l) * V;
        if constexpr (V == 4) {
          const uint4 q = *(const uint4 *)(x + e);
          v[i][0] = q.x; v[i][1] = q.y; v[i][2] = q.z; v[i][3] = q.w;
        } else if constexpr (V == 2) {
          const uint2 q = *(const uint2 *)(x + e);
          v[i][0] = q.x; v[i][1] = q.y;
        } else {
          v[i][0] = (uint32_t)x[e];
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < R; i++)
#pragma unroll
        for (int j = 0; j < V; j++) {
          const int64_t e = wbase + (int64_t)(i * 32 + l) * V + j;
          v[i][j] = e < n ? (uint32_t)x[e] : 0u;
        }
    }
    // rows: lane prefix, warp scan of lane totals, running warp carry
    uint32_t carry = 0u;
#pragma unroll
    for (int i = 0; i < R; i++) {
#pragma unroll
      for (int j = 1; j < V; j++) v[i][j] += v[i][j - 1];
      const uint32_t r = v[i][V - 1];
      const uint32_t incl = warp_incl_scan_u32(r);
      const uint32_t add = carry + (incl - r);
#pragma unroll
      for (int j = 0; j < V; j++) v[i][j] += add;
      carry += (uint32_t)bcast31((int)incl);
    }
    if (l == 0) s_w[w] = carry;
    __syncthreads();
    if (w == 0) {
      const uint32_t a = l < W ? s_w[l] : 0u;
      const uint32_t incl = warp_incl_scan_u32(a);
      const uint32_t agg = (uint32_t)bcast31((int)incl);
      const uint32_t pre = lookback(c, agg, status, tag, hdr);
      if (l < W) s_w[l] = pre + (incl - a);
    }
    __syncthreads();
    const uint32_t off = s_w[w];
    if (full) {
#pragma unroll
      for (int i = 0; i < R; i++) {
        const int64_t e = wbase + (int64_t)(i * 32 + l) * V;
        if constexpr (V == 4) {
          st_stream4(y + e, v[i][0] + off, v[i][1] + off, v[i][2] + off, v[i][3] + off);
        } else if constexpr (V == 2) {
          uint2 q;
          q.x = v[i][0] + off; q.y = v[i][1] + off;
          *(uint2 *)(y + e) = q;
        } else {
          y[e] = (int32_t)(v[i][0] + off);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < R; i++)
#pragma unroll
        for (int j = 0; j < V; j++) {
          const int64_t e = wbase + (int64_t)(i * 32 + l) * V + j;
          if (e < n) y[e] = (int32_t)(v[i][j] + off);
        }
    }
  }
  if (threadIdx.x == 0) finish_call(hdr, s_ticket, (uint32_t)(nch + gridDim.x - 1), s_epoch);
}

template <int K>
__global__ __launch_bounds__(1024) void k_compact_i32(const int32_t *__restrict__ x, int32_t *__restrict__ out,
                                                      long long *__restrict__ count, int64_t n, int64_t nch,
                                                      uint64_t *__restrict__ status, uint32_t *__restrict__ hdr) {
  constexpr int V = K < 4 ? K : 4;
  constexpr int R = K / V;
  __shared__ uint32_t s_epoch, s_ticket;
  __shared__ uint32_t s_w[32];
  const int W = blockDim.x >> 5;
  const int w = threadIdx.x >> 5, l = threadIdx.x & 31;
  const int64_t S = (int64_t)blockDim.x * K;
  if (threadIdx.x == 0) s_epoch = ld_epoch(hdr);

  for (;;) {
    if (threadIdx.x == 0) s_ticket = add_dev32(&hdr[HDR_TICKET], 1u);
    __syncthreads();
    const int64_t c = s_ticket;
    if (c >= nch) break;
    const uint32_t tag = tag_of_epoch(s_epoch);
    const int64_t wbase = c * S + (int64_t)w * 32 * K;
    const bool full = (c + 1) * S <= n;
    int32_t v[R][V];
    if (full) {
#pragma unroll
      for (int i = 0; i < R; i++) {
        const int64_t e = wbase + (int64_t)(i * 32 + l) * V;
        if constexpr (V == 4) {
          const int4 q = *(const int4 *)(x + e);
          v[i][0] = q.x; v[i][1] = q.y; v[i][2] = q.z; v[i][3] = q.w;
        } else if constexpr (V == 2) {
          const int2 q = *(const int2 *)(x + e);
          v[i][0] = q.x; v[i][1] = q.y;
        } else {
          v[i][0] = x[e];
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < R; i++)
#pragma unroll
        for (int j = 0; j < V; j++) {
          const int64_t e = wbase + (int64_t)(i * 32 + l) * V + j;
          v[i][j] = e < n ? x[e] : 0;
        }
    }
    // warp-local ranks from ballots
    const uint32_t lt = lanemask_lt();
    uint32_t rank[R][V];
    uint32_t run = 0u;
#pragma unroll
    for (int i = 0; i < R; i++) {
      uint32_t base = 0u, rowcnt = 0u, own = 0u;
#pragma unroll
      for (int j = 0; j < V; j++) {
        const uint32_t B = ballot(v[i][j] > 0);
        base += __popc(B & lt);
        rowcnt += __popc(B);
      }
#pragma unroll
      for (int j = 0; j < V; j++) {
        rank[i][j] = run + base + own;
        own += v[i][j] > 0 ? 1u : 0u;
      }
      run += rowcnt;
    }
    if (l == 0) s_w[w] = run;
    __syncthreads();
    if (w == 0) {
      const uint32_t a = l < W ? s_w[l] : 0u;
      const uint32_t incl = warp_incl_scan_u32(a);
      const uint32_t agg = (uint32_t)bcast31((int)incl);
      const uint32_t pre = lookback(c, agg, status, tag, hdr);
      if (l < W) s_w[l] = pre + (incl - a);
      if (c == nch - 1 && l == 0) *count = (long long)pre + (long long)agg;
    }
    __syncthreads();
    const uint32_t off = s_w[w];
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
      for (int j = 0; j < V; j++) {
        // the bound only matters if a look-back wait gave up (HDR_ERR set)
        const uint64_t pos = (uint64_t)off + rank[i][j];
        if (v[i][j] > 0 && pos < (uint64_t)n) out[pos] = v[i][j];
      }
  }
  if (threadIdx.x == 0) {
    if (nch == 0 && s_ticket == (uint32_t)(gridDim.x - 1)) *count = 0;
    finish_call(hdr, s_ticket, (uint32_t)(nch + gridDim.x - 1), s_epoch);
  }
}

using scan_fn = void (*)(const int32_t *, int32_t *, int64_t, int64_t, uint64_t *, uint32_t *);
using compact_fn = void (*)(const int32_t *, int32_t *, long long *, int64_t, int64_t, uint64_t *, uint32_t *);

static scan_fn pick_scan(int k) {
  switch (k) {
  case 1: return k_scan_i32<1>;
  case 2: return k_scan_i32<2>;
  case 4: return k_scan_i32<4>;
  case 8: return k_scan_i32<8>;
  case 16: return k_scan_i32<16>;
  case 32: return k_scan_i32<32>;
  }
  return nullptr;
}
static compact_fn pick_compact(int k) {
  switch (k) {
  case 1: return k_compact_i32<1>;
  case 2: return k_compact_i32<2>;
  case 4: return k_compact_i32<4>;
  case 8: return k_compact_i32<8>;
  case 16: return k_compact_i32<16>;
  case 32: return k_compact_i32<32>;
  }
  return nullptr;
}

static cox_status check_lookback_call(cox_op op, int64_t n, const void *x, const cox_cfg *cfg, void *ws,
                                      size_t ws_bytes, Sigma *sg, int64_t *nch) {
  if (n < 0) return COX_ERR_INVALID;
  cox_status st = resolve_cfg(op, COX_I32, cfg, sg);
  if (st != COX_OK) return st;
  if (n > 0 && !x) return COX_ERR_INVALID;
  if (n > 0 && !aligned16(x)) return COX_ERR_ALIGN;
  const int64_t S = (int64_t)32 * sg->W * sg->k;
  *nch = (n + S - 1) / S;
  // tickets and counts are 32-bit
  if (*nch > (int64_t)0x7fffffff - 65536 || n > (int64_t)0xffffffffLL) return COX_ERR_INVALID;
  if (!ws || ws_bytes < cox_workspace_bytes(op, COX_I32, n, 0, cfg)) return COX_ERR_WORKSPACE;
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
  scan_fn fn = pick_scan(sg.k);
  if (!fn) return COX_ERR_UNSUPPORTED;
  const int block = 32 * sg.W;
  const int grid = persistent_grid((const void *)fn, block, nch, sg.G);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(block), 0, (hipStream_t)stream, x, y, n, nch,
                     (uint64_t *)((char *)ws + WS_HEADER), (uint32_t *)ws);
  return launch_status();
}

cox_status cox_ballot_compact(const int32_t *x, int64_t n, int32_t *out, int64_t *count,
                              const cox_cfg *cfg, void *ws, size_t ws_bytes, void *stream) {
  Sigma sg;
  int64_t nch;
  cox_status st = check_lookback_call(COX_OP_COMPACT, n, x, cfg, ws, ws_bytes, &sg, &nch);
  if (st != COX_OK) return st;
  if (!count || (n > 0 && !out)) return COX_ERR_INVALID;
  compact_fn fn = pick_compact(sg.k);
  if (!fn) return COX_ERR_UNSUPPORTED;
  const int block = 32 * sg.W;
  const int grid = persistent_grid((const void *)fn, block, nch > 0 ? nch : 1, sg.G);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(block), 0, (hipStream_t)stream, x, out, (long long *)count, n,
                     nch, (uint64_t *)((char *)ws + WS_HEADER), (uint32_t *)ws);
  return launch_status();
}

}  // extern "C"
