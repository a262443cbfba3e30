// Warp-shuffle reductions.
//
// k_reduce_blocks_i32: 256-thread blocks of 8 logical warps, one element
// per thread; shfl_down tree per warp, ballot(x > 0) per warp, shared-memory
// combine of the 8 warp values by warp 0 (the SDK reduction pattern that
// COX's Code 1 simplifies, Sec. 2.3).
//
// k_reduce: chunked sum / dot under the fixed schedule sigma = (k, W)
// (documented in cox.h); persistent blocks walk chunks c = b, b + G, ...;
// every chunk partial is published as a 64-bit word [tag | value bits]
// with a device-scope atomic store (tag = this call's epoch), and the last
// block to finish (device-scope counter) collects the words, checking each
// tag, and runs the FP64 (or int64) final combine.  No memory fences are
// needed: a word with the current tag can only hold this call's partial,
// and the last block resets the counter and advances the epoch only after
// it has seen every block's words, whose tags every block derived from its
// own read of the epoch.
//
// The shfl_down tree is evaluated at lane 0, which only ever reads
// in-range sources (offset o reads lanes below 2o); the exchanges use the
// xor partner l ^ o, which for every lane l < o is exactly l + o, so lane
// 0's value is the one CUDA's __shfl_down_sync tree produces, bit for bit.
#include "cox_internal.hpp"

namespace cox {

// ---------------------------------------------------------------- K-R0
__device__ __forceinline__ uint32_t tree_u32(uint32_t v) {
  v += (uint32_t)xor_lane<16>((int)v);
  v += (uint32_t)xor_lane<8>((int)v);
  v += (uint32_t)xor_lane<4>((int)v);
  v += (uint32_t)xor_lane<2>((int)v);
  v += (uint32_t)xor_lane<1>((int)v);
  return v;
}

__global__ __launch_bounds__(256) void k_reduce_blocks_i32(const int32_t *__restrict__ x, int64_t n,
                                                           int32_t *__restrict__ bsum,
                                                           int32_t *__restrict__ wpos) {
  __shared__ uint32_t slot[8];
  const int t = threadIdx.x, w = t >> 5, l = t & 31;
  const int64_t e = (int64_t)blockIdx.x * 256 + t;
  const int32_t xv = e < n ? x[e] : 0;
  uint32_t v = tree_u32((uint32_t)xv);
  const uint32_t b = ballot(xv > 0);
  if (l == 0) {
    const int64_t g = (int64_t)blockIdx.x * 8 + w;
    if (32 * g < n) wpos[g] = __popc(b);
    slot[w] = v;
  }
  __syncthreads();
  if (w == 0) {
    uint32_t a = l < 8 ? slot[l] : 0u;
    a = tree_u32(a);
    if (l == 0) bsum[blockIdx.x] = (int32_t)a;
  }
}

// ---------------------------------------------------------------- chunked reduce
enum { DT_I32 = COX_I32, DT_F32 = COX_F32, DT_BF16 = COX_BF16 };
enum { OP_SUM = 0, OP_DOT = 1 };

template <int DT> struct ElemT;
template <> struct ElemT<DT_I32> { static constexpr int size = 4; };
template <> struct ElemT<DT_F32> { static constexpr int size = 4; };
template <> struct ElemT<DT_BF16> { static constexpr int size = 2; };

// raw 32-bit value of element v of a vector of V elements (bfloat16 widened)
template <int ESZ, int V>
__device__ __forceinline__ void load_vec(const void *__restrict__ base, int64_t idx, uint32_t (&r)[V]) {
  constexpr int BYTES = ESZ * V;
  const char *p = (const char *)base + idx * ESZ;
  uint32_t w[(BYTES + 3) / 4];
  if constexpr (BYTES == 16) {
    const u32x4 q = ld_stream4(p);
    w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
  } else if constexpr (BYTES == 8) {
    const u32x2 q = ld_stream2(p);
    w[0] = q.x; w[1] = q.y;
  } else if constexpr (BYTES == 4) {
    w[0] = ld_stream1(p);
  } else {
    w[0] = ld_stream_h(p);
  }
  if constexpr (ESZ == 4) {
#pragma unroll
    for (int v = 0; v < V; v++) r[v] = w[v];
  } else {
#pragma unroll
    for (int v = 0; v < V; v++) r[v] = (v & 1) ? (w[v >> 1] & 0xffff0000u) : (w[v >> 1] << 16);
  }
}

template <int ESZ>
__device__ __forceinline__ uint32_t load_one(const void *__restrict__ base, int64_t idx) {
  if constexpr (ESZ == 4) return ld_stream1((const uint32_t *)base + idx);
  else return (uint32_t)ld_stream_h((const uint16_t *)base + idx) << 16;
}

// per-lane accumulator
struct Acc {
  float s, c;
  uint32_t i;
};

template <int DT, int ACC>
__device__ __forceinline__ Acc acc_identity() {
  Acc a;
  a.s = -0.0f;
  a.c = -0.0f;
  a.i = 0u;
  return a;
}

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  float ss = a + b;
  float bb = ss - a;
  e = (a - (ss - bb)) + (b - bb);
  s = ss;
}

template <int DT, int OP, int ACC>
__device__ __forceinline__ void acc_step(Acc &a, uint32_t xr, uint32_t yr) {
  if constexpr (DT == DT_I32) {
    a.i += xr;
  } else {
    const float xv = i2f((int)xr);
    if constexpr (OP == OP_SUM) {
      if constexpr (ACC == COX_ACC_PLAIN) {
        a.s = a.s + xv;
      } else {
        float s, e;
        two_sum(a.s, xv, s, e);
        a.s = s;
        a.c = a.c + e;
      }
    } else {
      const float yv = i2f((int)yr);
      if constexpr (ACC == COX_ACC_PLAIN) {
        a.s = __builtin_fmaf(xv, yv, a.s);
      } else {
        const float p = xv * yv;
        const float pe = __builtin_fmaf(xv, yv, -p);
        float s, q;
        two_sum(a.s, p, s, q);
        a.s = s;
        a.c = a.c + (pe + q);
      }
    }
  }
}

// combine own value with the partner's (own operand first)
template <int DT, int ACC>
__device__ __forceinline__ Acc acc_combine(Acc a, Acc b) {
  if constexpr (DT == DT_I32) {
    a.i += b.i;
  } else if constexpr (ACC == COX_ACC_PLAIN) {
    a.s = a.s + b.s;
  } else {
    float s, e;
    two_sum(a.s, b.s, s, e);
    a.c = (a.c + b.c) + e;
    a.s = s;
  }
  return a;
}

template <int M, int DT, int ACC>
__device__ __forceinline__ Acc acc_xor(Acc a) {
  Acc r = a;
  if constexpr (DT == DT_I32) {
    r.i = (uint32_t)xor_lane<M>((int)a.i);
  } else {
    r.s = xor_lane_f<M>(a.s);
    if constexpr (ACC == COX_ACC_TWOSUM) r.c = xor_lane_f<M>(a.c);
  }
  return r;
}

// shfl_down tree, offsets 16, 8, 4, 2, 1 (value valid at lane 0)
template <int DT, int ACC>
__device__ __forceinline__ Acc warp_tree(Acc a) {
  a = acc_combine<DT, ACC>(a, acc_xor<16, DT, ACC>(a));
  a = acc_combine<DT, ACC>(a, acc_xor<8, DT, ACC>(a));
  a = acc_combine<DT, ACC>(a, acc_xor<4, DT, ACC>(a));
  a = acc_combine<DT, ACC>(a, acc_xor<2, DT, ACC>(a));
  a = acc_combine<DT, ACC>(a, acc_xor<1, DT, ACC>(a));
  return a;
}

__device__ __forceinline__ double tree_f64(double v) {
  v = v + xor_lane_d<16>(v);
  v = v + xor_lane_d<8>(v);
  v = v + xor_lane_d<4>(v);
  v = v + xor_lane_d<2>(v);
  v = v + xor_lane_d<1>(v);
  return v;
}

// chunk partial: optional plain copy for the caller, tagged word(s) for the
// final combine (two words per chunk for TWOSUM: s then c)
template <int DT, int ACC>
__device__ __forceinline__ void store_partial(void *part, uint64_t *pw, uint32_t tag, int64_t c, const Acc &a) {
  const uint64_t hi = (uint64_t)tag << 32;
  if constexpr (DT == DT_I32) {
    if (part) ((int32_t *)part)[c] = (int32_t)a.i;
    st_dev(&pw[c], hi | a.i);
  } else if constexpr (ACC == COX_ACC_PLAIN) {
    if (part) ((float *)part)[c] = a.s;
    st_dev(&pw[c], hi | (uint32_t)f2i(a.s));
  } else {
    if (part) ((float2 *)part)[c] = make_float2(a.s, a.c);
    st_dev(&pw[2 * c], hi | (uint32_t)f2i(a.s));
    st_dev(&pw[2 * c + 1], hi | (uint32_t)f2i(a.c));
  }
}

// a tagged word that did not yet carry `tag` when first read: wait for it
// (bounded; running out sets HDR_ERR)
__device__ __noinline__ uint64_t wait_word(const uint64_t *p, uint32_t tag, uint32_t *hdr) {
  uint64_t s = ld_dev(p);
  uint32_t spins = 0;
  while ((uint32_t)(s >> 32) != tag) {
    if (++spins >= MAX_SPIN) {
      st_dev32(&hdr[HDR_ERR], tag);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
    s = ld_dev(p);
  }
  return s;
}

// value bits of FB tagged words p[i0 + b*stride] (b < FB, index < lim):
// all loads are issued first, then any word not yet carrying the tag is
// waited for; out-of-range entries get `pad`
template <int FB>
__device__ __forceinline__ void take_words(const uint64_t *p, int64_t i0, int64_t stride, int64_t lim,
                                           uint32_t tag, uint32_t *hdr, uint32_t pad, uint32_t (&out)[FB]) {
  uint64_t w[FB];
#pragma unroll
  for (int b = 0; b < FB; b++) {
    const int64_t i = i0 + (int64_t)b * stride;
    w[b] = i < lim ? ld_dev(&p[i]) : (((uint64_t)tag << 32) | pad);
  }
#pragma unroll
  for (int b = 0; b < FB; b++) {
    const int64_t i = i0 + (int64_t)b * stride;
    if ((uint32_t)(w[b] >> 32) != tag) w[b] = wait_word(&p[i], tag, hdr);
    out[b] = (uint32_t)w[b];
  }
}

template <int K, int DT, int OP, int ACC>
__global__ __launch_bounds__(1024) void k_reduce(const void *__restrict__ x, const void *__restrict__ y,
                                                 int64_t n, int64_t nch, void *__restrict__ part,
                                                 void *__restrict__ total, uint32_t *__restrict__ hdr) {
  constexpr int ESZ = ElemT<DT>::size;
  constexpr int V = K < 16 / ESZ ? K : 16 / ESZ;
  constexpr int R = K / V;
  constexpr uint32_t XPAD = DT == DT_I32 ? 0u : 0x80000000u;  // -0.0f
  constexpr uint32_t YPAD = 0u;                                // +0.0f
  __shared__ Acc slot[32];
  __shared__ double fin[256];
  __shared__ uint32_t s_last, s_epoch;

  const int W = blockDim.x >> 5;
  uint64_t *pw = (uint64_t *)(hdr + HDR_WORDS);
  if (threadIdx.x == 0) s_epoch = ld_dev32(&hdr[HDR_EPOCH]);
  __syncthreads();
  const uint32_t epoch = s_epoch;
  const uint32_t tag = tag_of_epoch(epoch);
  const int w = threadIdx.x >> 5, l = threadIdx.x & 31;
  const int64_t S = (int64_t)blockDim.x * K;

  // Full chunks c = blockIdx.x + i * gridDim.x run double-buffered: the
  // next chunk's vectors are requested before the current chunk is
  // reduced, so loads stay in flight across the block's barriers.  Past the
  // block's last full chunk the request is kept (loads stay unconditional)
  // but every lane reads the array's first vector: one line, not a chunk.
  // The partial last chunk (if any) is reduced afterwards with element-wise
  // bounds.
  const int64_t nfull = n / S;
  auto load_full = [&](int64_t c, uint32_t (&xr)[R][V], uint32_t (&yr)[R][V]) {
    const bool dummy = c >= nfull;
    // one base index and one row stride per lane (not a select per load)
    const int64_t b0 = dummy ? 0 : c * S + (int64_t)w * 32 * K + (int64_t)l * V;
    const int rs = dummy ? 0 : 32 * V;
#pragma unroll
    for (int i = 0; i < R; i++) {
      load_vec<ESZ, V>(x, b0 + (int64_t)i * rs, xr[i]);
      if constexpr (OP == OP_DOT) load_vec<ESZ, V>(y, b0 + (int64_t)i * rs, yr[i]);
    }
  };
  auto reduce_chunk = [&](int64_t c, const uint32_t (&xr)[R][V], const uint32_t (&yr)[R][V]) {
    Acc a = acc_identity<DT, ACC>();
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
      for (int v = 0; v < V; v++) acc_step<DT, OP, ACC>(a, xr[i][v], OP == OP_DOT ? yr[i][v] : 0u);
    a = warp_tree<DT, ACC>(a);
    if (l == 0) slot[w] = a;
    __syncthreads();
    if (w == 0) {
      Acc b = l < W ? slot[l] : acc_identity<DT, ACC>();
      b = warp_tree<DT, ACC>(b);
      if (l == 0) store_partial<DT, ACC>(part, pw, tag, c, b);
    }
    __syncthreads();
  };
  if (nfull > 0) {
    uint32_t xa[R][V], ya[R][V], xb[R][V], yb[R][V];
    int64_t c = blockIdx.x;
    load_full(c, xa, ya);
    while (c < nfull) {
      int64_t cn = c + gridDim.x;
      load_full(cn, xb, yb);
      reduce_chunk(c, xa, ya);
      c = cn;
      if (c >= nfull) break;
      cn = c + gridDim.x;
      load_full(cn, xa, ya);
      reduce_chunk(c, xb, yb);
      c = cn;
    }
  }
  if (nfull * S < n && blockIdx.x == nfull % gridDim.x) {
    uint32_t xr[R][V], yr[R][V];
    const int64_t wbase = nfull * S + (int64_t)w * 32 * K;
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
      for (int v = 0; v < V; v++) {
        const int64_t e = wbase + (int64_t)(i * 32 + l) * V + v;
        xr[i][v] = e < n ? load_one<ESZ>(x, e) : XPAD;
        yr[i][v] = (OP == OP_DOT && e < n) ? load_one<ESZ>(y, e) : YPAD;
      }
    reduce_chunk(nfull, xr, yr);
  }

  // the last block to finish combines the chunk partials
  if (threadIdx.x == 0) s_last = (add_dev32(&hdr[HDR_DONE], 1u) == gridDim.x - 1) ? 1u : 0u;
  __syncthreads();
  if (!s_last) return;

  // Loads of the partials are issued in batches of FB independent loads per
  // thread before they are added, so the fixed serial order costs one
  // memory latency per batch rather than one per chunk.
  constexpr int FB = 32;
  if constexpr (DT == DT_I32) {
    __shared__ long long isum[32];
    long long s = 0;
    for (int64_t c0 = threadIdx.x; c0 < nch; c0 += (int64_t)FB * blockDim.x) {
      uint32_t buf[FB];
      take_words<FB>(pw, c0, blockDim.x, nch, tag, hdr, 0u, buf);
#pragma unroll
      for (int b = 0; b < FB; b++) s += (long long)(int32_t)buf[b];
    }
    // block sum of int64 (order does not matter for integers)
    for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
    if (l == 0) isum[w] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long tot = 0;
      for (int j = 0; j < W; j++) tot += isum[j];
      *(long long *)total = tot;
      st_dev32(&hdr[HDR_DONE], 0u);
      st_dev32(&hdr[HDR_EPOCH], epoch + 1u);
    }
  } else {
    // FP64 final tree shaped like a 256-thread block (see cox.h); a chain
    // padded with -0.0 at its end is unchanged
    for (int j = threadIdx.x; j < 256; j += blockDim.x) {
      double s = -0.0;
      for (int64_t c0 = j; c0 < nch; c0 += (int64_t)FB * 256) {
        double buf[FB];
        if constexpr (ACC == COX_ACC_PLAIN) {
          uint32_t v[FB];
          take_words<FB>(pw, c0, 256, nch, tag, hdr, 0x80000000u, v);
#pragma unroll
          for (int b = 0; b < FB; b++) buf[b] = (double)i2f((int)v[b]);
        } else {
          // words 2c (s) and 2c + 1 (c); padding (-0.0, -0.0) adds -0.0
          uint32_t vs[FB], vc[FB];
          take_words<FB>(pw, 2 * c0, 512, 2 * nch, tag, hdr, 0x80000000u, vs);
          take_words<FB>(pw, 2 * c0 + 1, 512, 2 * nch, tag, hdr, 0x80000000u, vc);
#pragma unroll
          for (int b = 0; b < FB; b++) buf[b] = (double)i2f((int)vs[b]) + (double)i2f((int)vc[b]);
        }
#pragma unroll
        for (int b = 0; b < FB; b++) s = s + buf[b];
      }
      fin[j] = s;
    }
    __syncthreads();
    if (threadIdx.x < 32) {
      double top = -0.0;
#pragma unroll 1
      for (int vw = 0; vw < 8; vw++) {
        const double r = tree_f64(fin[32 * vw + l]);
        const double r0 = __shfl(r, 0, 32);
        if (l == vw) top = r0;
      }
      top = tree_f64(top);
      if (l == 0) {
        *(double *)total = top;
        st_dev32(&hdr[HDR_DONE], 0u);
        st_dev32(&hdr[HDR_EPOCH], epoch + 1u);
      }
    }
  }
}

// ---------------------------------------------------------------- dispatch
using reduce_fn = void (*)(const void *, const void *, int64_t, int64_t, void *, void *, uint32_t *);

template <int DT, int OP, int ACC>
static reduce_fn pick_k(int k) {
  switch (k) {
  case 1: return k_reduce<1, DT, OP, ACC>;
  case 2: return k_reduce<2, DT, OP, ACC>;
  case 4: return k_reduce<4, DT, OP, ACC>;
  case 8: return k_reduce<8, DT, OP, ACC>;
  case 16: return k_reduce<16, DT, OP, ACC>;
  case 32: return k_reduce<32, DT, OP, ACC>;
  }
  return nullptr;
}

static reduce_fn pick(int dt, int op, int acc, int k) {
  if (dt == DT_I32) return op == OP_SUM && acc == COX_ACC_PLAIN ? pick_k<DT_I32, OP_SUM, COX_ACC_PLAIN>(k) : nullptr;
  if (dt == DT_F32) {
    if (op == OP_SUM) return acc == COX_ACC_PLAIN ? pick_k<DT_F32, OP_SUM, COX_ACC_PLAIN>(k) : pick_k<DT_F32, OP_SUM, COX_ACC_TWOSUM>(k);
    return acc == COX_ACC_PLAIN ? pick_k<DT_F32, OP_DOT, COX_ACC_PLAIN>(k) : pick_k<DT_F32, OP_DOT, COX_ACC_TWOSUM>(k);
  }
  if (dt == DT_BF16) {
    if (op == OP_SUM) return acc == COX_ACC_PLAIN ? pick_k<DT_BF16, OP_SUM, COX_ACC_PLAIN>(k) : pick_k<DT_BF16, OP_SUM, COX_ACC_TWOSUM>(k);
    return acc == COX_ACC_PLAIN ? pick_k<DT_BF16, OP_DOT, COX_ACC_PLAIN>(k) : pick_k<DT_BF16, OP_DOT, COX_ACC_TWOSUM>(k);
  }
  return nullptr;
}

// default persistent grid: about 512 threads per compute unit (measured
// best for streaming reads on MI355X: fewer concurrent streams keep DRAM
// pages open)
static int reduce_blocks_per_cu(int block) { return block >= 512 ? 1 : 512 / block; }

static cox_status reduce_any(const void *x, const void *y, cox_dtype dtype, int op, int64_t n, cox_acc acc,
                             const cox_cfg *cfg, void *chunk_partials, void *total, void *ws,
                             size_t ws_bytes, void *stream) {
  if (n < 0 || !total) return COX_ERR_INVALID;
  if (acc != COX_ACC_PLAIN && acc != COX_ACC_TWOSUM) return COX_ERR_DTYPE;
  if (dtype != COX_I32 && dtype != COX_F32 && dtype != COX_BF16) return COX_ERR_DTYPE;
  if (dtype == COX_I32 && (acc != COX_ACC_PLAIN || op != OP_SUM)) return COX_ERR_DTYPE;
  Sigma sg;
  cox_status st = resolve_cfg(op == OP_SUM ? COX_OP_REDUCE : COX_OP_DOT, dtype, cfg, &sg);
  if (st != COX_OK) return st;
  if (n > 0 && (!x || (op == OP_DOT && !y))) return COX_ERR_INVALID;
  if (n > 0 && (!aligned16(x) || (op == OP_DOT && !aligned16(y)))) return COX_ERR_ALIGN;
  const size_t need = cox_workspace_bytes(op == OP_SUM ? COX_OP_REDUCE : COX_OP_DOT, dtype, n, 0, cfg);
  if (!ws || ws_bytes < need) return COX_ERR_WORKSPACE;
  reduce_fn fn = pick(dtype, op, acc, sg.k);
  if (!fn) return COX_ERR_UNSUPPORTED;
  const int block = 32 * sg.W;
  const int64_t S = (int64_t)block * sg.k;
  const int64_t nch = (n + S - 1) / S;
  void *part = chunk_partials;  // optional plain copy; tagged words live in the workspace
  const int grid = persistent_grid((const void *)fn, block, nch > 0 ? nch : 1, sg.G, 0, reduce_blocks_per_cu(block));
  hipLaunchKernelGGL(fn, dim3(grid), dim3(block), 0, (hipStream_t)stream, x, y, n, nch, part, total,
                     (uint32_t *)ws);
  return launch_status();
}

}  // namespace cox

using namespace cox;

extern "C" {

cox_status cox_warp_reduce_blocks_i32(const int32_t *x, int64_t n, int32_t *block_sums,
                                      int32_t *warp_pos_count, void *stream) {
  if (n < 0) return COX_ERR_INVALID;
  if (n == 0) return COX_OK;
  if (!x || !block_sums || !warp_pos_count) return COX_ERR_INVALID;
  const int64_t nb = (n + 255) / 256;
  if (nb > 0x7fffffff) return COX_ERR_INVALID;
  hipLaunchKernelGGL(k_reduce_blocks_i32, dim3((unsigned)nb), dim3(256), 0, (hipStream_t)stream, x, n,
                     block_sums, warp_pos_count);
  return launch_status();
}

cox_status cox_warp_reduce(const void *x, cox_dtype dtype, int64_t n, cox_acc acc, const cox_cfg *cfg,
                           void *chunk_partials, void *total, void *ws, size_t ws_bytes, void *stream) {
  return reduce_any(x, nullptr, dtype, OP_SUM, n, acc, cfg, chunk_partials, total, ws, ws_bytes, stream);
}

cox_status cox_warp_dot(const void *a, const void *b, cox_dtype dtype, int64_t n, cox_acc acc,
                        const cox_cfg *cfg, void *chunk_partials, double *total, void *ws, size_t ws_bytes,
                        void *stream) {
  if (dtype != COX_F32 && dtype != COX_BF16) return COX_ERR_DTYPE;
  return reduce_any(a, b, dtype, OP_DOT, n, acc, cfg, chunk_partials, total, ws, ws_bytes, stream);
}

}  // extern "C"
