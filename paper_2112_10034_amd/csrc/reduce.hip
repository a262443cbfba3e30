// Warp-shuffle reductions.
//
// k_reduce_blocks_i32: 256-thread blocks of 8 logical warps, one element
// per thread; shfl_down tree per warp, ballot(x > 0) per warp, shared-memory
// combine of the 8 warp values by warp 0 (the SDK reduction pattern that
// COX's Code 1 simplifies, Sec. 2.3).
//
// k_reduce: chunked sum / dot under the fixed schedule sigma = (k, W)
// (documented in cox.h); persistent blocks walk chunks c = b, b + G, ...;
// every chunk partial is stored, and the last block to finish (device-scope
// counter) runs the FP64 (or int64) final combine.
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
    uint4 q = *(const uint4 *)p;
    w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
  } else if constexpr (BYTES == 8) {
    uint2 q = *(const uint2 *)p;
    w[0] = q.x; w[1] = q.y;
  } else if constexpr (BYTES == 4) {
    w[0] = *(const uint32_t *)p;
  } else {
    w[0] = *(const uint16_t *)p;
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
  if constexpr (ESZ == 4) return ((const uint32_t *)base)[idx];
  else return (uint32_t)((const uint16_t *)base)[idx] << 16;
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

template <int DT, int ACC>
__device__ __forceinline__ void store_partial(void *part, int64_t c, const Acc &a) {
  if constexpr (DT == DT_I32) ((int32_t *)part)[c] = (int32_t)a.i;
  else if constexpr (ACC == COX_ACC_PLAIN) ((float *)part)[c] = a.s;
  else ((float2 *)part)[c] = make_float2(a.s, a.c);
}

template <int DT, int ACC>
__device__ __forceinline__ double partial_f64(const void *part, int64_t c) {
  if constexpr (ACC == COX_ACC_PLAIN) {
    return (double)((const float *)part)[c];
  } else {
    const float2 q = ((const float2 *)part)[c];
    return (double)q.x + (double)q.y;
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
  __shared__ uint32_t s_last;

  const int W = blockDim.x >> 5;
  const int w = threadIdx.x >> 5, l = threadIdx.x & 31;
  const int64_t S = (int64_t)blockDim.x * K;

  for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const int64_t wbase = c * S + (int64_t)w * 32 * K;
    uint32_t xr[R][V], yr[R][V];
    if ((c + 1) * S <= n) {
#pragma unroll
      for (int i = 0; i < R; i++) {
        load_vec<ESZ, V>(x, wbase + (int64_t)(i * 32 + l) * V, xr[i]);
        if constexpr (OP == OP_DOT) load_vec<ESZ, V>(y, wbase + (int64_t)(i * 32 + l) * V, yr[i]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < R; i++)
#pragma unroll
        for (int v = 0; v < V; v++) {
          const int64_t e = wbase + (int64_t)(i * 32 + l) * V + v;
          xr[i][v] = e < n ? load_one<ESZ>(x, e) : XPAD;
          if constexpr (OP == OP_DOT) yr[i][v] = e < n ? load_one<ESZ>(y, e) : YPAD;
        }
    }
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
      if (l == 0) store_partial<DT, ACC>(part, c, b);
    }
    __syncthreads();
  }

  // last block to finish combines the chunk partials
  __threadfence();
  if (threadIdx.x == 0) s_last = (atomicAdd(&hdr[HDR_DONE], 1u) == gridDim.x - 1) ? 1u : 0u;
  __syncthreads();
  if (!s_last) return;
  __threadfence();

  if constexpr (DT == DT_I32) {
    __shared__ long long isum[32];
    long long s = 0;
    for (int64_t c = threadIdx.x; c < nch; c += blockDim.x) s += (long long)((const int32_t *)part)[c];
    // block sum of int64 (order does not matter for integers)
    for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
    if (l == 0) isum[w] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long tot = 0;
      for (int j = 0; j < W; j++) tot += isum[j];
      *(long long *)total = tot;
      hdr[HDR_DONE] = 0u;
    }
  } else {
    // FP64 final tree shaped like a 256-thread block (see cox.h)
    for (int j = threadIdx.x; j < 256; j += blockDim.x) {
      double s = -0.0;
      for (int64_t c = j; c < nch; c += 256) s = s + partial_f64<DT, ACC>(part, c);
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
        hdr[HDR_DONE] = 0u;
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
  void *part = chunk_partials ? chunk_partials : (void *)((char *)ws + WS_HEADER);
  const int grid = persistent_grid((const void *)fn, block, nch > 0 ? nch : 1, sg.G);
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
