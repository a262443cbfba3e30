// thread_block_tile<T> reductions and masked (divergent) warp operations.
//
// Both kernels keep CUDA's one-element-per-lane mapping: element e sits in
// logical lane e & 31 of logical warp e >> 5.  A block handles R rows of 256
// consecutive elements per round (coalesced streaming 4-byte loads, R loads
// in flight per thread), and the whole block runs every round so that the
// fixed-pattern exchanges always see full warps.  The default grid is four
// 256-thread blocks per compute unit.
#include "cox_internal.hpp"

namespace cox {

template <int T>
__device__ __forceinline__ uint32_t tile_tree(uint32_t v) {
  // tile.shfl_down(v, o) for o = T/2 .. 1; the tile's first lane only reads
  // lanes of its own tile, where the xor partner l ^ o equals l + o
  if constexpr (T >= 32) v += (uint32_t)xor_lane<16>((int)v);
  if constexpr (T >= 16) v += (uint32_t)xor_lane<8>((int)v);
  if constexpr (T >= 8) v += (uint32_t)xor_lane<4>((int)v);
  if constexpr (T >= 4) v += (uint32_t)xor_lane<2>((int)v);
  if constexpr (T >= 2) v += (uint32_t)xor_lane<1>((int)v);
  return v;
}

template <int T, int R>
__global__ __launch_bounds__(256) void k_tile_reduce(const int32_t *__restrict__ x, int64_t n,
                                                     int32_t *__restrict__ out) {
  const int t = threadIdx.x, l = t & 31;
  const int64_t per_block = 256 * R;
  const int64_t stride = (int64_t)gridDim.x * per_block;
  const int64_t rounds = (n + stride - 1) / stride;
  for (int64_t it = 0; it < rounds; it++) {
    const int64_t base = it * stride + (int64_t)blockIdx.x * per_block;
    uint32_t v[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t e = base + r * 256 + t;
      v[r] = e < n ? ld_stream1(x + e) : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t e = base + r * 256 + t;
      const uint32_t s = tile_tree<T>(v[r]);
      if ((l & (T - 1)) == 0 && e < n) out[e / T] = (int32_t)s;
    }
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_warp_masked(const int32_t *__restrict__ x, int64_t n, int D,
                                                     int32_t *__restrict__ out, uint32_t *__restrict__ rec) {
  const int t = threadIdx.x, l = t & 31;
  const int64_t per_block = 256 * R;
  const int64_t stride = (int64_t)gridDim.x * per_block;
  const int64_t rounds = (n + stride - 1) / stride;
  for (int64_t it = 0; it < rounds; it++) {
    const int64_t base = it * stride + (int64_t)blockIdx.x * per_block;
    int32_t xs[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t e = base + r * 256 + t;
      xs[r] = e < n ? (int32_t)ld_stream1(x + e) : 0;
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t e = base + r * 256 + t;
      if (e >= n) continue;  // whole logical warps (n % 32 == 0)
      const int32_t xv = xs[r];
      const int64_t g = e >> 5;
      const bool p = ((uint32_t)xv & 1023u) < (uint32_t)D;
      const uint32_t m = ballot(p);
      if (p) {
        // divergent region: exactly the lanes of m execute
        const uint32_t b = ballot_sync(m, xv > 0);
        const bool A = any_sync(m, ((xv >> 10) & 31) == 0);
        const bool L = all_sync(m, ((xv >> 15) & 31) != 0);
        const uint32_t above = l == 31 ? 0u : (m & (FULL << (l + 1)));
        const int src = above ? __builtin_ctz(above) : __builtin_ctz(m);
        const int ld = __builtin_ctz(m);
        const int32_t s = shfl(xv, src);
        const int32_t bc = shfl(xv, ld);
        out[e] = s;
        if (l == ld)
          *(uint4 *)(rec + 4 * g) = make_uint4(m, b, (uint32_t)A | ((uint32_t)L << 1), (uint32_t)bc);
      } else {
        out[e] = INT32_MIN;
      }
      if (m == 0u && l == 0) *(uint4 *)(rec + 4 * g) = make_uint4(0u, 0u, 0u, 0u);
    }
  }
}

using tred_fn = void (*)(const int32_t *, int64_t, int32_t *);
static tred_fn pick_tile(int T) {
  switch (T) {
  case 2: return k_tile_reduce<2, 8>;
  case 4: return k_tile_reduce<4, 8>;
  case 8: return k_tile_reduce<8, 8>;
  case 16: return k_tile_reduce<16, 8>;
  case 32: return k_tile_reduce<32, 8>;
  }
  return nullptr;
}

}  // namespace cox

using namespace cox;

extern "C" {

cox_status cox_tile_reduce(const int32_t *x, int64_t n, int tile, int32_t *out, void *stream) {
  if (n < 0) return COX_ERR_INVALID;
  tred_fn fn = pick_tile(tile);
  if (!fn) return COX_ERR_INVALID;
  if (n == 0) return COX_OK;
  if (!x || !out) return COX_ERR_INVALID;
  const int grid = persistent_grid((const void *)fn, 256, (n + 256 * 8 - 1) / (256 * 8), 0, 0, 4);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, (hipStream_t)stream, x, n, out);
  return launch_status();
}

cox_status cox_warp_masked(const int32_t *x, int64_t n, int density, int32_t *out, uint32_t *rec,
                           void *stream) {
  if (n < 0 || n % 32 || density < 0 || density > 1024) return COX_ERR_INVALID;
  if (n == 0) return COX_OK;
  if (!x || !out || !rec) return COX_ERR_INVALID;
  if (!aligned16(rec)) return COX_ERR_ALIGN;
  auto fn = k_warp_masked<8>;
  const int grid = persistent_grid((const void *)fn, 256, (n + 256 * 8 - 1) / (256 * 8), 0, 0, 4);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, (hipStream_t)stream, x, n, density, out, rec);
  return launch_status();
}

}  // extern "C"
