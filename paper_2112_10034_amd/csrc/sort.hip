// Bitonic tile sort of groups of T = 32 .. 1024 keys.
//
// A group of T consecutive keys lives in LG = T/K consecutive lanes, K keys
// per lane (lane g of the group holds keys gK..gK+K-1, loaded as one
// vector), so key index i = g*K + r.  The network is the bitonic sorter in
// its all-ascending form: for each merge size k2 = 2, 4, .., T a first
// layer compares i with i ^ (k2 - 1) (the mirror inside the k2-block), then
// half-cleaner layers compare i with i ^ j for j = k2/4 .. 1; the smaller
// index always keeps the minimum.  A layer whose partner differs only in
// the low log2(K) bits is a compare-exchange between two registers of one
// lane; every other layer exchanges with partner lane g ^ (mask / K),
// register r ^ (mask mod K), then keeps min or max:
//   - partner in the same 32-lane half: a __shfl_xor_sync (DPP or
//     ds_swizzle; with K = 4 and T = 32 all are DPP quad_perm /
//     row_half_mirror exchanges);
//   - partner in the other half of the wave (a group of 64 lanes, the
//     full-wave sort): the in-half exchange, then v_permlane32_swap;
//   - partner in another wave (groups wider than a wave, the multi-warp
//     sort): through shared memory, between two block barriers.
// The layers inside one lane's K registers (every merge size up to K) are
// replaced by Batcher's odd-even merge sort of the K registers, which needs
// fewer comparators.  The sorted result is the unique ascending order, so
// any such network gives the same output as a one-key-per-lane network.
#include "cox_internal.hpp"

namespace cox {

// value of lane t ^ LM of the wave (LM < 64)
template <int LM>
__device__ __forceinline__ uint32_t xor_lane_wave(uint32_t v) {
  if constexpr (LM < 32) {
    return (uint32_t)xor_lane<LM>((int)v);
  } else {
    const uint32_t u = LM == 32 ? v : (uint32_t)xor_lane<LM - 32>((int)v);
    // swaps the upper half of the first operand with the lower half of the
    // second: every lane receives the other half's value
    const auto pr = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return lhalf() ? (uint32_t)pr[0] : (uint32_t)pr[1];
  }
}

template <int K, int PM, int LB, int U>
__device__ __forceinline__ void cx_layer(uint32_t (&key)[U][K], int g, uint32_t *lds) {
  constexpr int RM = PM & (K - 1);  // register part of the partner mask
  constexpr int LM = PM / K;        // lane part
  if constexpr (LM == 0) {
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int r = 0; r < K; r++) {
        const int r2 = r ^ RM;
        if (r < r2) {
          const uint32_t a = key[u][r], b = key[u][r2];
          key[u][r] = a < b ? a : b;
          key[u][r2] = a < b ? b : a;
        }
      }
  } else {
    // the lower lane of a pair keeps min = med3(a, b, 0), the upper one
    // max = med3(a, b, ~0): one exchange and one median per key
    const uint32_t sel = (g & (LB / K)) ? 0xffffffffu : 0u;
    uint32_t other[U][K];
    if constexpr (LM < 64) {
#pragma unroll
      for (int u = 0; u < U; u++)
#pragma unroll
        for (int r = 0; r < K; r++) other[u][r] = xor_lane_wave<LM>(key[u][r ^ RM]);
    } else {
      const int t = threadIdx.x;
#pragma unroll
      for (int u = 0; u < U; u++)
#pragma unroll
        for (int r = 0; r < K; r++) lds[(u * 256 + t) * K + r] = key[u][r];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < U; u++)
#pragma unroll
        for (int r = 0; r < K; r++) other[u][r] = lds[u * 256 * K + ((t * K + r) ^ PM)];
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int r = 0; r < K; r++) key[u][r] = med3u(key[u][r], other[u][r], sel);
  }
}

template <int K, int J, int U>
__device__ __forceinline__ void half_cleaners(uint32_t (&key)[U][K], int g, uint32_t *lds) {
  if constexpr (J >= 1) {
    cx_layer<K, J, J, U>(key, g, lds);
    half_cleaners<K, J / 2, U>(key, g, lds);
  }
}

template <int K, int K2, int T, int U>
__device__ __forceinline__ void merge_stages(uint32_t (&key)[U][K], int g, uint32_t *lds) {
  if constexpr (K2 <= T) {
    cx_layer<K, K2 - 1, K2 / 2, U>(key, g, lds);  // mirror layer
    half_cleaners<K, K2 / 4, U>(key, g, lds);
    merge_stages<K, K2 * 2, T, U>(key, g, lds);
  }
}

// compare-exchange of registers a < b of every row (a keeps the minimum)
template <int K, int U>
__device__ __forceinline__ void cx_reg(uint32_t (&key)[U][K], int a, int b) {
#pragma unroll
  for (int u = 0; u < U; u++) {
    const uint32_t x = key[u][a], y = key[u][b];
    key[u][a] = x < y ? x : y;
    key[u][b] = x < y ? y : x;
  }
}

// Batcher's odd-even merge sort of the K registers of each row: 1, 5, 19
// and 63 comparators for K = 2, 4, 8, 16, where the bitonic sorter takes
// 1, 6, 24 and 80.  Any sorting network gives the same sorted block, and
// the bitonic merges of the group continue from sorted blocks of K keys.
template <int K, int U, int LO, int N, int R>
__device__ __forceinline__ void oem_merge(uint32_t (&key)[U][K]) {
  constexpr int M = 2 * R;
  if constexpr (M < N) {
    oem_merge<K, U, LO, N, M>(key);
    oem_merge<K, U, LO + R, N, M>(key);
#pragma unroll
    for (int i = LO + R; i < LO + N - R; i += M) cx_reg<K, U>(key, i, i + R);
  } else {
    cx_reg<K, U>(key, LO, LO + R);
  }
}

template <int K, int U, int LO, int N>
__device__ __forceinline__ void oem_sort(uint32_t (&key)[U][K]) {
  if constexpr (N > 1) {
    oem_sort<K, U, LO, N / 2>(key);
    oem_sort<K, U, LO + N / 2, N / 2>(key);
    oem_merge<K, U, LO, N, 1>(key);
  }
}

// the group's network: the keys of each lane sorted in registers, then
// the bitonic merges of blocks of 2K, 4K, .., T keys
template <int K, int T, int U>
__device__ __forceinline__ void sort_group(uint32_t (&key)[U][K], int g, uint32_t *lds) {
  oem_sort<K, U, 0, K>(key);
  merge_stages<K, 2 * K, T, U>(key, g, lds);
}

template <int K>
__device__ __forceinline__ void load_keys(const uint32_t *__restrict__ p, uint32_t (&key)[K]) {
  if constexpr (K % 4 == 0) {
#pragma unroll
    for (int q = 0; q < K / 4; q++) {
      const u32x4 v = ld_stream4(p + 4 * q);
      key[4 * q] = v.x; key[4 * q + 1] = v.y; key[4 * q + 2] = v.z; key[4 * q + 3] = v.w;
    }
  } else if constexpr (K == 2) {
    const u32x2 v = ld_stream2(p);
    key[0] = v.x; key[1] = v.y;
  } else {
    key[0] = ld_stream1(p);
  }
}

template <int K>
__device__ __forceinline__ void store_keys(uint32_t *__restrict__ p, const uint32_t (&key)[K]) {
  if constexpr (K % 4 == 0) {
#pragma unroll
    for (int q = 0; q < K / 4; q++)
      st_stream4(p + 4 * q, key[4 * q], key[4 * q + 1], key[4 * q + 2], key[4 * q + 3]);
  } else if constexpr (K == 2) {
    st_stream2(p, key[0], key[1]);
  } else {
    st_stream1(p, key[0]);
  }
}

// keys of one round: U rows of 256 lane vectors starting at lane vector
// vbase (row u = vectors vbase + 256u); a round that runs past n loads
// element by element and pads with the maximum key
template <int K, int U>
__device__ __forceinline__ void load_round(const uint32_t *keys, int64_t vbase, int64_t n, bool full,
                                           uint32_t (&key)[U][K]) {
  if (full) {
#pragma unroll
    for (int u = 0; u < U; u++) load_keys<K>(keys + (vbase + 256 * u) * K, key[u]);
  } else {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t e0 = (vbase + 256 * u) * K;
#pragma unroll
      for (int r = 0; r < K; r++) key[u][r] = e0 + r < n ? keys[e0 + r] : 0xffffffffu;
    }
  }
}

template <int K, int U>
__device__ __forceinline__ void store_round(uint32_t *out, int64_t vbase, int64_t n, bool full,
                                            const uint32_t (&key)[U][K]) {
  if (full) {
#pragma unroll
    for (int u = 0; u < U; u++) store_keys<K>(out + (vbase + 256 * u) * K, key[u]);
  } else {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t e0 = (vbase + 256 * u) * K;
#pragma unroll
      for (int r = 0; r < K; r++)
        if (e0 + r < n) out[e0 + r] = key[u][r];
    }
  }
}

// Grid-stride rounds; in a round a block handles U rows of 256 lane
// vectors (row u = vectors [base + 256u, base + 256u + 256)), and each
// thread first requests its U vectors, then sorts and stores them, so U
// independent loads per lane are in flight.  (Requesting the next round's
// keys before sorting the current ones, in a second register set, measured
// slower: 0.37-0.38 against 0.36 ms at 2^28.)  Every group is held by LG
// aligned lanes of one block row (T <= 256 K).  keys and out may be the
// same buffer (each lane writes back only the positions it read, after its
// whole group has been sorted).
template <int K, int T>
__global__ __launch_bounds__(256) void k_tile_sort(const uint32_t *keys, uint32_t *out, int64_t n) {
  constexpr int LG = T / K;
  static_assert(LG >= 1 && LG <= 256, "a group fits in one block row");
  constexpr int U = K >= 16 ? 1 : 16 / K > 4 ? 4 : 16 / K;
  uint32_t *lds = nullptr;
  if constexpr (LG > 64) {
    __shared__ uint32_t s_x[U * 256 * K];  // the exchanges between waves
    lds = s_x;
  }
  const int g = (int)(threadIdx.x % LG);
  const int64_t nvec = (n + K - 1) / K;
  const int64_t per_round = (int64_t)gridDim.x * 256 * U;
  // the whole block iterates together so that partial groups see full warps
  const int64_t rounds = (nvec + per_round - 1) / per_round;
  for (int64_t it = 0; it < rounds; it++) {
    const int64_t vbase = it * per_round + (int64_t)blockIdx.x * 256 * U + threadIdx.x;
    const bool full = (vbase - threadIdx.x + 256 * U) * K <= n;
    uint32_t key[U][K];
    load_round<K, U>(keys, vbase, n, full, key);
    sort_group<K, T, U>(key, g, lds);
    store_round<K, U>(out, vbase, n, full, key);
  }
}

// Key-value form: the network runs on 64-bit composites (key << 32 |
// position in the group), so equal keys keep their original order (a
// stable sort, which makes the result unique) and every comparison is one
// 64-bit compare.  After the network each output takes its value from the
// group's original values at its position (the group's 128 bytes, loaded
// once).
template <int K, int PM, int LB>
__device__ __forceinline__ void cx_layer_kv(uint64_t (&c)[K], int g) {
  constexpr int RM = PM & (K - 1);
  constexpr int LM = PM / K;
  if constexpr (LM == 0) {
#pragma unroll
    for (int r = 0; r < K; r++) {
      const int r2 = r ^ RM;
      if (r < r2) {
        const uint64_t a = c[r], b = c[r2];
        c[r] = a < b ? a : b;
        c[r2] = a < b ? b : a;
      }
    }
  } else {
    uint64_t other[K];
#pragma unroll
    for (int r = 0; r < K; r++) {
      const uint64_t v = c[r ^ RM];
      const uint32_t lo = (uint32_t)xor_lane<LM>((int)(uint32_t)v);
      const uint32_t hi = (uint32_t)xor_lane<LM>((int)(uint32_t)(v >> 32));
      other[r] = ((uint64_t)hi << 32) | lo;
    }
    const bool upper = (g & (LB / K)) != 0;
#pragma unroll
    for (int r = 0; r < K; r++) {
      const bool less = other[r] < c[r];
      c[r] = (less != upper) ? other[r] : c[r];
    }
  }
}

template <int K, int K2, int J>
__device__ __forceinline__ void half_cleaners_kv(uint64_t (&c)[K], int g) {
  if constexpr (J >= 1) {
    cx_layer_kv<K, J, J>(c, g);
    half_cleaners_kv<K, K2, J / 2>(c, g);
  }
}

template <int K, int K2>
__device__ __forceinline__ void merge_stages_kv(uint64_t (&c)[K], int g) {
  if constexpr (K2 <= 32) {
    cx_layer_kv<K, K2 - 1, K2 / 2>(c, g);
    half_cleaners_kv<K, K2, K2 / 4>(c, g);
    merge_stages_kv<K, K2 * 2>(c, g);
  }
}

// same rounds and row layout as k_tile_sort; keys / out_keys may be the
// same buffer, vals / out_vals may not
template <int K>
__global__ __launch_bounds__(256) void k_tile_sort_kv(const uint32_t *keys, const uint32_t *__restrict__ vals,
                                                      uint32_t *out_keys, uint32_t *__restrict__ out_vals,
                                                      int64_t n) {
  constexpr int LG = 32 / K;
  constexpr int U = K >= 8 ? 1 : 8 / K > 4 ? 4 : 8 / K;
  const int g = (int)(threadIdx.x % LG);
  const int64_t nvec = (n + K - 1) / K;
  const int64_t per_round = (int64_t)gridDim.x * 256 * U;
  const int64_t rounds = (nvec + per_round - 1) / per_round;
  for (int64_t it = 0; it < rounds; it++) {
    const int64_t vbase = it * per_round + (int64_t)blockIdx.x * 256 * U + threadIdx.x;
    const bool full = (vbase - threadIdx.x + 256 * U) * K <= n;
    uint64_t c[U][K];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t e0 = (vbase + 256 * u) * K;
      uint32_t key[K];
      if (full) {
        load_keys<K>(keys + e0, key);
      } else {
#pragma unroll
        for (int r = 0; r < K; r++) key[r] = e0 + r < n ? keys[e0 + r] : 0xffffffffu;
      }
#pragma unroll
      for (int r = 0; r < K; r++) c[u][r] = ((uint64_t)key[r] << 32) | (uint32_t)(g * K + r);
    }
#pragma unroll
    for (int u = 0; u < U; u++) merge_stages_kv<K, 2>(c[u], g);
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t e0 = (vbase + 256 * u) * K;
      const int64_t gb = e0 & ~(int64_t)31;
      uint32_t key[K], val[K];
#pragma unroll
      for (int r = 0; r < K; r++) {
        key[r] = (uint32_t)(c[u][r] >> 32);
        const bool ok = full || e0 + r < n;
        val[r] = ok ? vals[gb + ((uint32_t)c[u][r] & 31u)] : 0u;
      }
      if (full) {
        store_keys<K>(out_keys + e0, key);
        store_keys<K>(out_vals + e0, val);
      } else {
#pragma unroll
        for (int r = 0; r < K; r++)
          if (e0 + r < n) {
            out_keys[e0 + r] = key[r];
            out_vals[e0 + r] = val[r];
          }
      }
    }
  }
}

using sort_fn = void (*)(const uint32_t *, uint32_t *, int64_t);
static sort_fn pick_sort(int k, int tile) {
  if (tile == 32) {
    switch (k) {
    case 1: return k_tile_sort<1, 32>;
    case 2: return k_tile_sort<2, 32>;
    case 4: return k_tile_sort<4, 32>;
    case 8: return k_tile_sort<8, 32>;
    case 16: return k_tile_sort<16, 32>;
    }
  } else if (k == 1) {
    switch (tile) {
    case 64: return k_tile_sort<1, 64>;
    case 128: return k_tile_sort<1, 128>;
    case 256: return k_tile_sort<1, 256>;
    }
  } else if (k == 4) {
    switch (tile) {
    case 64: return k_tile_sort<4, 64>;
    case 128: return k_tile_sort<4, 128>;
    case 256: return k_tile_sort<4, 256>;
    case 512: return k_tile_sort<4, 512>;
    case 1024: return k_tile_sort<4, 1024>;
    }
  }
  return nullptr;
}

using sort_kv_fn = void (*)(const uint32_t *, const uint32_t *, uint32_t *, uint32_t *, int64_t);
static sort_kv_fn pick_sort_kv(int k) {
  switch (k) {
  case 1: return k_tile_sort_kv<1>;
  case 2: return k_tile_sort_kv<2>;
  case 4: return k_tile_sort_kv<4>;
  case 8: return k_tile_sort_kv<8>;
  }
  return nullptr;
}

}  // namespace cox

using namespace cox;

extern "C" cox_status cox_tile_sort(const uint32_t *keys, uint32_t *out, int64_t n, int tile,
                                    const cox_cfg *cfg, void *stream) {
  if (n < 0 || tile < 32 || tile > 1024 || (tile & (tile - 1))) return COX_ERR_INVALID;
  const int k = (cfg && cfg->items_per_lane) ? cfg->items_per_lane : 4;
  if (cfg && cfg->grid_blocks < 0) return COX_ERR_INVALID;
  sort_fn fn = pick_sort(k, tile);
  if (!fn) return k > 0 && k <= 32 && (k & (k - 1)) == 0 ? COX_ERR_UNSUPPORTED : COX_ERR_INVALID;
  if (n == 0) return COX_OK;
  if (!keys || !out) return COX_ERR_INVALID;
  if (!aligned16(keys) || !aligned16(out)) return COX_ERR_ALIGN;
  const int64_t nvec = (n + k - 1) / k;
  const int U = k >= 16 ? 1 : 16 / k > 4 ? 4 : 16 / k;
  // default blocks per compute unit (measured at 2^28 keys): two for
  // 32-key groups and for 64-key groups with several keys per lane; six
  // for 64 keys over a full wave (0.420 ms against 0.434 with eight); eight
  // for wider groups, whose longer networks need more waves in flight
  // (1024-key groups: 0.69 ms against 0.95 ms with two)
  const int per_cu = tile == 32 || (k >= 2 && tile <= 64) ? 2 : tile == 64 ? 6 : 8;
  const int grid = persistent_grid((const void *)fn, 256, (nvec + 256 * U - 1) / (256 * U),
                                   cfg ? cfg->grid_blocks : 0, 0, per_cu);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, (hipStream_t)stream, keys, out, n);
  return launch_status();
}

extern "C" cox_status cox_tile_sort_kv(const uint32_t *keys, const uint32_t *vals, uint32_t *out_keys,
                                       uint32_t *out_vals, int64_t n, int tile, const cox_cfg *cfg, void *stream) {
  if (n < 0 || tile != 32) return COX_ERR_INVALID;
  const int k = (cfg && cfg->items_per_lane) ? cfg->items_per_lane : 4;
  if (cfg && cfg->grid_blocks < 0) return COX_ERR_INVALID;
  sort_kv_fn fn = pick_sort_kv(k);
  if (!fn) return k > 0 && k <= 32 && (k & (k - 1)) == 0 ? COX_ERR_UNSUPPORTED : COX_ERR_INVALID;
  if (n == 0) return COX_OK;
  if (!keys || !vals || !out_keys || !out_vals) return COX_ERR_INVALID;
  if (!aligned16(keys) || !aligned16(out_keys) || !aligned16(out_vals)) return COX_ERR_ALIGN;
  if (out_vals == vals) return COX_ERR_INVALID;
  const int64_t nvec = (n + k - 1) / k;
  const int U = k >= 8 ? 1 : 8 / k > 4 ? 4 : 8 / k;
  // default: four 256-thread blocks per compute unit (measured at 2^28
  // pairs: 0.82 ms against 1.21 ms with two)
  const int grid = persistent_grid((const void *)fn, 256, (nvec + 256 * U - 1) / (256 * U),
                                   cfg ? cfg->grid_blocks : 0, 0, 4);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, (hipStream_t)stream, keys, vals, out_keys, out_vals, n);
  return launch_status();
}
