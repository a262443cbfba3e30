// Dynamic groups: coalesced_threads(), __match_any_sync / __match_all_sync
// and __reduce_{add,min,max,and,or,xor}_sync, with a warp-aggregated append
// (the pattern of the filter kernel that needs a dynamic cooperative group,
// which COX could not run: its Table 1; Sec. 2.2.2-2.2.3 for the groups).
//
// One element per lane (element e: logical lane e & 31 of logical warp
// e >> 5), rows of 1024 consecutive elements, R rows per round.  Per row:
//   p = ((uint32)x & 1023) < D; the members m of a logical warp are the
//   lanes with p (the group coalesced_threads() returns inside `if (p)`);
//   rank = popc(m & lanemask_lt) (mbcnt over the wave's 64-bit ballot);
//   match_any(m, key): the wave walks the distinct (half, key) classes of
//   its members -- a leader's key by v_readlane, one 64-bit ballot per
//   class -- so any 32-bit operand works, in one step per distinct value;
//   match_all: a member's match set is the whole mask;
//   the six reductions: xor butterflies inside the 32-lane half with the
//   operation's identity for lanes outside m;
//   append: the rank-0 member takes the group's slots from a block
//   counter in shared memory, the members read the base from it (a
//   shuffle from the rank-0 lane); once per round one global atomic turns
//   the block's slots into output positions.
// Lanes outside m compute and discard: the stored values are those of the
// divergent code, whose executing lanes are exactly m.
#include "cox_internal.hpp"

namespace cox {

template <int M>
__device__ __forceinline__ uint32_t xl(uint32_t v) {
  return (uint32_t)xor_lane<M>((int)v);
}

__device__ __forceinline__ int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }
__device__ __forceinline__ int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }

template <int R>
__global__ __launch_bounds__(1024) void k_warp_dynamic(const int32_t *__restrict__ x, int64_t n, int D,
                                                      uint32_t *__restrict__ mm_out, uint32_t *__restrict__ rank_out,
                                                      uint32_t *__restrict__ rec, int32_t *__restrict__ filt,
                                                      unsigned long long *__restrict__ counter) {
  __shared__ uint32_t s_cnt;
  __shared__ unsigned long long s_base;
  const int t = threadIdx.x, l = t & 31, t64 = t & 63;
  const bool hi = (t & 32) != 0;
  const uint64_t my_half = hi ? 0xFFFFFFFF00000000ull : 0x00000000FFFFFFFFull;
  const uint32_t lt = l ? (0xFFFFFFFFu >> (32 - l)) : 0u;
  const int64_t per_block = (int64_t)blockDim.x * R;
  const int64_t stride = (int64_t)gridDim.x * per_block;
  const int64_t rounds = (n + stride - 1) / stride;
  if (t == 0) s_cnt = 0u;
  __syncthreads();
  for (int64_t it = 0; it < rounds; it++) {
    const int64_t base = it * stride + (int64_t)blockIdx.x * per_block;
    int32_t xs[R];
    uint32_t wb[R], rk[R];
    uint32_t pbits = 0u;  // bit r: member in row r
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t e = base + (int64_t)r * blockDim.x + t;
      const bool in = e < n;  // whole logical warps (n % 32 == 0)
      xs[r] = in ? (int32_t)ld_stream1(x + e) : 0;
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t e = base + (int64_t)r * blockDim.x + t;
      const bool in = e < n;
      const int32_t xv = xs[r];
      const bool p = in && ((uint32_t)xv & 1023u) < (uint32_t)D;
      const uint64_t P = __builtin_amdgcn_ballot_w64(p);
      const uint32_t m = (uint32_t)((P & my_half) >> (hi ? 32 : 0));
      const uint32_t rank = (uint32_t)__builtin_popcount(m & lt);
      const uint32_t key = ((uint32_t)xv >> 10) & 7u;
      // match_any: one ballot per distinct (half, key) class of members
      uint32_t mm = 0u;
      uint64_t rem = P;
      while (rem) {
        const int ld = __builtin_ctzll(rem);
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, ld);
        const uint64_t cls = __builtin_amdgcn_ballot_w64(key == k) & P &
                             (ld < 32 ? 0x00000000FFFFFFFFull : 0xFFFFFFFF00000000ull);
        if ((cls >> t64) & 1ull) mm = (uint32_t)((cls & my_half) >> (hi ? 32 : 0));
        rem &= ~cls;
      }
      const uint32_t ma = (p && mm == m) ? m : 0u;
      // reductions over the members of the half
      uint32_t ra = p ? ((uint32_t)xv & 0xFFFFu) : 0u;
      int32_t rmn = p ? xv : INT32_MAX, rmx = p ? xv : INT32_MIN;
      uint32_t rnd = p ? (uint32_t)xv : 0xFFFFFFFFu, rr = p ? (uint32_t)xv : 0u, rx = rr;
#define COX_DYN_STEP(M)                                                   \
  ra += xl<M>(ra);                                                        \
  rmn = imin(rmn, (int32_t)xl<M>((uint32_t)rmn));                         \
  rmx = imax(rmx, (int32_t)xl<M>((uint32_t)rmx));                         \
  rnd &= xl<M>(rnd);                                                      \
  rr |= xl<M>(rr);                                                        \
  rx ^= xl<M>(rx);
      COX_DYN_STEP(16)
      COX_DYN_STEP(8)
      COX_DYN_STEP(4)
      COX_DYN_STEP(2)
      COX_DYN_STEP(1)
#undef COX_DYN_STEP
      // the warp's record, from its rank-0 member (lane 0 if m is empty)
      const int wl = m ? __builtin_ctz(m) : 0;
      if (in && l == wl) {
        uint4 *dst = (uint4 *)(rec + 8 * (e >> 5));
        if (m) {
          dst[0] = make_uint4(m, ma, ra, (uint32_t)rmn);
          dst[1] = make_uint4((uint32_t)rmx, rnd, rr, rx);
        } else {
          dst[0] = make_uint4(0u, 0u, 0u, 0u);
          dst[1] = make_uint4(0u, 0u, 0u, 0u);
        }
      }
      // warp-aggregated append: the group's slots in the block's range
      uint32_t slot = 0u;
      if (p && rank == 0u) slot = atomicAdd(&s_cnt, (uint32_t)__builtin_popcount(m));
      wb[r] = (uint32_t)bperm((int)slot, (hi ? 32 : 0) + wl);
      rk[r] = rank;
      pbits |= p ? (1u << r) : 0u;
      if (in) {
        mm_out[e] = p ? mm : 0u;
        rank_out[e] = p ? rank : 0xFFFFFFFFu;
      }
    }
    __syncthreads();
    if (t == 0) {
      s_base = atomicAdd(counter, (unsigned long long)s_cnt);
      s_cnt = 0u;
    }
    __syncthreads();
    const unsigned long long gb = s_base;
#pragma unroll
    for (int r = 0; r < R; r++)
      if ((pbits >> r) & 1u) filt[gb + wb[r] + rk[r]] = xs[r];
    // s_base is rewritten only after the next round's first barrier
  }
}

__global__ void k_dyn_zero(unsigned long long *p) { *p = 0ull; }

}  // namespace cox

using namespace cox;

extern "C" {

cox_status cox_warp_dynamic(const int32_t *x, int64_t n, int density, uint32_t *match_any, uint32_t *rank,
                            uint32_t *rec, int32_t *filtered, int64_t *filtered_count, void *stream) {
  if (n < 0 || n % 32 || density < 0 || density > 1024) return COX_ERR_INVALID;
  if (!filtered_count) return COX_ERR_INVALID;
  hipLaunchKernelGGL(k_dyn_zero, dim3(1), dim3(1), 0, (hipStream_t)stream,
                     (unsigned long long *)filtered_count);
  cox_status st = launch_status();
  if (st != COX_OK || n == 0) return st;
  if (!x || !match_any || !rank || !rec || !filtered) return COX_ERR_INVALID;
  if (!aligned16(rec)) return COX_ERR_ALIGN;
  auto fn = k_warp_dynamic<16>;
  const int grid = persistent_grid((const void *)fn, 1024, (n + 1024 * 16 - 1) / (1024 * 16), 0, 0, 2);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(1024), 0, (hipStream_t)stream, x, n, density, match_any, rank, rec,
                     filtered, (unsigned long long *)filtered_count);
  return launch_status();
}

}  // extern "C"
