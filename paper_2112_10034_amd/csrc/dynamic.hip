// Dynamic groups: coalesced_threads(), __match_any_sync / __match_all_sync
// and __reduce_{add,min,max,and,or,xor}_sync, with a warp-aggregated append
// (the pattern of the filter kernel that needs a dynamic cooperative group,
// which COX could not run: its Table 1; Sec. 2.2.2-2.2.3 for the groups).
//
// One element per lane (element e: logical lane e & 31 of logical warp
// e >> 5), rows of blockDim consecutive elements, R rows per round.  Per
// row:
//   p = ((uint32)x & 1023) < D; the members m of a logical warp are the
//   lanes with p (the group coalesced_threads() returns inside `if (p)`);
//   rank = popc(m & lanemask_lt) (mbcnt over the wave's 64-bit ballot);
//   the six reductions: all-reduce inside each 16-lane row by DPP row
//   rotations (8, 4, 2, 1) fused into the ALU op, then one row swap
//   (v_permlane16_swap); lanes outside m hold the operation's identity;
//   match_any(m, key): m intersected, for every key bit on which the
//   members differ, with the members agreeing with the lane on that bit
//   (one ballot per bit) -- one step per varying bit.  The key is bits
//   10..12 of x, so the bits on which the members differ are those of
//   (OR ^ AND) of x over the members, already reduced;
//   match_all: a member's match set is the whole mask;
//   append: the rank-0 member takes the group's slots from a block
//   counter in shared memory, the members read the base from it (a
//   shuffle from the rank-0 lane); once per round one global atomic turns
//   the block's slots into output positions.
// Lanes outside m compute and discard: the stored values are those of the
// divergent code, whose executing lanes are exactly m.
#include "cox_internal.hpp"

namespace cox {

// all-reduce of v over the logical warp's 32 lanes for a commutative op
// with identity ID (every lane ends with the result): rotations inside the
// 16-lane rows, then v_permlane16_swap of v with itself, which leaves every
// lane its own row's value and the other row's, in one order or the other.
// The rotation is a DPP update whose old value is the identity: the
// compiler folds it into the op (v_add_u32_dpp, v_min_i32_dpp, ...; a
// plain DPP move would stay a separate instruction).  Row rotations read
// no invalid lane, so the old value never shows.
template <uint32_t ID, class F>
__device__ __forceinline__ uint32_t allreduce32(uint32_t v, F op) {
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)ID, (int)v, 0x128, 0xf, 0xf, false));  // row_ror:8
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)ID, (int)v, 0x124, 0xf, 0xf, false));  // row_ror:4
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)ID, (int)v, 0x122, 0xf, 0xf, false));  // row_ror:2
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)ID, (int)v, 0x121, 0xf, 0xf, false));  // row_ror:1
  const auto pr = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return op((uint32_t)pr[0], (uint32_t)pr[1]);
}

template <int R>
__global__ __launch_bounds__(1024) void k_warp_dynamic(const int32_t *__restrict__ x, int64_t n, int D,
                                                      uint32_t *__restrict__ mm_out, uint32_t *__restrict__ rank_out,
                                                      uint32_t *__restrict__ rec, int32_t *__restrict__ filt,
                                                      unsigned long long *__restrict__ counter) {
  __shared__ uint32_t s_cnt;
  __shared__ unsigned long long s_base;
  const int t = threadIdx.x, l = t & 31;
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
    // a member's slot in the block's range (< 2^15), two rows per register
    uint32_t pos2[R / 2];
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
      // reductions over the members of the warp (identity elsewhere)
      const auto add = [](uint32_t a, uint32_t b) { return a + b; };
      const auto mn = [](uint32_t a, uint32_t b) { return (int32_t)a < (int32_t)b ? a : b; };
      const auto mx = [](uint32_t a, uint32_t b) { return (int32_t)a > (int32_t)b ? a : b; };
      const auto bor = [](uint32_t a, uint32_t b) { return a | b; };
      const auto bxor = [](uint32_t a, uint32_t b) { return a ^ b; };
      const uint32_t ra = allreduce32<0u>(p ? ((uint32_t)xv & 0xFFFFu) : 0u, add);
      const uint32_t rmn = allreduce32<(uint32_t)INT32_MAX>(p ? (uint32_t)xv : (uint32_t)INT32_MAX, mn);
      const uint32_t rmx = allreduce32<(uint32_t)INT32_MIN>(p ? (uint32_t)xv : (uint32_t)INT32_MIN, mx);
      // AND as the complement of the OR of the complements (an OR update
      // folds into its op; an AND one does not)
      const uint32_t rnd = ~allreduce32<0u>(p ? ~(uint32_t)xv : 0u, bor);
      const uint32_t rr = allreduce32<0u>(p ? (uint32_t)xv : 0u, bor);
      const uint32_t rx = allreduce32<0u>(p ? (uint32_t)xv : 0u, bxor);
      // match_any: m narrowed by one agreement ballot per key bit on which
      // the wave's members differ
      const uint32_t kvary = ((rr ^ rnd) >> 10) & 7u;
      uint32_t vary = (uint32_t)__builtin_amdgcn_readlane((int)kvary, 0) |
                      (uint32_t)__builtin_amdgcn_readlane((int)kvary, 32);
      uint32_t mm = m;
      while (vary) {
        const int b = __builtin_ctz(vary);
        const bool bit = (key >> b) & 1u;
        const uint64_t B = __builtin_amdgcn_ballot_w64(bit);
        const uint32_t Bh = (uint32_t)((B & my_half) >> (hi ? 32 : 0));
        mm &= bit ? Bh : ~Bh;
        vary &= vary - 1u;
      }
      const uint32_t ma = (p && mm == m) ? m : 0u;
      // the warp's record, from its rank-0 member (lane 0 if m is empty)
      const int wl = m ? __builtin_ctz(m) : 0;
      if (in && l == wl) {
        uint4 *dst = (uint4 *)(rec + 8 * (e >> 5));
        if (m) {
          dst[0] = make_uint4(m, ma, ra, rmn);
          dst[1] = make_uint4(rmx, rnd, rr, rx);
        } else {
          dst[0] = make_uint4(0u, 0u, 0u, 0u);
          dst[1] = make_uint4(0u, 0u, 0u, 0u);
        }
      }
      // warp-aggregated append: the group's slots in the block's range
      uint32_t slot = 0u;
      if (p && rank == 0u) slot = atomicAdd(&s_cnt, (uint32_t)__builtin_popcount(m));
      const uint32_t pos = (uint32_t)bperm((int)slot, (hi ? 32 : 0) + wl) + rank;
      if (r & 1) pos2[r / 2] |= pos << 16;
      else pos2[r / 2] = pos;
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
      if ((pbits >> r) & 1u) filt[gb + ((pos2[r / 2] >> (16 * (r & 1))) & 0xFFFFu)] = xs[r];
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
  // 512-thread blocks: three per compute unit at this kernel's registers
  auto fn = k_warp_dynamic<16>;
  const int grid = persistent_grid((const void *)fn, 512, (n + 512 * 16 - 1) / (512 * 16), 0, 0, 4);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(512), 0, (hipStream_t)stream, x, n, density, match_any, rank, rec,
                     filtered, (unsigned long long *)filtered_count);
  return launch_status();
}

}  // extern "C"
