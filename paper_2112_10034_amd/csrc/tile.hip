// thread_block_tile<T> reductions and masked (divergent) warp operations.
//
// Masked operations keep CUDA's one-element-per-lane mapping: element e
// sits in logical lane e & 31 of logical warp e >> 5, since the masks are
// built from per-lane predicates.  A block handles R rows of 256
// consecutive elements per round (coalesced streaming 4-byte loads, R loads
// in flight per thread), and the whole block runs every round so that the
// exchanges always see full warps (16 rows per round, eight blocks per
// compute unit).  Into a 16-byte aligned output, each group of four lanes
// writes its four outputs as one streaming 16-byte vector.
//
// Tile reductions are int32 sums modulo 2^32, whose value does not depend
// on the order of the additions, so the kernel loads 16-byte vectors: a
// lane holds 4 consecutive elements, adds them, and a tile of T elements is
// finished by the xor exchanges of the T/4 lanes holding it -- the same bits
// as the one-element-per-lane shfl_down tree.  A block takes two rows of
// 1024 elements per round, four 256-thread blocks per compute unit (eight
// for tiles of 2); tiles of 4, 8 and 16 write four consecutive sums as one
// streaming 16-byte vector into an aligned output.
#include "cox_internal.hpp"

namespace cox {

// 16-byte vectors at 4-byte aligned addresses (one dwordx4 access each)
typedef uint32_t u32x4u __attribute__((ext_vector_type(4), aligned(4)));

// the lanes of a tile hold T/4 x 4 consecutive elements: in-lane sum, then
// xor exchanges inside the T/4-lane group (every lane of it ends with the sum)
template <int T>
__device__ __forceinline__ void tile_sums(const uint32_t (&v)[4], uint32_t &a, uint32_t &b) {
  if constexpr (T == 2) {
    a = v[0] + v[1];
    b = v[2] + v[3];
  } else {
    uint32_t s = (v[0] + v[1]) + (v[2] + v[3]);
    if constexpr (T >= 8) s += (uint32_t)xor_lane<1>((int)s);
    if constexpr (T >= 16) s += (uint32_t)xor_lane<2>((int)s);
    if constexpr (T >= 32) s += (uint32_t)xor_lane<4>((int)s);
    a = s;
    b = 0u;
  }
}

template <int T, int R>
__global__ __launch_bounds__(256) void k_tile_reduce(const int32_t *__restrict__ x, int64_t n,
                                                     int32_t *__restrict__ out, bool vec_out) {
  constexpr int G = T >= 4 ? T / 4 : 1;  // lanes per tile
  const int t = threadIdx.x, l = t & 31;
  const int64_t per_block = 1024 * R;
  const int64_t stride = (int64_t)gridDim.x * per_block;
  const int64_t rounds = (n + stride - 1) / stride;
  const int64_t nt = (n + T - 1) / T;
  for (int64_t it = 0; it < rounds; it++) {
    const int64_t base = it * stride + (int64_t)blockIdx.x * per_block;
    uint32_t v[R][4];
    const bool full = base + per_block <= n;
    if (full) {
#pragma unroll
      for (int r = 0; r < R; r++) {
        const u32x4u q = __builtin_nontemporal_load((const u32x4u *)(x + base + r * 1024 + 4 * t));
        v[r][0] = q.x; v[r][1] = q.y; v[r][2] = q.z; v[r][3] = q.w;
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; r++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int64_t e = base + r * 1024 + 4 * t + j;
          v[r][j] = e < n ? ld_stream1(x + e) : 0u;
        }
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t e = base + r * 1024 + 4 * t;  // first element of the lane
      uint32_t a, b;
      tile_sums<T>(v[r], a, b);
      if constexpr (T >= 4 && T <= 16) {
        // every lane of a tile holds its sum; in a full round the first lane
        // of four consecutive tiles takes the other three from lanes G, 2G
        // and 3G further on (all in its 16-lane row) and writes the four as
        // one streaming 16-byte vector
        if (vec_out && full) {
          const uint32_t a1 = (uint32_t)dpp_mov<0x100 + G>((int)a);      // row_shl:G
          const uint32_t a2 = (uint32_t)dpp_mov<0x100 + 2 * G>((int)a);  // row_shl:2G
          const uint32_t a3 = (uint32_t)dpp_mov<0x100 + 3 * G>((int)a);  // row_shl:3G
          if ((l & (4 * G - 1)) == 0) st_stream4(out + e / T, a, a1, a2, a3);
          continue;
        }
      }
      if constexpr (T == 2) {
        if (e / 2 < nt) out[e / 2] = (int32_t)a;
        if (e / 2 + 1 < nt) out[e / 2 + 1] = (int32_t)b;
      } else {
        if ((l & (G - 1)) == 0 && e / T < nt) out[e / T] = (int32_t)a;
      }
    }
  }
}

// v with lane `lane` replaced by the wave-uniform value u (v_writelane writes
// one lane of a vector register, whatever the execution mask)
template <int L>
__device__ __forceinline__ uint32_t with_lane(uint32_t v, uint32_t u) {
  asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(__builtin_amdgcn_readfirstlane((int)u)), "i"(L));
  return v;
}

// row r of a wave's round of masked operations (see k_warp_masked): the
// two warps' record values go to lanes 2r and 2r + 1 of rm (mask), rb
// (ballot of x > 0), ra / rl (the any / all ballots within the mask) and
// rc (leader value); the flags word is formed from them once per round
template <int r, int R, bool VEC>
__device__ __forceinline__ void masked_rows(const int32_t (&xs)[R], int32_t *__restrict__ dst, uint32_t D,
                                            uint32_t hib, uint32_t lp1, uint32_t &rm, uint32_t &rb, uint32_t &ra,
                                            uint32_t &rl, uint32_t &rc) {
  if constexpr (r < R) {
    const int32_t xv = xs[r];
    const bool p = ((uint32_t)xv & 1023u) < D;
    const uint64_t P = __builtin_amdgcn_ballot_w64(p);
    const uint64_t Bq = __builtin_amdgcn_ballot_w64(xv > 0) & P;
    const uint64_t Aq = __builtin_amdgcn_ballot_w64((xv & 0x7c00) == 0) & P;
    const uint64_t Lq = __builtin_amdgcn_ballot_w64((xv & 0xf8000) != 0) & P;
    // m = this half's mask; lanes outside m read some lane and discard it
    // (m == 0 leaves the count undefined, and every such lane discards)
    const uint32_t m = (uint32_t)(P >> hib);
    const uint32_t c = (uint32_t)__builtin_ctz(__builtin_amdgcn_alignbit(m, m, lp1));
    const int32_t sv = bperm(xv, (int)(((c + lp1) & 31u) | hib));
    const int32_t ov = p ? sv : INT32_MIN;
    if constexpr (VEC) {
      // lanes 4q .. 4q + 3 hold consecutive outputs: lane 4q takes the other
      // three (DPP row_shl:1, 2, 3) and writes one streaming 16-byte vector
      const int32_t o1 = dpp_mov<0x101>(ov), o2 = dpp_mov<0x102>(ov), o3 = dpp_mov<0x103>(ov);
      if ((lp1 & 3u) == 1u) st_stream4(dst + r * 64, (uint32_t)ov, (uint32_t)o1, (uint32_t)o2, (uint32_t)o3);
    } else {
      dst[r * 64] = ov;
    }
    const uint32_t m0 = (uint32_t)P, m1 = (uint32_t)(P >> 32);
    // leader values read unconditionally (no branch), zero for an empty warp
    const uint32_t bl0 = (uint32_t)__builtin_amdgcn_readlane(xv, m0 ? __builtin_ctz(m0) : 0);
    const uint32_t bl1 = (uint32_t)__builtin_amdgcn_readlane(xv, 32 + (m1 ? __builtin_ctz(m1) : 0));
    rm = with_lane<2 * r + 1>(with_lane<2 * r>(rm, m0), m1);
    rb = with_lane<2 * r + 1>(with_lane<2 * r>(rb, (uint32_t)Bq), (uint32_t)(Bq >> 32));
    ra = with_lane<2 * r + 1>(with_lane<2 * r>(ra, (uint32_t)Aq), (uint32_t)(Aq >> 32));
    rl = with_lane<2 * r + 1>(with_lane<2 * r>(rl, (uint32_t)Lq), (uint32_t)(Lq >> 32));
    rc = with_lane<2 * r + 1>(with_lane<2 * r>(rc, m0 ? bl0 : 0u), m1 ? bl1 : 0u);
    masked_rows<r + 1, R, VEC>(xs, dst, D, hib, lp1, rm, rb, ra, rl, rc);
  }
}

// The masked operations without a divergent branch: every ballot is taken
// once over the whole wave (a wave-uniform 64-bit value in scalar
// registers), each logical warp's mask m, its ballot b, any / all results
// and leader broadcast are derived from the half of that value, and every
// lane computes its shuffle; lanes outside m then store INT32_MIN instead.
// The stored values are those of the divergent CUDA code, whose lanes of m
// are exactly the lanes that would execute it.
//
// A wave owns 64R consecutive elements per round (row r: elements
// 64r .. 64r + 63, the logical warps 2r and 2r + 1 of the wave), so one
// base address serves every row.  The next lane of m above l, wrapping, is
// the first set bit of m rotated right by l + 1, counted from lane l + 1.
// The 2R records of a round are gathered in lanes 0 .. 2R - 1 (lane 2r + h
// holds warp 2r + h's values, written with v_writelane from the
// wave-uniform ballots), their flag words formed there, and stored as one
// contiguous run of 16-byte vectors.
template <int R, bool VEC>
__global__ __launch_bounds__(256) void k_warp_masked(const int32_t *__restrict__ x, int64_t n, int D,
                                                     int32_t *__restrict__ out, uint32_t *__restrict__ rec) {
  static_assert(2 * R <= 64, "records of a round fit in one wave");
  const int t = threadIdx.x, l = t & 31, lane = t & 63;
  const uint32_t hib = (uint32_t)(t & 32);  // first lane of the caller's half
  const uint32_t lp1 = (uint32_t)l + 1u;
  const int64_t per_wave = 64 * R;
  const int64_t per_block = 4 * per_wave;
  const int64_t stride = (int64_t)gridDim.x * per_block;
  const int64_t rounds = (n + stride - 1) / stride;
  for (int64_t it = 0; it < rounds; it++) {
    const int64_t wbase = it * stride + (int64_t)blockIdx.x * per_block + (t >> 6) * per_wave;
    if (wbase + per_wave <= n) {
      const int32_t *src = x + wbase + lane;
      int32_t *dst = out + wbase + lane;
      int32_t xs[R];
#pragma unroll
      for (int r = 0; r < R; r++) xs[r] = (int32_t)ld_stream1(src + r * 64);
      uint32_t rm = 0u, rb = 0u, ra = 0u, rl = 0u, rc = 0u;
      masked_rows<0, R, VEC>(xs, dst, (uint32_t)D, hib, lp1, rm, rb, ra, rl, rc);
      // flags: any in bit 0, all in bit 1 (an empty warp's record is zero)
      const uint32_t rf = (ra != 0u ? 1u : 0u) | (rm != 0u && rl == rm ? 2u : 0u);
      if (lane < 2 * R) *(uint4 *)(rec + 4 * ((wbase >> 5) + lane)) = make_uint4(rm, rb, rf, rc);
    } else {
      // partial last round: whole logical warps only (n % 32 == 0), so a
      // warp is either entirely in range or entirely out
#pragma unroll 1
      for (int r = 0; r < R; r++) {
        const int64_t e = wbase + r * 64 + lane;
        const int64_t e32 = e & ~(int64_t)31;
        if (e32 >= n) continue;  // uniform per logical warp
        const int32_t xv = (int32_t)ld_stream1(x + e);
        const bool p = ((uint32_t)xv & 1023u) < (uint32_t)D;
        const uint32_t m = ballot(p);
        const uint32_t b = ballot(xv > 0) & m;
        const uint32_t A = (ballot(((xv >> 10) & 31) == 0) & m) != 0u;
        const uint32_t L = (ballot(((xv >> 15) & 31) != 0) & m) == m;
        const uint32_t above = m & (l == 31 ? 0u : (FULL << (l + 1)));
        const int sl = above ? __builtin_ctz(above) : (m ? __builtin_ctz(m) : l);
        const int32_t sv = shfl(xv, sl);
        const int32_t bc = shfl(xv, m ? __builtin_ctz(m) : 0);
        out[e] = p ? sv : INT32_MIN;
        if (l == 0)
          *(uint4 *)(rec + 4 * (e >> 5)) = m ? make_uint4(m, b, A | (L << 1), (uint32_t)bc) : make_uint4(0u, 0u, 0u, 0u);
      }
    }
  }
}

using tred_fn = void (*)(const int32_t *, int64_t, int32_t *, bool);
static tred_fn pick_tile(int T) {
  switch (T) {
  case 2: return k_tile_reduce<2, 2>;
  case 4: return k_tile_reduce<4, 2>;
  case 8: return k_tile_reduce<8, 2>;
  case 16: return k_tile_reduce<16, 2>;
  case 32: return k_tile_reduce<32, 2>;
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
  // two rows of 1024 elements per block and round, four blocks per compute
  // unit (eight for tiles of 2), measured over 2^26 elements after a cache
  // scrub: 45.9 / 50.8 / 55.9 us for T = 32 / 16 / 8 against 48.6 / 52.7 /
  // 57.9 us with four rows.  Tiles of 4, 8 and 16 write their sums as
  // 16-byte vectors into an aligned out: 58.3 / 52.3 / 47.2 us against
  // 61.8 / 55.5 / 51.0 with one 4-byte store per tile (tiles of 4 with
  // eight blocks per compute unit: 64.1 us)
  const int grid = persistent_grid((const void *)fn, 256, (n + 1024 * 2 - 1) / (1024 * 2), 0, 0, tile <= 2 ? 8 : 4);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, (hipStream_t)stream, x, n, out, aligned16(out));
  return launch_status();
}

cox_status cox_warp_masked(const int32_t *x, int64_t n, int density, int32_t *out, uint32_t *rec,
                           void *stream) {
  if (n < 0 || n % 32 || density < 0 || density > 1024) return COX_ERR_INVALID;
  if (n == 0) return COX_OK;
  if (!x || !out || !rec) return COX_ERR_INVALID;
  if (!aligned16(rec)) return COX_ERR_ALIGN;
  // an aligned out takes 16-byte streaming stores of four lanes' outputs:
  // 104 against 107 us over 2^26 elements after a cache scrub
  auto fn = aligned16(out) ? k_warp_masked<16, true> : k_warp_masked<16, false>;
  const int grid = persistent_grid((const void *)fn, 256, (n + 256 * 16 - 1) / (256 * 16), 0, 0, 8);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, (hipStream_t)stream, x, n, density, out, rec);
  return launch_status();
}

}  // extern "C"
