// Logical 32-lane warps on gfx950 wave64.
//
// Every 64-lane wavefront carries two logical CUDA warps: physical lanes
// 0-31 are warp 2q, lanes 32-63 warp 2q+1.  A logical lane is lane & 31.
// Every primitive below keeps its data inside its own 32-lane half.
//
// General primitives (runtime arguments, any lane pattern) use ds_bpermute
// with the source index confined to the caller's half; they implement the
// CUDA rules exactly (out-of-range sources return the caller's own value,
// width segments, xor reading earlier segments).  Fixed-pattern exchanges
// used inside kernels are DPP or ds_swizzle:
//   xor 1, 2, 3   -> DPP quad_perm          (within 4 lanes)
//   xor 7         -> DPP row_half_mirror    (lane i <-> 7-i within 8)
//   xor 8         -> DPP row_ror:8          (within a 16-lane row)
//   xor 15        -> DPP row_mirror         (lane i <-> 15-i within a row)
//   any xor < 32  -> ds_swizzle bitmask mode (works on 32-lane groups,
//                    which are exactly the logical warps)
//   shift up by d within 16 lanes -> DPP row_shr:d
//   lane 15 of a row into the next row -> DPP row_bcast:15 (row_mask 0xa
//                    writes rows 1 and 3 only, so nothing crosses 31 -> 32)
//   lane 31 of each half to the whole half -> ds_swizzle (and 0, or 31)
// A ballot is one 32-bit half of the 64-bit wave ballot.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cox {

constexpr uint32_t FULL = 0xffffffffu;

__device__ __forceinline__ int lane64() { return (int)__lane_id(); }
__device__ __forceinline__ int llane() { return (int)__lane_id() & 31; }
__device__ __forceinline__ int lhalf() { return (int)__lane_id() >> 5; }

// ---------------------------------------------------------------- bit casts
__device__ __forceinline__ int f2i(float f) { return __builtin_bit_cast(int, f); }
__device__ __forceinline__ float i2f(int i) { return __builtin_bit_cast(float, i); }

// ---------------------------------------------------------------- general shuffles
// ds_bpermute: lane reads lane (addr / 4) mod 64 of the wave
__device__ __forceinline__ int bperm(int v, int phys_lane) {
  return __builtin_amdgcn_ds_bpermute(phys_lane << 2, v);
}
__device__ __forceinline__ int to_phys(int logical) { return (lhalf() << 5) | (logical & 31); }

__device__ __forceinline__ int shfl_idx_src(int l, int src, int w) {
  return (l & ~(w - 1)) + (src & (w - 1));
}
__device__ __forceinline__ int shfl_up_src(int l, int d, int w) {
  int b = l & ~(w - 1);
  return (l - b >= d) ? l - d : l;
}
__device__ __forceinline__ int shfl_down_src(int l, int d, int w) {
  int b = l & ~(w - 1);
  return (l - b + d < w) ? l + d : l;
}
__device__ __forceinline__ int shfl_xor_src(int l, int m, int w) {
  int b = l & ~(w - 1);
  int j = l ^ m;
  return (j < b + w) ? j : l;
}

__device__ __forceinline__ int shfl(int v, int src, int w = 32) {
  return bperm(v, to_phys(shfl_idx_src(llane(), src, w)));
}
__device__ __forceinline__ int shfl_up(int v, int d, int w = 32) {
  return bperm(v, to_phys(shfl_up_src(llane(), d, w)));
}
__device__ __forceinline__ int shfl_down(int v, int d, int w = 32) {
  return bperm(v, to_phys(shfl_down_src(llane(), d, w)));
}
__device__ __forceinline__ int shfl_xor(int v, int m, int w = 32) {
  return bperm(v, to_phys(shfl_xor_src(llane(), m, w)));
}

// ---------------------------------------------------------------- votes
// ballot over the executing lanes of the caller's logical warp
__device__ __forceinline__ uint32_t ballot(bool p) {
  uint64_t b = __builtin_amdgcn_ballot_w64(p);
  return lhalf() ? (uint32_t)(b >> 32) : (uint32_t)b;
}
__device__ __forceinline__ uint32_t activemask() { return ballot(true); }
// masked votes: every lane of `mask` executes the call (CUDA requirement)
__device__ __forceinline__ uint32_t ballot_sync(uint32_t mask, bool p) { return ballot(p) & mask; }
__device__ __forceinline__ bool any_sync(uint32_t mask, bool p) { return ballot_sync(mask, p) != 0; }
__device__ __forceinline__ bool all_sync(uint32_t mask, bool p) { return ballot_sync(mask, p) == mask; }
__device__ __forceinline__ uint32_t lanemask_lt() {
  int l = llane();
  return l ? (FULL >> (32 - l)) : 0u;
}

// ---------------------------------------------------------------- fixed patterns
// DPP controls (GFX9 encoding)
enum : int {
  DPP_QUAD_XOR1 = 0xB1,  // quad_perm [1,0,3,2]
  DPP_QUAD_XOR2 = 0x4E,  // quad_perm [2,3,0,1]
  DPP_QUAD_XOR3 = 0x1B,  // quad_perm [3,2,1,0]
  DPP_ROW_SHR1 = 0x111,
  DPP_ROW_SHR2 = 0x112,
  DPP_ROW_SHR4 = 0x114,
  DPP_ROW_SHR8 = 0x118,
  DPP_ROW_ROR8 = 0x128,
  DPP_WAVE_SHR1 = 0x138,
  DPP_ROW_MIRROR = 0x140,
  DPP_ROW_HALF_MIRROR = 0x141,
  DPP_ROW_BCAST15 = 0x142,
};

// lane gets `v` of the DPP source lane; `old` where the source is invalid
// or the row is masked off
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ int dpp(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROW_MASK, BANK_MASK, false);
}

// ds_swizzle bitmask mode within each 32-lane group: lane l reads
// ((l & AND) | OR) ^ XOR
template <int AND, int OR, int XOR>
__device__ __forceinline__ int swz(int v) {
  return __builtin_amdgcn_ds_swizzle(v, (XOR << 10) | (OR << 5) | AND);
}

// DPP move for patterns whose every source lane is valid (no "old" value
// needed, so no copy into the destination first)
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, false);
}

// value of logical partner lane l ^ M (M < 32), fixed pattern
template <int M>
__device__ __forceinline__ int xor_lane(int v) {
  if constexpr (M == 1) return dpp_mov<DPP_QUAD_XOR1>(v);
  else if constexpr (M == 2) return dpp_mov<DPP_QUAD_XOR2>(v);
  else if constexpr (M == 3) return dpp_mov<DPP_QUAD_XOR3>(v);
  else if constexpr (M == 7) return dpp_mov<DPP_ROW_HALF_MIRROR>(v);
  else if constexpr (M == 8) return dpp_mov<DPP_ROW_ROR8>(v);
  else if constexpr (M == 15) return dpp_mov<DPP_ROW_MIRROR>(v);
  else return swz<0x1f, 0, M>(v);
}

// median of three unsigned values (one v_med3_u32); med3(a, b, 0) is
// min(a, b) and med3(a, b, ~0) is max(a, b)
__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// logical lane 31's value in every lane of the half
__device__ __forceinline__ int bcast31(int v) { return swz<0, 31, 0>(v); }

template <int M>
__device__ __forceinline__ float xor_lane_f(float v) { return i2f(xor_lane<M>(f2i(v))); }
template <int M>
__device__ __forceinline__ double xor_lane_d(double v) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = xor_lane<M>(p.x);
  p.y = xor_lane<M>(p.y);
  return __builtin_bit_cast(double, p);
}

}  // namespace cox
