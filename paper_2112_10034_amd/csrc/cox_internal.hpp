// Host/device helpers shared by the library's HIP sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cox.h"
#include "cox_warp.hpp"

namespace cox {

// ---------------------------------------------------------------- workspace
// First 256 bytes: header words; data (status words / partials) follows.
enum : int { HDR_TICKET = 0, HDR_EPOCH = 1, HDR_DONE = 2, HDR_ERR = 3, HDR_WORDS = 64 };
constexpr size_t WS_HEADER = 256;

// HDR_ERR holds the tag of a call whose bounded wait gave up; ERR_LAYOUT
// (never a tag: tags are below 2^30) reports segment offsets whose chunks
// exceed the workspace's capacity
constexpr uint32_t ERR_LAYOUT = 0x80000000u;

// look-back status word: [tag:30][flag:2][value:32].  In a workspace the
// words of consecutive chunks sit ST_STRIDE words (128 bytes) apart, one
// per cache line: device-scope polls of one chunk's word and stores of its
// neighbours' then no longer meet on a line (scan 0.372 -> 0.356 ms,
// compaction 0.344 -> 0.325 ms at 2^28).
constexpr int ST_STRIDE = 16;
enum : uint32_t { ST_AGG = 1, ST_PREFIX = 2 };
constexpr uint32_t TAG_MOD = (1u << 30) - 1;
__host__ __device__ __forceinline__ uint32_t tag_of_epoch(uint32_t e) { return 1u + e % TAG_MOD; }
__device__ __forceinline__ uint64_t st_pack(uint32_t tag, uint32_t flag, uint32_t v) {
  return ((uint64_t)tag << 34) | ((uint64_t)flag << 32) | v;
}
__device__ __forceinline__ uint32_t st_tag(uint64_t s) { return (uint32_t)(s >> 34); }
__device__ __forceinline__ uint32_t st_flag(uint64_t s) { return (uint32_t)(s >> 32) & 3u; }
__device__ __forceinline__ uint32_t st_val(uint64_t s) { return (uint32_t)s; }

// device-scope (all XCDs) relaxed atomics: on gfx950 these are sc1
// loads/stores that bypass the per-XCD L2's non-coherent copies
__device__ __forceinline__ uint64_t ld_dev(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_dev32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_dev32(uint32_t *p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The call's epoch, read with acquire ordering before the block draws any
// ticket (the block that resets the epoch does so after every block has
// drawn its last ticket).
__device__ __forceinline__ uint32_t ld_epoch(const uint32_t *hdr) {
  return __hip_atomic_load(&hdr[HDR_EPOCH], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// spin bound of every cross-block wait (well under a second); a wait that
// runs out, or that sees another wait's failure, sets HDR_ERR and proceeds,
// so no kernel can hang
constexpr uint32_t MAX_SPIN = 1u << 20;

// Streaming (non-temporal) 16/8/4-byte loads and stores.  Data that is
// read or written once per call bypasses the cache hierarchy's retention;
// on MI355X this raises sustained HBM read bandwidth from about 4.6 to
// about 6.6 TB/s for a plain streaming read.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_stream4(void *p, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  u32x4 v = {a, b, c, d};
  __builtin_nontemporal_store(v, (u32x4 *)p);
}
__device__ __forceinline__ void st_stream2(void *p, uint32_t a, uint32_t b) {
  u32x2 v = {a, b};
  __builtin_nontemporal_store(v, (u32x2 *)p);
}
__device__ __forceinline__ void st_stream1(void *p, uint32_t a) { __builtin_nontemporal_store(a, (uint32_t *)p); }
__device__ __forceinline__ u32x4 ld_stream4(const void *p) { return __builtin_nontemporal_load((const u32x4 *)p); }
__device__ __forceinline__ u32x2 ld_stream2(const void *p) { return __builtin_nontemporal_load((const u32x2 *)p); }
__device__ __forceinline__ uint32_t ld_stream1(const void *p) {
  return __builtin_nontemporal_load((const uint32_t *)p);
}
__device__ __forceinline__ uint16_t ld_stream_h(const void *p) {
  return __builtin_nontemporal_load((const uint16_t *)p);
}

// ---------------------------------------------------------------- host side
void set_hip_error(hipError_t e);
cox_status launch_status();                      // hipGetLastError -> status
int device_cus();                                // compute units of the current device
size_t device_max_lds();                         // shared memory per block of the current device
int blocks_per_cu(const void *kernel, int block, size_t dyn_lds = 0);  // occupancy, cached
// grid of a persistent kernel: `requested` if nonzero, else
// min(occupancy, per_cu) blocks on every compute unit; never more blocks
// than work items
int persistent_grid(const void *kernel, int block, int64_t work_items, int32_t requested, size_t dyn_lds = 0,
                    int per_cu = 1 << 30);

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
inline bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

// resolved schedule
struct Sigma {
  int k, W, G;
};
cox_status resolve_cfg(cox_op op, cox_dtype dt, const cox_cfg *cfg, Sigma *out);
// workspace bytes of a segmented call over nseg segments and at most maxch chunks
size_t seg_workspace_bytes(int64_t nseg, int64_t maxch);
// workspace bytes of a conjugate-gradient solve (n rows, schedule (R, W)) and
// of the grid exchange over G blocks
size_t cg_workspace_bytes(int64_t n, int R, int W);
size_t gx_workspace_bytes(int64_t G);
// workspace bytes of an integral image of height x width pixels
size_t ii_workspace_bytes(int64_t H, int64_t W);

}  // namespace cox
