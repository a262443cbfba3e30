// C ABI plumbing: status strings, schedules, workspaces, occupancy, and the
// warp-function probes (warp builtins applied to arrays).
#include <map>
#include <mutex>
#include <tuple>
#include <utility>

#include "cox_internal.hpp"

namespace cox {

static thread_local int t_last_hip = 0;

void set_hip_error(hipError_t e) { t_last_hip = (int)e; }

cox_status launch_status() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_hip_error(e);
    return COX_ERR_HIP;
  }
  return COX_OK;
}

int device_cus() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  cache[dev] = cus;
  return cus;
}

size_t device_max_lds() {
  static std::mutex mu;
  static std::map<int, size_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    v = 65536;
  cache[dev] = (size_t)v;
  return (size_t)v;
}

int blocks_per_cu(const void *kernel, int block, size_t dyn_lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void *, int, size_t>, int> cache;
  std::lock_guard<std::mutex> g(mu);
  auto key = std::make_tuple(kernel, block, dyn_lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, dyn_lds) != hipSuccess || nb <= 0)
    nb = 1;
  cache[key] = nb;
  return nb;
}

int persistent_grid(const void *kernel, int block, int64_t work_items, int32_t requested, size_t dyn_lds,
                    int per_cu) {
  int occ = blocks_per_cu(kernel, block, dyn_lds);
  if (per_cu < occ) occ = per_cu;
  int64_t g = requested > 0 ? requested : (int64_t)occ * device_cus();
  if (g > work_items) g = work_items;
  if (g < 1) g = 1;
  return (int)g;
}

cox_status resolve_cfg(cox_op op, cox_dtype dt, const cox_cfg *cfg, Sigma *out) {
  cox_cfg d;
  cox_default_cfg(op, dt, &d);
  int k = (cfg && cfg->items_per_lane) ? cfg->items_per_lane : d.items_per_lane;
  int W = (cfg && cfg->warps_per_block) ? cfg->warps_per_block : d.warps_per_block;
  int G = cfg ? cfg->grid_blocks : 0;
  if (!pow2_in(k, 1, 32) || !pow2_in(W, 1, 32) || G < 0) return COX_ERR_INVALID;
  out->k = k;
  out->W = W;
  out->G = G;
  return COX_OK;
}

// ---------------------------------------------------------------- kernels
__global__ void k_fill_zero(uint32_t *p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// One thread per element; whole logical warps exit together (n % 32 == 0).
// The permute runs with every lane of the warp active and lanes outside
// the mask discard its result, so a source outside the mask reads that
// lane's input.
__global__ void k_warp_shfl(const int32_t *__restrict__ v, int32_t *__restrict__ out, int64_t n,
                            int op, int arg, const int32_t *__restrict__ argv, int width,
                            const uint32_t *__restrict__ mask) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint32_t m = mask ? mask[e >> 5] : FULL;
  const int l = (int)(e & 31);
  const int val = v[e];
  const int a = argv ? argv[e] : arg;
  int src;
  switch (op) {
  case COX_SHFL_IDX: src = shfl_idx_src(l, a, width); break;
  case COX_SHFL_UP: src = shfl_up_src(l, a, width); break;
  case COX_SHFL_DOWN: src = shfl_down_src(l, a, width); break;
  default: src = shfl_xor_src(l, a, width); break;
  }
  const int r = bperm(val, to_phys(src));
  out[e] = ((m >> l) & 1u) ? r : val;
}

// Lanes of the mask execute the votes inside the branch (divergent code);
// the mask's lowest lane stores the warp's results.
__global__ void k_warp_vote(const int32_t *__restrict__ pred, const uint32_t *__restrict__ mask,
                            int64_t n, uint32_t *__restrict__ ballot_out,
                            int32_t *__restrict__ anyall) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t g = e >> 5;
  const uint32_t m = mask ? mask[g] : FULL;
  const int l = (int)(e & 31);
  const bool p = pred[e] != 0;
  if ((m >> l) & 1u) {
    const uint32_t b = ballot_sync(m, p);
    const bool a = any_sync(m, p);
    const bool t = all_sync(m, p);
    if (l == __builtin_ctz(m)) {
      ballot_out[g] = b;
      anyall[g] = (int)a | ((int)t << 1);
    }
  } else if (m == 0u && l == 0) {
    ballot_out[g] = 0u;
    anyall[g] = 0;
  }
}

// Tile-scoped votes of thread_block_tile<T>: one element per lane; the
// logical warp's ballot, shifted down to the lane's tile and cut to T bits,
// is the tile's ballot; the tile's rank-0 lane stores it with any | all << 1.
__global__ void k_tile_vote(const int32_t *__restrict__ pred, int64_t n, int T, uint32_t *__restrict__ ballot_out,
                            int32_t *__restrict__ anyall) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;  // whole logical warps exit together (n % 32 == 0)
  const int l = (int)(e & 31);
  const uint32_t full = T == 32 ? FULL : (1u << T) - 1u;
  const uint32_t b = (ballot(pred[e] != 0) >> (l & ~(T - 1))) & full;
  if ((l & (T - 1)) == 0) {
    ballot_out[e / T] = b;
    anyall[e / T] = (b != 0u ? 1 : 0) | (b == full ? 2 : 0);
  }
}

}  // namespace cox

using namespace cox;

extern "C" {

const char *cox_status_string(cox_status s) {
  switch (s) {
  case COX_OK: return "ok";
  case COX_ERR_INVALID: return "invalid argument";
  case COX_ERR_DTYPE: return "dtype or accumulation not supported by this entry point";
  case COX_ERR_ALIGN: return "data pointer not 16-byte aligned";
  case COX_ERR_HIP: return "HIP call failed";
  case COX_ERR_WORKSPACE: return "workspace missing or too small";
  case COX_ERR_UNSUPPORTED: return "schedule not in the compiled set";
  case COX_ERR_TIMEOUT: return "a bounded cross-block wait gave up";
  }
  return "unknown status";
}

int cox_last_hip_error(void) { return t_last_hip; }

int cox_version(void) { return 100; }

cox_status cox_default_cfg(cox_op op, cox_dtype dtype, cox_cfg *out) {
  if (!out) return COX_ERR_INVALID;
  out->grid_blocks = 0;
  out->reserved = 0;
  // measured on MI355X at 2^28 elements (schedule sweep)
  switch (op) {
  case COX_OP_REDUCE:
    // float32: (32, 32) is fastest for both plain and TwoSum sums;
    // bfloat16: (16, 32)
    out->items_per_lane = dtype == COX_F32 ? 32 : 16;
    out->warps_per_block = dtype == COX_I32 || dtype == COX_U32 ? 16 : 32;
    break;
  case COX_OP_DOT:
    out->items_per_lane = dtype == COX_BF16 ? 32 : 16;
    out->warps_per_block = dtype == COX_BF16 ? 32 : 16;
    break;
  case COX_OP_SCAN:
    out->items_per_lane = 32;
    out->warps_per_block = 32;
    break;
  case COX_OP_COMPACT:
    out->items_per_lane = 32;
    out->warps_per_block = 32;
    break;
  case COX_OP_SEGMENTED:
    // measured on the 10,000-segment lognormal workload: 512-thread blocks
    // of 16384-element chunks, two blocks per compute unit (0.33 / 0.36 ms
    // for int32 / float32 against 0.34 / 0.38 with 256-thread blocks)
    out->items_per_lane = 32;
    out->warps_per_block = 16;
    break;
  case COX_OP_CG:
    out->items_per_lane = 4;
    out->warps_per_block = 32;
    break;
  case COX_OP_GRID_EXCHANGE:
    out->items_per_lane = 1;
    out->warps_per_block = 32;
    break;
  case COX_OP_INTEGRAL_IMAGE:
    out->items_per_lane = 4;
    out->warps_per_block = 8;
    break;
  default: return COX_ERR_INVALID;
  }
  return COX_OK;
}

size_t cox_workspace_bytes(cox_op op, cox_dtype dtype, int64_t n, int64_t nseg, const cox_cfg *cfg) {
  Sigma s;
  if (n < 0 || resolve_cfg(op, dtype, cfg, &s) != COX_OK) return 0;
  const int64_t S = (int64_t)32 * s.W * s.k;
  const int64_t nch = (n + S - 1) / S;
  switch (op) {
  case COX_OP_REDUCE:
  case COX_OP_DOT: return WS_HEADER + 16 * (size_t)(nch + 1);  // up to two tagged words per chunk
  case COX_OP_SCAN:
  case COX_OP_COMPACT: return WS_HEADER + 8 * ST_STRIDE * (size_t)(nch + 1);
  case COX_OP_SEGMENTED: {
    // chunks of every segment (each segment rounds up)
    if (nseg < 0) return 0;
    return seg_workspace_bytes(nseg, n / S + nseg + 1);
  }
  case COX_OP_CG: return cg_workspace_bytes(n, s.k, s.W);
  case COX_OP_GRID_EXCHANGE: return gx_workspace_bytes(n);
  case COX_OP_INTEGRAL_IMAGE: return nseg < 0 ? 0 : ii_workspace_bytes(n, nseg);
  }
  return 0;
}

cox_status cox_workspace_init(void *ws, size_t ws_bytes, void *stream) {
  if (!ws || ws_bytes < WS_HEADER || (ws_bytes & 3)) return COX_ERR_WORKSPACE;
  const int64_t words = (int64_t)(ws_bytes / 4);
  int grid = (int)((words + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, (hipStream_t)stream, (uint32_t *)ws, words);
  return launch_status();
}

cox_status cox_workspace_status(void *ws, void *stream) {
  if (!ws) return COX_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  uint32_t err = 0;
  hipError_t e = hipMemcpyAsync(&err, (uint32_t *)ws + HDR_ERR, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_hip_error(e);
    return COX_ERR_HIP;
  }
  if (!err) return COX_OK;
  const uint32_t zero = 0;
  e = hipMemcpyAsync((uint32_t *)ws + HDR_ERR, &zero, 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_hip_error(e);
    return COX_ERR_HIP;
  }
  return err == ERR_LAYOUT ? COX_ERR_INVALID : COX_ERR_TIMEOUT;
}

cox_status cox_warp_shfl(const int32_t *v, int32_t *out, int64_t n, int op, int32_t arg,
                         const int32_t *argv, int width, const uint32_t *mask, void *stream) {
  if (n < 0 || n % 32 || !pow2_in(width, 1, 32) || op < COX_SHFL_IDX || op > COX_SHFL_XOR)
    return COX_ERR_INVALID;
  if (op != COX_SHFL_IDX && !argv && (arg < 0 || arg > 31)) return COX_ERR_INVALID;
  if (n == 0) return COX_OK;
  if (!v || !out) return COX_ERR_INVALID;
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(k_warp_shfl, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, v, out, n,
                     op, (int)arg, argv, width, mask);
  return launch_status();
}

cox_status cox_tile_vote(const int32_t *pred, int64_t n, int tile, uint32_t *ballot, int32_t *anyall,
                         void *stream) {
  if (n < 0 || n % 32 || !pow2_in(tile, 1, 32)) return COX_ERR_INVALID;
  if (n == 0) return COX_OK;
  if (!pred || !ballot || !anyall) return COX_ERR_INVALID;
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(k_tile_vote, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, pred, n, tile, ballot,
                     anyall);
  return launch_status();
}

cox_status cox_warp_vote(const int32_t *pred, const uint32_t *mask, int64_t n, uint32_t *ballot,
                         int32_t *anyall, void *stream) {
  if (n < 0 || n % 32) return COX_ERR_INVALID;
  if (n == 0) return COX_OK;
  if (!pred || !ballot || !anyall) return COX_ERR_INVALID;
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(k_warp_vote, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, pred, mask,
                     n, ballot, anyall);
  return launch_status();
}

}  // extern "C"
