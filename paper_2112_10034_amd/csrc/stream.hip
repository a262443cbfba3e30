// Bandwidth reference kernels: a plain read and a plain copy of a byte
// range with 16-byte vector accesses, UNROLL vectors in flight per thread.
// They set the achievable HBM ceiling next to which the warp-primitive
// kernels are measured, and are the known-size reference for hardware byte
// counters.
#include "cox_internal.hpp"

namespace cox {

constexpr int UNROLL = 8;

__global__ __launch_bounds__(256) void k_stream_read(const uint4 *__restrict__ x, int64_t nvec,
                                                     uint32_t *__restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  uint32_t acc = 0u;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + (UNROLL - 1) * stride < nvec; i += UNROLL * stride) {
    u32x4 q[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; u++) q[u] = ld_stream4(&x[i + u * stride]);
#pragma unroll
    for (int u = 0; u < UNROLL; u++) acc ^= q[u].x ^ q[u].y ^ q[u].z ^ q[u].w;
  }
  for (; i < nvec; i += stride) {
    const u32x4 q = ld_stream4(&x[i]);
    acc ^= q.x ^ q.y ^ q.z ^ q.w;
  }
  // one word per wave keeps the loads live
  acc ^= (uint32_t)__shfl_xor((int)acc, 32, 64);
  if (lane64() == 0) atomicXor(sink, acc);
}

// copy: persistent blocks walk tiles of 256 * UNROLL_C contiguous vectors
constexpr int UNROLL_C = 4;
__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ x, uint4 *__restrict__ y,
                                                     int64_t nvec) {
  const int64_t ntiles = nvec / (256 * UNROLL_C);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t o = t * 256 * UNROLL_C + threadIdx.x;
    u32x4 q[UNROLL_C];
#pragma unroll
    for (int u = 0; u < UNROLL_C; u++) q[u] = ld_stream4(&x[o + u * 256]);
#pragma unroll
    for (int u = 0; u < UNROLL_C; u++) st_stream4(&y[o + u * 256], q[u].x, q[u].y, q[u].z, q[u].w);
  }
  // remainder vectors past the last whole tile
  for (int64_t i = ntiles * 256 * UNROLL_C + (int64_t)blockIdx.x * 256 + threadIdx.x; i < nvec;
       i += (int64_t)gridDim.x * 256) {
    const u32x4 q = ld_stream4(&x[i]);
    st_stream4(&y[i], q.x, q.y, q.z, q.w);
  }
}

}  // namespace cox

using namespace cox;

extern "C" {

cox_status cox_stream_read(const void *x, size_t bytes, uint32_t *sink, int32_t grid_blocks, void *stream) {
  if ((bytes & 15) || grid_blocks < 0 || !sink) return COX_ERR_INVALID;
  if (bytes == 0) return COX_OK;
  if (!x) return COX_ERR_INVALID;
  if (!aligned16(x)) return COX_ERR_ALIGN;
  const int64_t nvec = (int64_t)(bytes / 16);
  const int grid = persistent_grid((const void *)k_stream_read, 256, (nvec + 255) / 256, grid_blocks, 0, 2);
  hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const uint4 *)x, nvec, sink);
  return launch_status();
}

cox_status cox_stream_copy(const void *src, void *dst, size_t bytes, int32_t grid_blocks, void *stream) {
  if ((bytes & 15) || grid_blocks < 0) return COX_ERR_INVALID;
  if (bytes == 0) return COX_OK;
  if (!src || !dst) return COX_ERR_INVALID;
  if (!aligned16(src) || !aligned16(dst)) return COX_ERR_ALIGN;
  const int64_t nvec = (int64_t)(bytes / 16);
  const int grid = persistent_grid((const void *)k_stream_copy, 256, (nvec + 255) / 256, grid_blocks, 0, 16);
  hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const uint4 *)src,
                     (uint4 *)dst, nvec);
  return launch_status();
}

}  // extern "C"
