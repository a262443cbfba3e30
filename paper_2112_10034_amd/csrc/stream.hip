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
    uint4 q[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; u++) q[u] = x[i + u * stride];
#pragma unroll
    for (int u = 0; u < UNROLL; u++) acc ^= q[u].x ^ q[u].y ^ q[u].z ^ q[u].w;
  }
  for (; i < nvec; i += stride) {
    const uint4 q = x[i];
    acc ^= q.x ^ q.y ^ q.z ^ q.w;
  }
  // one word per wave keeps the loads live
  acc ^= (uint32_t)__shfl_xor((int)acc, 32, 64);
  if (lane64() == 0) atomicXor(sink, acc);
}

__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ x, uint4 *__restrict__ y,
                                                     int64_t nvec) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + (UNROLL - 1) * stride < nvec; i += UNROLL * stride) {
    uint4 q[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; u++) q[u] = x[i + u * stride];
#pragma unroll
    for (int u = 0; u < UNROLL; u++) st_stream4(&y[i + u * stride], q[u].x, q[u].y, q[u].z, q[u].w);
  }
  for (; i < nvec; i += stride) {
    const uint4 q = x[i];
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
  const int grid = persistent_grid((const void *)k_stream_read, 256, (nvec + 255) / 256, grid_blocks);
  hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const uint4 *)x, nvec, sink);
  return launch_status();
}

cox_status cox_stream_copy(const void *src, void *dst, size_t bytes, int32_t grid_blocks, void *stream) {
  if ((bytes & 15) || grid_blocks < 0) return COX_ERR_INVALID;
  if (bytes == 0) return COX_OK;
  if (!src || !dst) return COX_ERR_INVALID;
  if (!aligned16(src) || !aligned16(dst)) return COX_ERR_ALIGN;
  const int64_t nvec = (int64_t)(bytes / 16);
  const int grid = persistent_grid((const void *)k_stream_copy, 256, (nvec + 255) / 256, grid_blocks);
  hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const uint4 *)src,
                     (uint4 *)dst, nvec);
  return launch_status();
}

}  // extern "C"
