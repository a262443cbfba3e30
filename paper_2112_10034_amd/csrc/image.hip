// Integral image (summed-area table) of a uint8 image, mod 2^32: the
// application of the shuffle scans that Table 1 lists (the row pass and the
// vertical pass of the CUDA scan sample).
//
// Instead of a row pass and a column pass over the whole image (13 bytes
// per pixel: 1 + 4 read, 4 + 4 written), the image is cut into tiles of
// TH rows x TW columns (band b, segment s) and reduced, carried, then
// scanned:
//   k_ii_reduce  per tile: column sums (colsum[b][x]), row sums
//                (rowsum[s][y]) and the tile total (total[b][s]);
//   k_ii_colscan per column: colsum[b][x] replaced by its exclusive prefix
//                over the bands above, T[b][x];
//   k_ii_scan    per tile: sat[y][x] = rowprefix_x(T[b][.] + column sums
//                of rows y0..y)[x] + corner + sum of L over rows y0..y,
//                with L[y] the row sums of the segments to the left and
//                corner the totals of the tiles above and to the left.
// Every row of a tile is an inclusive scan over TW columns: lane-serial
// over a thread's 4 columns, a 32-lane shuffle scan (DPP row shifts), and
// the warp totals combined in shared memory.  About 6.1 bytes per pixel
// move (the image is read twice), all in uint32 arithmetic, so the result
// is exact (mod 2^32) whatever the order.
#include "cox_internal.hpp"

namespace cox {

constexpr int II_TH = 64;     // rows per tile
constexpr int II_TW = 1024;   // columns per tile
constexpr int II_BT = 256;    // threads per block, 4 columns each
constexpr int II_RB = 8;      // rows per round of the reduce kernel (its butterfly sums 8)
constexpr int II_RS = 4;      // rows per shared-memory round of the scan kernel (measured: 4 rows
                              // 93 us, 8 rows 99 us, 16 rows 106 us at 8192 x 8192)
// wave 0 (64 threads) handles the tile's rows: one row per thread, two
// logical warps
static_assert(II_TH == 64 && II_BT >= 64 && II_TW == 4 * II_BT, "tile shape the kernels assume");

// inclusive scan over the 32 lanes of a logical warp
__device__ __forceinline__ uint32_t ii_warp_scan(uint32_t v) {
  v += (uint32_t)dpp<DPP_ROW_SHR1>(0, (int)v);
  v += (uint32_t)dpp<DPP_ROW_SHR2>(0, (int)v);
  v += (uint32_t)dpp<DPP_ROW_SHR4>(0, (int)v);
  v += (uint32_t)dpp<DPP_ROW_SHR8>(0, (int)v);
  v += (uint32_t)dpp<DPP_ROW_BCAST15, 0xa>(0, (int)v);
  return v;
}

__device__ __forceinline__ uint32_t ii_warp_sum(uint32_t v) {
  v += (uint32_t)xor_lane<16>((int)v);
  v += (uint32_t)xor_lane<8>((int)v);
  v += (uint32_t)xor_lane<4>((int)v);
  v += (uint32_t)xor_lane<2>((int)v);
  v += (uint32_t)xor_lane<1>((int)v);
  return v;
}

struct IiArgs {
  const uint8_t *img;
  uint32_t *sat;
  int64_t H, W;
  int64_t nb, ns;     // bands, segments
  uint32_t *colsum;   // [nb][W]: column sums, then their exclusive prefix T
  uint32_t *rowsum;   // [ns][H]
  uint32_t *total;    // [nb][ns]
};

// The 4 pixels of a thread in row y (columns x .. x + 3; zero past W, and
// zero for rows past the tile).  VEC (W % 4 == 0, image 4-byte aligned):
// one 4-byte load.
template <bool VEC>
__device__ __forceinline__ void ii_pixels(const IiArgs &a, int64_t y, bool row_ok, int64_t x, uint32_t (&p)[4]) {
  const uint8_t *row = a.img + y * a.W;
  if constexpr (VEC) {
    const uint32_t w = row_ok && x < a.W ? ld_stream1(row + x) : 0u;
#pragma unroll
    for (int j = 0; j < 4; j++) p[j] = (w >> (8 * j)) & 0xffu;
  } else {
#pragma unroll
    for (int j = 0; j < 4; j++) p[j] = row_ok && x + j < a.W ? (uint32_t)row[x + j] : 0u;
  }
}

// Sums of 8 values over a logical warp, one value per row: a butterfly
// that halves the values a lane holds at every step (xor 16, 8, 4), then
// two plain steps (xor 2, 1).  Returns, in every lane, the warp sum of
// value ((lane >> 2) & 7).
__device__ __forceinline__ uint32_t ii_warp_sum8(const uint32_t (&v)[8]) {
  const int l = llane();
  uint32_t a[4], b[2];
  const bool h16 = (l & 16) != 0, h8 = (l & 8) != 0, h4 = (l & 4) != 0;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const uint32_t send = h16 ? v[i] : v[i + 4];
    a[i] = (h16 ? v[i + 4] : v[i]) + (uint32_t)xor_lane<16>((int)send);
  }
#pragma unroll
  for (int i = 0; i < 2; i++) {
    const uint32_t send = h8 ? a[i] : a[i + 2];
    b[i] = (h8 ? a[i + 2] : a[i]) + (uint32_t)xor_lane<8>((int)send);
  }
  uint32_t c = (h4 ? b[1] : b[0]) + (uint32_t)xor_lane<4>((int)(h4 ? b[0] : b[1]));
  c += (uint32_t)xor_lane<2>((int)c);
  c += (uint32_t)xor_lane<1>((int)c);
  return c;
}

template <bool VEC>
__global__ __launch_bounds__(II_BT) void k_ii_reduce(IiArgs a) {
  static_assert(II_RB == 8, "row sums are reduced 8 rows at a time");
  __shared__ uint32_t s_rows[II_BT / 32][II_TH];
  __shared__ uint32_t s_tot[2];
  const int t = threadIdx.x, w = t >> 5, l = t & 31;
  for (int64_t tile = blockIdx.x; tile < a.nb * a.ns; tile += gridDim.x) {
    const int64_t b = tile / a.ns, s = tile % a.ns;
    const int64_t y0 = b * II_TH, x = s * II_TW + 4 * t;
    const int rows = (int)(a.H - y0 < II_TH ? a.H - y0 : II_TH);
    uint32_t cs[4] = {0u, 0u, 0u, 0u};
    for (int r0 = 0; r0 < rows; r0 += II_RB) {
      uint32_t p[II_RB][4];
#pragma unroll
      for (int r = 0; r < II_RB; r++) ii_pixels<VEC>(a, y0 + r0 + r, r0 + r < rows, x, p[r]);
      uint32_t rp[II_RB];
#pragma unroll
      for (int r = 0; r < II_RB; r++) {
        cs[0] += p[r][0];
        cs[1] += p[r][1];
        cs[2] += p[r][2];
        cs[3] += p[r][3];
        rp[r] = p[r][0] + p[r][1] + p[r][2] + p[r][3];
      }
      const uint32_t rs = ii_warp_sum8(rp);
      const int r = (l >> 2) & 7;
      if ((l & 3) == 0 && r0 + r < rows) s_rows[w][r0 + r] = rs;
    }
#pragma unroll
    for (int j = 0; j < 4; j++)
      if (x + j < a.W) a.colsum[b * a.W + x + j] = cs[j];
    __syncthreads();
    if (t < II_TH) {
      uint32_t v = 0u;
#pragma unroll
      for (int k = 0; k < II_BT / 32; k++) v += s_rows[k][t];
      if (t < rows) a.rowsum[s * a.H + y0 + t] = v;
      // tile total: the first two warps (all of wave 0) sum the row sums
      const uint32_t tot = ii_warp_sum(t < rows ? v : 0u);
      if (l == 0) s_tot[w] = tot;
    }
    __syncthreads();
    if (t == 0) a.total[b * a.ns + s] = s_tot[0] + s_tot[1];
    __syncthreads();
  }
}

// exclusive prefix of every column's band sums, 64 bands per batch of loads
__global__ __launch_bounds__(256) void k_ii_colscan(IiArgs a) {
  constexpr int NB = 64;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < a.W; x += (int64_t)gridDim.x * blockDim.x) {
    uint32_t run = 0u;
    for (int64_t b0 = 0; b0 < a.nb; b0 += NB) {
      uint32_t v[NB];
#pragma unroll
      for (int k = 0; k < NB; k++) v[k] = b0 + k < a.nb ? a.colsum[(b0 + k) * a.W + x] : 0u;
#pragma unroll
      for (int k = 0; k < NB; k++) {
        if (b0 + k < a.nb) a.colsum[(b0 + k) * a.W + x] = run;
        run += v[k];
      }
    }
  }
}

template <bool VEC>
__global__ __launch_bounds__(II_BT) void k_ii_scan(IiArgs a) {
  __shared__ uint32_t s_lin[II_TH];             // row carries, prefixed inside each 32-row half
  __shared__ uint32_t s_left[II_TH];            // corner + row carries, prefixed over the tile's rows
  __shared__ uint32_t s_wt[2][II_RS][II_BT / 32];  // warp totals of a round of rows
  __shared__ uint32_t s_red[II_BT / 32];
  const int t = threadIdx.x, w = t >> 5, l = t & 31;
  int buf = 0;
  for (int64_t tile = blockIdx.x; tile < a.nb * a.ns; tile += gridDim.x) {
    const int64_t b = tile / a.ns, s = tile % a.ns;
    const int64_t y0 = b * II_TH, x = s * II_TW + 4 * t;
    const int rows = (int)(a.H - y0 < II_TH ? a.H - y0 : II_TH);
    // corner: totals of the tiles above and to the left
    uint32_t cv = 0u;
    for (int64_t k = t; k < b * s; k += II_BT) cv += a.total[(k / s) * a.ns + (k % s)];
    cv = ii_warp_sum(cv);
    if (l == 0) s_red[w] = cv;
    // row carries (thread t < TH: row y0 + t): row sums of the segments to
    // the left, then an inclusive scan inside each 32-row half
    uint32_t lv = 0u;
    if (t < rows && t < II_TH)
      for (int64_t k = 0; k < s; k++) lv += a.rowsum[k * a.H + y0 + t];
    lv = ii_warp_scan(lv);
    if (t < II_TH) s_lin[t] = lv;
    // column carries: the band sums above
    uint32_t c[4];
#pragma unroll
    for (int j = 0; j < 4; j++) c[j] = x + j < a.W ? a.colsum[b * a.W + x + j] : 0u;
    __syncthreads();
    if (t < II_TH) {
      uint32_t corner = 0u;
#pragma unroll
      for (int k = 0; k < II_BT / 32; k++) corner += s_red[k];
      s_left[t] = corner + s_lin[t] + (t >= 32 ? s_lin[31] : 0u);
    }
    __syncthreads();
    // rounds of II_RS rows; the next round's pixels are requested before
    // the current round's barrier and stores
    uint32_t pn[II_RS][4];
#pragma unroll
    for (int r = 0; r < II_RS; r++) ii_pixels<VEC>(a, y0 + r, r < rows, x, pn[r]);
    for (int r0 = 0; r0 < rows; r0 += II_RS) {
      uint32_t q[II_RS][4];
#pragma unroll
      for (int r = 0; r < II_RS; r++) {
#pragma unroll
        for (int j = 0; j < 4; j++) c[j] += pn[r][j];
        q[r][0] = c[0];
        q[r][1] = q[r][0] + c[1];
        q[r][2] = q[r][1] + c[2];
        q[r][3] = q[r][2] + c[3];
        const uint32_t incl = ii_warp_scan(q[r][3]);
        const uint32_t excl = incl - q[r][3];
#pragma unroll
        for (int j = 0; j < 4; j++) q[r][j] += excl;
        if (l == 31) s_wt[buf][r][w] = incl;
      }
#pragma unroll
      for (int r = 0; r < II_RS; r++) {
        const int rr = r0 + II_RS + r;
        ii_pixels<VEC>(a, y0 + rr, rr < rows, x, pn[r]);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < II_RS; r++) {
        if (r0 + r >= rows) break;
        uint32_t off = s_left[r0 + r];
#pragma unroll
        for (int k = 0; k < II_BT / 32; k++) off += k < w ? s_wt[buf][r][k] : 0u;
        const int64_t y = y0 + r0 + r;
        uint32_t *dst = a.sat + y * a.W + x;
        if constexpr (VEC) {
          if (x < a.W) st_stream4(dst, q[r][0] + off, q[r][1] + off, q[r][2] + off, q[r][3] + off);
        } else {
#pragma unroll
          for (int j = 0; j < 4; j++)
            if (x + j < a.W) dst[j] = q[r][j] + off;
        }
      }
      buf ^= 1;
    }
    __syncthreads();
  }
}

}  // namespace cox

namespace cox {

struct IiLayout {
  size_t colsum, rowsum, total, bytes;
};

static IiLayout ii_layout(int64_t H, int64_t W) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const int64_t nb = (H + II_TH - 1) / II_TH, ns = (W + II_TW - 1) / II_TW;
  IiLayout L;
  L.colsum = WS_HEADER;
  L.rowsum = L.colsum + up((size_t)nb * W * 4);
  L.total = L.rowsum + up((size_t)ns * H * 4);
  L.bytes = L.total + up((size_t)nb * ns * 4);
  return L;
}

size_t ii_workspace_bytes(int64_t H, int64_t W) { return ii_layout(H, W).bytes; }

}  // namespace cox

using namespace cox;

extern "C" cox_status cox_integral_image(const uint8_t *img, int64_t height, int64_t width, uint32_t *sat, void *ws,
                                         size_t ws_bytes, void *stream) {
  if (height < 0 || width < 0) return COX_ERR_INVALID;
  if (height == 0 || width == 0) return COX_OK;
  if (!img || !sat) return COX_ERR_INVALID;
  const IiLayout L = ii_layout(height, width);
  if (!ws || ws_bytes < L.bytes) return COX_ERR_WORKSPACE;
  char *w = (char *)ws;
  IiArgs a;
  a.img = img;
  a.sat = sat;
  a.H = height;
  a.W = width;
  a.nb = (height + II_TH - 1) / II_TH;
  a.ns = (width + II_TW - 1) / II_TW;
  a.colsum = (uint32_t *)(w + L.colsum);
  a.rowsum = (uint32_t *)(w + L.rowsum);
  a.total = (uint32_t *)(w + L.total);
  const bool vec = width % 4 == 0 && ((uintptr_t)img & 3u) == 0 && aligned16(sat);
  auto reduce = vec ? k_ii_reduce<true> : k_ii_reduce<false>;
  auto scan = vec ? k_ii_scan<true> : k_ii_scan<false>;
  hipStream_t hs = (hipStream_t)stream;
  const int64_t tiles = a.nb * a.ns;
  const int g1 = persistent_grid((const void *)reduce, II_BT, tiles, 0, 0, 8);
  hipLaunchKernelGGL(reduce, dim3(g1), dim3(II_BT), 0, hs, a);
  const int64_t gc = (width + 255) / 256;
  hipLaunchKernelGGL(k_ii_colscan, dim3((unsigned)(gc < 65536 ? gc : 65536)), dim3(256), 0, hs, a);
  const int g3 = persistent_grid((const void *)scan, II_BT, tiles, 0, 0, 8);
  hipLaunchKernelGGL(scan, dim3(g3), dim3(II_BT), 0, hs, a);
  return launch_status();
}
