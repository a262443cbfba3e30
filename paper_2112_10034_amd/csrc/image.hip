// Integral image (summed-area table) of a uint8 image, mod 2^32: the
// application of the shuffle scans that Table 1 lists (the row pass and the
// vertical pass of the CUDA scan sample).
//
// Instead of a row pass and a column pass over the whole image (13 bytes
// per pixel: 1 + 4 read, 4 + 4 written), the image is cut into tiles of
// TH rows x TW columns (band b, segment s) and reduced, carried, then
// scanned:
//   k_ii_reduce  per tile (k_ii_reduce16 with 16-pixel loads where the
//                shape allows): column sums (colsum[b][x]), row sums
//                (rowsum[s][y]) and the tile total (total[b][s]);
//   k_ii_colscan per column: colsum[b][x] replaced by its exclusive prefix
//                over the bands above, T[b][x] (8 waves per 64 columns);
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

// value of lane t ^ 32 of the wave: every lane receives the other half's
// value of the same register
__device__ __forceinline__ uint32_t ii_xor32(uint32_t v) {
  const auto pr = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return lhalf() ? (uint32_t)pr[0] : (uint32_t)pr[1];
}

// Sums of 16 values over the 64 lanes of a wave: a butterfly that halves
// the values a lane holds at every step (xor 32, 16, 8, 4), then two plain
// steps (xor 2, 1).  Returns, in every lane, the wave sum of value
// ((lane >> 2) & 15).
__device__ __forceinline__ uint32_t ii_wave_sum16(const uint32_t (&v)[16]) {
  const int L = (int)__lane_id();
  uint32_t a[8], b[4], c[2];
  const bool h32 = (L & 32) != 0, h16 = (L & 16) != 0, h8 = (L & 8) != 0, h4 = (L & 4) != 0;
#pragma unroll
  for (int i = 0; i < 8; i++) a[i] = (h32 ? v[i + 8] : v[i]) + ii_xor32(h32 ? v[i] : v[i + 8]);
#pragma unroll
  for (int i = 0; i < 4; i++) b[i] = (h16 ? a[i + 4] : a[i]) + (uint32_t)xor_lane<16>((int)(h16 ? a[i] : a[i + 4]));
#pragma unroll
  for (int i = 0; i < 2; i++) c[i] = (h8 ? b[i + 2] : b[i]) + (uint32_t)xor_lane<8>((int)(h8 ? b[i] : b[i + 2]));
  uint32_t d = (h4 ? c[1] : c[0]) + (uint32_t)xor_lane<4>((int)(h4 ? c[0] : c[1]));
  d += (uint32_t)xor_lane<2>((int)d);
  d += (uint32_t)xor_lane<1>((int)d);
  return d;
}

// Tile sums with 16-pixel loads (width a multiple of 16, image 16-byte
// aligned).  Lane c of wave g covers columns 16c .. 16c + 15 of the tile
// and rows g, g + 4, .., g + 60, so a row's sum is a wave sum; the four
// waves' column sums meet in shared memory.  Same outputs as k_ii_reduce.
__global__ __launch_bounds__(II_BT) void k_ii_reduce16(IiArgs a) {
  static_assert(II_BT == 256 && II_TW == 1024 && II_TH == 64, "4 waves x 64 lanes x 16 columns, 16 rows a wave");
  __shared__ __align__(16) uint32_t s_col[4][II_TW];
  __shared__ uint32_t s_tot[4];
  const int t = threadIdx.x, g = t >> 6, L = t & 63;
  for (int64_t tile = blockIdx.x; tile < a.nb * a.ns; tile += gridDim.x) {
    const int64_t b = tile / a.ns, s = tile % a.ns;
    const int64_t y0 = b * II_TH, x = s * II_TW + 16 * L;
    const int rows = (int)(a.H - y0 < II_TH ? a.H - y0 : II_TH);
    const bool okx = x < a.W;
    // column sums packed two to a word (even and odd bytes in 16-bit
    // halves; at most 16 * 255 each, no carry between halves), row sums by
    // v_sad_u8 against zero; rows in two batches of 8 loads
    uint32_t ev[4] = {0u, 0u, 0u, 0u}, od[4] = {0u, 0u, 0u, 0u}, rs[16];
#pragma unroll
    for (int i0 = 0; i0 < 16; i0 += 8) {
      u32x4 px[8];
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const int r = g + 4 * (i0 + i);
        px[i] = okx && r < rows ? ld_stream4(a.img + (y0 + r) * a.W + x) : u32x4{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int i = 0; i < 8; i++) {
        uint32_t sum = 0u;
#pragma unroll
        for (int w = 0; w < 4; w++) {
          const uint32_t word = px[i][w];
          ev[w] += word & 0x00ff00ffu;
          od[w] += (word >> 8) & 0x00ff00ffu;
          sum = __builtin_amdgcn_sad_u8(word, 0u, sum);
        }
        rs[i0 + i] = sum;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    uint32_t cs[16];
#pragma unroll
    for (int w = 0; w < 4; w++) {
      cs[4 * w + 0] = ev[w] & 0xffffu;
      cs[4 * w + 1] = od[w] & 0xffffu;
      cs[4 * w + 2] = ev[w] >> 16;
      cs[4 * w + 3] = od[w] >> 16;
    }
    // row g + 4 * slot of the tile, slot = (lane >> 2) & 15
    const uint32_t row_sum = ii_wave_sum16(rs);
    const int r = g + 4 * ((L >> 2) & 15);
    if ((L & 3) == 0 && r < rows) a.rowsum[s * a.H + y0 + r] = row_sum;
    // tile total: every row sum once (lanes with (L & 3) == 0), per wave
    uint32_t tv = (L & 3) == 0 && r < rows ? row_sum : 0u;
    tv = ii_warp_sum(tv);
    tv += ii_xor32(tv);
    if (L == 0) s_tot[g] = tv;
#pragma unroll
    for (int j = 0; j < 16; j += 4)
      *(u32x4 *)&s_col[g][16 * L + j] = u32x4{cs[j], cs[j + 1], cs[j + 2], cs[j + 3]};
    __syncthreads();
    {
      const int c0 = 4 * t;  // 4 columns a thread
      const int64_t xc = s * II_TW + c0;
      uint32_t out[4];
#pragma unroll
      for (int j = 0; j < 4; j++) out[j] = s_col[0][c0 + j] + s_col[1][c0 + j] + s_col[2][c0 + j] + s_col[3][c0 + j];
      if (xc < a.W) *(u32x4 *)&a.colsum[b * a.W + xc] = u32x4{out[0], out[1], out[2], out[3]};
    }
    if (t == 0) a.total[b * a.ns + s] = s_tot[0] + s_tot[1] + s_tot[2] + s_tot[3];
    __syncthreads();
  }
}

// exclusive prefix of every column's band sums.  A block takes 64
// columns (one per lane) and batches of 8 x 16 bands: wave g loads and
// sums bands g*16 .. g*16 + 15 of the batch, the 8 group sums meet in
// shared memory, and every wave writes its bands' exclusive prefixes
// (carry of the batches above + groups above + its own bands above).
constexpr int II_CS_WAVES = 8, II_CS_PB = 16;
__global__ __launch_bounds__(64 * II_CS_WAVES) void k_ii_colscan(IiArgs a) {
  __shared__ uint32_t s_grp[II_CS_WAVES][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  for (int64_t x0 = (int64_t)blockIdx.x * 64; x0 < a.W; x0 += (int64_t)gridDim.x * 64) {
    const int64_t x = x0 + lane;
    const bool okx = x < a.W;
    uint32_t carry = 0u;
    for (int64_t b0 = 0; b0 < a.nb; b0 += II_CS_WAVES * II_CS_PB) {
      const int64_t bg = b0 + (int64_t)g * II_CS_PB;
      uint32_t v[II_CS_PB], sum = 0u;
#pragma unroll
      for (int k = 0; k < II_CS_PB; k++) v[k] = okx && bg + k < a.nb ? a.colsum[(bg + k) * a.W + x] : 0u;
#pragma unroll
      for (int k = 0; k < II_CS_PB; k++) sum += v[k];
      s_grp[g][lane] = sum;
      __syncthreads();
      uint32_t off = carry, tot = 0u;
#pragma unroll
      for (int h = 0; h < II_CS_WAVES; h++) {
        const uint32_t u = s_grp[h][lane];
        off += h < g ? u : 0u;
        tot += u;
      }
#pragma unroll
      for (int k = 0; k < II_CS_PB; k++) {
        if (okx && bg + k < a.nb) a.colsum[(bg + k) * a.W + x] = off;
        off += v[k];
      }
      carry += tot;
      __syncthreads();  // s_grp is rewritten by the next batch
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
          // plain (cached) stores: the table is four times the image, and
          // for write-dominated traffic they beat non-temporal stores
          if (x < a.W) *(u32x4 *)dst = u32x4{q[r][0] + off, q[r][1] + off, q[r][2] + off, q[r][3] + off};
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
  const bool vec16 = width % 16 == 0 && ((uintptr_t)img & 15u) == 0;
  auto reduce = vec16 ? k_ii_reduce16 : vec ? k_ii_reduce<true> : k_ii_reduce<false>;
  auto scan = vec ? k_ii_scan<true> : k_ii_scan<false>;
  hipStream_t hs = (hipStream_t)stream;
  const int64_t tiles = a.nb * a.ns;
  const int g1 = persistent_grid((const void *)reduce, II_BT, tiles, 0, 0, 8);
  hipLaunchKernelGGL(reduce, dim3(g1), dim3(II_BT), 0, hs, a);
  const int64_t gc = (width + 63) / 64;
  hipLaunchKernelGGL(k_ii_colscan, dim3((unsigned)(gc < 65536 ? gc : 65536)), dim3(64 * II_CS_WAVES), 0, hs, a);
  const int g3 = persistent_grid((const void *)scan, II_BT, tiles, 0, 0, 8);
  hipLaunchKernelGGL(scan, dim3(g3), dim3(II_BT), 0, hs, a);
  return launch_status();
}
