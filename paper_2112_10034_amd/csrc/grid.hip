// Grid-wide barrier (cooperative groups' this_grid().sync(), Sec. 2.2.2) on
// a cooperative launch, and two kernels built on it: an exchange kernel
// that checks and times the barrier, and a conjugate-gradient solver whose
// whole iteration loop runs in one launch -- the CG sample that Table 1
// lists among the kernels COX could not run because of grid
// synchronisation (Sec. 5.1).
//
// Memory protocol.  The per-XCD L2 caches of MI355X are not coherent with
// each other for ordinary stores; an agent-scope release / acquire pair
// makes them so by writing back and invalidating a whole L2, and with one
// such pair per block a barrier costs 10 us at 256 blocks.  Here every
// value that one block writes and another reads during a launch moves with
// device-coherent (sc1) loads and stores instead -- the accesses of relaxed
// agent-scope atomics, which bypass the non-coherent cached copies -- and
// the barrier needs no cache maintenance: every wave waits for its own
// stores to complete (s_waitcnt vmcnt(0)) before the block arrives, and
// every read after the barrier is issued after the generation change was
// seen.  Values a thread writes and later reads itself use ordinary
// accesses.
//
// Barrier.  Blocks arrive in eight groups (block b in group b mod 8), so no
// counter takes more than ceil(G / 8) of the atomics that serialise at one
// address; the last arrival of a group counts the group at the top, and the
// last group advances the generation the other blocks poll.  The waits are
// bounded: one that runs out sets an abort word that every other wait also
// obeys, so all blocks leave within one more timeout, and the call reports
// COX_ERR_TIMEOUT through the workspace.
//
// CG (Hestenes and Stiefel; binary32 vectors, binary64 scalars, the
// schedule of every inner product fixed by (R, W), see cox.h).  Two grid
// barriers per iteration.  Phase 1 fuses p = r + beta p into the sparse
// product: the block forms p over its rows and a halo of HALO rows on each
// side in shared memory (from the previous p and r, with the same fmaf as
// the stored p, so the same bits), stores its own rows' p (double-buffered
// by iteration parity), and gathers from shared memory (columns outside the
// window form p_j from global memory).  Phase 2 updates x and r with the
// <r, r> partials.  Every block combines the chunk partials itself in the
// fixed final order, so all blocks take the same decisions without a
// broadcast.  Chunk c belongs to block c mod G in every phase, so results do
// not depend on G.  When every block holds at most one chunk, x, r, p and q
// of the block's rows stay in registers for the whole solve and only r and
// p (for the other blocks' gathers) and the partials are stored.
#include <algorithm>

#include "cox_internal.hpp"

namespace cox {

// ---------------------------------------------------------------- barrier
// Barrier words (uint32, one 128-byte line each), after the workspace
// header: line g < 8 arrivals of group g, line 8 groups complete, line 9
// generation, line 10 abort.
enum : int { GB_LINE = 32, GB_GROUPS = 8, GB_TOP = 8 * 32, GB_GEN = 9 * 32, GB_ABORT = 10 * 32, GB_WORDS = 11 * 32 };
constexpr size_t GB_BYTES = 2048;  // GB_WORDS * 4 rounded up
constexpr uint32_t GRID_MAX_SPIN = 1u << 20;

// device-coherent accesses
__device__ __forceinline__ uint32_t ldc32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ldcf(const float *p) { return i2f((int)ldc32((const uint32_t *)p)); }
__device__ __forceinline__ void stcf(float *p, float v) { stc32((uint32_t *)p, (uint32_t)f2i(v)); }
__device__ __forceinline__ double ldcd(const double *p) {
  return __builtin_bit_cast(double, __hip_atomic_load((const uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void stcd(double *p, double v) {
  __hip_atomic_store((uint64_t *)p, __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Every block of the (co-resident) grid calls this with every thread; the
// device-coherent writes of all blocks before it are visible to the
// device-coherent reads of all blocks after it.  false: the wait gave up,
// and the kernel should finish without further barriers.
__device__ bool grid_sync(uint32_t *bar, uint32_t *hdr, uint32_t spin_limit = GRID_MAX_SPIN) {
  __shared__ uint32_t s_ok;
  wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ok = 1u;
    const uint32_t G = gridDim.x;
    const uint32_t ng = G < GB_GROUPS ? G : GB_GROUPS;
    const uint32_t g = blockIdx.x % ng;
    const uint32_t members = (G - g + ng - 1) / ng;
    // read before arriving: the generation cannot advance without us
    const uint32_t gen = ldc32(&bar[GB_GEN]);
    bool released = false;
    if (__hip_atomic_fetch_add(&bar[g * GB_LINE], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == members - 1) {
      // the resets land before the generation advances, so no arrival at
      // the next barrier can precede them
      stc32(&bar[g * GB_LINE], 0u);
      wait_stores();
      if (__hip_atomic_fetch_add(&bar[GB_TOP], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ng - 1) {
        stc32(&bar[GB_TOP], 0u);
        wait_stores();
        stc32(&bar[GB_GEN], gen + 1u);
        released = true;
      }
    }
    if (!released) {
      uint32_t spins = 0;
      while (ldc32(&bar[GB_GEN]) == gen) {
        if (ldc32(&bar[GB_ABORT]) != 0u || ++spins > spin_limit) {
          stc32(&bar[GB_ABORT], 1u);
          stc32(&hdr[HDR_ERR], 1u);
          ok = 0u;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0u;
}

__global__ void k_grid_clear(uint32_t *bar, int words) {
  for (int i = threadIdx.x; i < words; i += blockDim.x) bar[i] = 0u;
}

// ---------------------------------------------------------------- exchange
// MurmurHash3's 32-bit finaliser (Appleby), the payload of the exchange
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

constexpr int GX_BLOCK = 1024;

// round r: write own row, barrier, add the row of block (b + r + 1) mod G,
// barrier.  Failure-handling check: block `absent` (-1: none) leaves before
// the first barrier, so the other blocks' waits give up after spin_limit
// polls and every block finishes.
__global__ __launch_bounds__(GX_BLOCK) void k_grid_exchange(uint32_t *slot, uint32_t *out, int rounds, uint32_t *bar,
                                                            uint32_t *hdr, int absent, uint32_t spin_limit) {
  const uint32_t G = gridDim.x, b = blockIdx.x, t = threadIdx.x;
  uint32_t sum = 0u;
  for (int r = 0; r < rounds; r++) {
    stc32(&slot[(size_t)b * GX_BLOCK + t], fmix32(((uint32_t)r << 20) ^ (b << 10) ^ t));
    if ((int)b == absent) break;
    if (!grid_sync(bar, hdr, spin_limit)) break;
    const uint32_t src = (uint32_t)(((uint64_t)b + (uint64_t)r + 1u) % G);
    sum += ldc32(&slot[(size_t)src * GX_BLOCK + t]);
    if (!grid_sync(bar, hdr, spin_limit)) break;
  }
  out[(size_t)b * GX_BLOCK + t] = sum;
}

// ---------------------------------------------------------------- CG
constexpr int HALO = 64;  // rows of the shared-memory window beyond the chunk on each side

struct CgState {
  uint32_t stop;
  uint32_t far;  // resident kernel: some block gathers outside its window or streams its rows
  double rr[2];  // rr_k at slot k & 1 (per-phase launches)
};

struct CgArgs {
  const int32_t *rp, *ci;
  const float *val, *b;
  float *x, *r, *p[2], *q;
  double *prr, *ppq;  // chunk partials of <r, r> and <p, A p>
  int64_t nch;
  int32_t n, nnz;
  int32_t max_iter;
  double tol2;
  int32_t *result;
  double *rr_hist;
  uint32_t *bar, *hdr;
  CgState *state;
  uint32_t lds_bytes;  // dynamic shared memory of the resident kernel (0: CSR never staged)
};

// shared memory of one block
template <int R, int W>
struct CgShared {
  double slot[32];
  double fin[256];
  double bcast;
  uint32_t elo, ehi;  // entry range of the chunk's rows (CSR staging)
  float win[32 * W * R + 2 * HALO];
};

// xor butterfly over a logical warp: every lane ends with the value lane 0
// of the shfl_down tree (offsets 16 .. 1) holds
__device__ __forceinline__ double tree64(double v) {
  v = v + xor_lane_d<16>(v);
  v = v + xor_lane_d<8>(v);
  v = v + xor_lane_d<4>(v);
  v = v + xor_lane_d<2>(v);
  v = v + xor_lane_d<1>(v);
  return v;
}

// chunk value of a per-thread FP64 sum: warp trees, then warp 0's tree over
// the W warp values (-0.0 beyond W); thread 0 stores it.  Ends with a block
// barrier, so the shared window may be reused after it.
template <int W, class SH>
__device__ __forceinline__ void chunk_store(double s, double *part, int64_t c, SH &sh) {
  const int t = threadIdx.x, l = t & 31;
  s = tree64(s);
  if (l == 0) sh.slot[t >> 5] = s;
  __syncthreads();
  if (t < 32) {
    const double v = tree64(l < W ? sh.slot[l] : -0.0);
    if (t == 0) stcd(&part[c], v);
  }
  __syncthreads();
}

// final combine of nch chunk values, computed by every block: thread j <
// 256 sums values j, j + 256, ... from -0.0 (a batch padded with -0.0 adds
// nothing); each group of 32 runs the tree; the tree again over the 8
// group values (-0.0 beyond 8)
template <class SH>
__device__ __forceinline__ double final64(const double *part, int64_t nch, SH &sh) {
  constexpr int FB = 8;
  const int t = threadIdx.x, l = t & 31;
  if (t < 256) {
    double s = -0.0;
    for (int64_t c0 = t; c0 < nch; c0 += 256 * FB) {
      double v[FB];
#pragma unroll
      for (int u = 0; u < FB; u++) v[u] = c0 + 256 * u < nch ? ldcd(&part[c0 + 256 * u]) : -0.0;
#pragma unroll
      for (int u = 0; u < FB; u++) s = s + v[u];
    }
    sh.fin[t] = s;
  }
  __syncthreads();
  if (t < 32) {
    double top = -0.0;
#pragma unroll
    for (int vw = 0; vw < 8; vw++) {
      const double v = tree64(sh.fin[32 * vw + l]);
      if (l == vw) top = v;
    }
    top = tree64(top);
    if (t == 0) sh.bcast = top;
  }
  __syncthreads();
  return sh.bcast;
}

// row bounds, clamped so that malformed CSR cannot read outside the arrays
__device__ __forceinline__ void row_bounds(const CgArgs &a, int32_t i, int32_t &lo, int32_t &hi) {
  int32_t u = a.rp[i], v = a.rp[i + 1];
  u = u < 0 ? 0 : (u > a.nnz ? a.nnz : u);
  v = v < u ? u : (v > a.nnz ? a.nnz : v);
  lo = u;
  hi = v;
}
__device__ __forceinline__ uint32_t col_at(const CgArgs &a, int32_t jj) {
  const uint32_t j = (uint32_t)a.ci[jj];
  return j < (uint32_t)a.n ? j : (uint32_t)a.n - 1u;
}

// (A v)_i for the R rows of a thread, each row accumulating its entries
// in storage order from +0.0f with fmaf.  The CSR work is fetched ahead:
// fetch_bounds requests the rows' bounds, fetch_entries the next SU
// entries of every row at once (so a row of up to SU entries costs one
// round trip, and callers issue both before unrelated loads and barriers),
// and spmv_finish consumes them, gathering v_j through vj.
// SU entries per row and fetch, as deep as registers allow without spills:
// 4 (2 for R = 8) in the streaming kernels, 2 (1 for R = 8) in the kernel
// that keeps x, r, p and q resident
template <int R>
constexpr int su_stream() {
  return R >= 8 ? 2 : 4;
}
template <int R>
constexpr int su_resident() {
  return R >= 8 ? 1 : 2;
}
template <int R, int SU>
struct RowFetch {
  int32_t lo[R], hi[R], len;
  uint32_t j[SU][R];
  float v[SU][R];
};

template <int R, int SU>
__device__ __forceinline__ void fetch_bounds(const CgArgs &a, const int32_t (&row)[R], RowFetch<R, SU> &f) {
  f.len = 0;
#pragma unroll
  for (int q = 0; q < R; q++) {
    if (row[q] < a.n) {
      row_bounds(a, row[q], f.lo[q], f.hi[q]);
    } else {
      f.lo[q] = 0;
      f.hi[q] = 0;
    }
    f.len = max(f.len, f.hi[q] - f.lo[q]);
  }
}

template <int R, int SU>
__device__ __forceinline__ void fetch_entries(const CgArgs &a, int32_t s0, RowFetch<R, SU> &f) {
#pragma unroll
  for (int u = 0; u < SU; u++)
#pragma unroll
    for (int q = 0; q < R; q++) {
      const int32_t k = f.lo[q] + s0 + u;
      const bool ok = k < f.hi[q];
      f.j[u][q] = ok ? col_at(a, k) : 0u;
      f.v[u][q] = ok ? a.val[k] : 0.0f;
    }
}

template <int R, int SU, class V>
__device__ __forceinline__ void spmv_finish(const CgArgs &a, RowFetch<R, SU> &f, float (&acc)[R], V vj) {
#pragma unroll
  for (int q = 0; q < R; q++) acc[q] = 0.0f;
  for (int32_t s0 = 0; s0 < f.len; s0 += SU) {
    if (s0) fetch_entries(a, s0, f);
    float g[SU][R];
#pragma unroll
    for (int u = 0; u < SU; u++)
#pragma unroll
      for (int q = 0; q < R; q++) g[u][q] = f.lo[q] + s0 + u < f.hi[q] ? vj(f.j[u][q]) : 0.0f;
#pragma unroll
    for (int u = 0; u < SU; u++)
#pragma unroll
      for (int q = 0; q < R; q++)
        if (f.lo[q] + s0 + u < f.hi[q]) acc[q] = __builtin_fmaf(f.v[u][q], g[u][q], acc[q]);
  }
}

template <int R, int W>
__device__ __forceinline__ void rows_of(int64_t c, int32_t (&row)[R]) {
  constexpr int BT = 32 * W;
#pragma unroll
  for (int q = 0; q < R; q++) row[q] = (int32_t)(c * (BT * R) + BT * q + threadIdx.x);
}

// p = r (first) or fmaf(beta, p_prev, r) over chunk c's rows and the halo,
// into sh.win (w0 = first row of the window); ends with a block barrier
template <int R, int W, class SH>
__device__ __forceinline__ int32_t cg_window(const CgArgs &a, int64_t c, bool first, float beta, const float *pp,
                                             SH &sh, int32_t &wn) {
  constexpr int BT = 32 * W, S = BT * R;
  static_assert(2 * HALO <= BT, "window loop covers S + 2 HALO rows in R + 1 steps");
  const int64_t lo = c * S;
  const int32_t w0 = (int32_t)(lo > HALO ? lo - HALO : 0);
  const int32_t w1 = (int32_t)(lo + S + HALO < a.n ? lo + S + HALO : a.n);
  float rv[R + 1], pv[R + 1];
#pragma unroll
  for (int m = 0; m <= R; m++) {
    const int32_t j = w0 + BT * m + (int32_t)threadIdx.x;
    const bool ok = j < w1;
    rv[m] = ok ? ldcf(a.r + j) : 0.0f;
    pv[m] = ok && !first ? ldcf(pp + j) : 0.0f;
  }
#pragma unroll
  for (int m = 0; m <= R; m++) {
    const int32_t j = w0 + BT * m + (int32_t)threadIdx.x;
    if (j < w1) sh.win[j - w0] = first ? rv[m] : __builtin_fmaf(beta, pv[m], rv[m]);
  }
  __syncthreads();
  wn = w1 - w0;
  return w0;
}

// r = b - A x, partials of <r, r>; the resident form keeps x and r
template <int R, int W, int SU, class SH>
__device__ __forceinline__ void cg_phase0_chunk(const CgArgs &a, int64_t c, SH &sh, float (&xv)[R], float (&rv)[R]) {
  int32_t row[R];
  float ax[R];
  rows_of<R, W>(c, row);
  RowFetch<R, SU> f;
  fetch_bounds(a, row, f);
  fetch_entries(a, 0, f);
  spmv_finish(a, f, ax, [&](uint32_t j) { return a.x[j]; });
  double s = -0.0;
#pragma unroll
  for (int q = 0; q < R; q++) {
    xv[q] = 0.0f;
    rv[q] = 0.0f;
    if (row[q] < a.n) {
      xv[q] = a.x[row[q]];
      rv[q] = a.b[row[q]] - ax[q];
      stcf(a.r + row[q], rv[q]);
      s = s + (double)rv[q] * (double)rv[q];
    }
  }
  chunk_store<W>(s, a.prr, c, sh);
}

// rows of chunk c that other chunks' windows read: the first and last HALO
__device__ __forceinline__ bool halo_row(int64_t c, int32_t row, int S) {
  const int64_t o = (int64_t)row - c * S;
  return o < HALO || o >= S - HALO;
}

// p of the chunk's rows from the window into p[k & 1], partials of <p, q>
template <int R, int W, class SH>
__device__ __forceinline__ void cg_phase1_tail(const CgArgs &a, int64_t c, const int32_t (&row)[R], int32_t w0,
                                               float *pn, SH &sh, float (&pv)[R], const float (&qv)[R],
                                               bool near = false) {
  double s = -0.0;
#pragma unroll
  for (int q = 0; q < R; q++) {
    pv[q] = 0.0f;
    if (row[q] < a.n) {
      pv[q] = sh.win[row[q] - w0];
      if (!near || halo_row(c, row[q], 32 * W * R)) stcf(pn + row[q], pv[q]);
      s = s + (double)pv[q] * (double)qv[q];
    }
  }
  chunk_store<W>(s, a.ppq, c, sh);
}

// p (into p[k & 1]) and q = A p, partials of <p, q>
template <int R, int W, int SU, class SH>
__device__ __forceinline__ void cg_phase1_chunk(const CgArgs &a, int64_t c, int k, float beta, SH &sh, float (&pv)[R],
                                                float (&qv)[R]) {
  const bool first = k == 0;
  const float *pp = a.p[(k + 1) & 1];
  float *pn = a.p[k & 1];
  // the rows' CSR bounds and first entries are requested before the
  // window's loads and barrier
  int32_t row[R];
  rows_of<R, W>(c, row);
  RowFetch<R, SU> f;
  fetch_bounds(a, row, f);
  fetch_entries(a, 0, f);
  int32_t wn;
  const int32_t w0 = cg_window<R, W>(a, c, first, beta, pp, sh, wn);
  spmv_finish(a, f, qv, [&](uint32_t j) {
    const uint32_t o = j - (uint32_t)w0;
    if (o < (uint32_t)wn) return sh.win[o];
    const float rj = ldcf(a.r + j);
    return first ? rj : __builtin_fmaf(beta, ldcf(pp + j), rj);
  });
  cg_phase1_tail<R, W>(a, c, row, w0, pn, sh, pv, qv);
}

// The resident kernel keeps its chunk's CSR rows in shared memory when they
// fit in the launch's dynamic allocation: per row its clamped entry range
// relative to the chunk's first entry (two 16-bit offsets), then the
// (column, value) pairs with columns clamped as col_at does.  Decided per
// block (uniformly); the staged values, and the order in which the SpMV
// accumulates them, are those the streaming form reads.  Returns 0 (not
// staged), 1 (staged; some column lies outside the chunk's window of
// HALO rows on each side) or 2 (staged; every column inside the window).
template <int R, int W, class SH>
__device__ int cg_stage(const CgArgs &a, int64_t c, uint8_t *dyn, SH &sh) {
  constexpr int BT = 32 * W, S = BT * R;
  if (a.lds_bytes < (uint32_t)S * 4u) return 0;
  int32_t row[R], lo[R], hi[R];
  rows_of<R, W>(c, row);
  if (threadIdx.x == 0) {
    sh.elo = 0xffffffffu;
    sh.ehi = 0u;
  }
  __syncthreads();
  uint32_t mlo = 0xffffffffu, mhi = 0u;
#pragma unroll
  for (int q = 0; q < R; q++) {
    lo[q] = hi[q] = 0;
    if (row[q] < a.n) {
      row_bounds(a, row[q], lo[q], hi[q]);
      mlo = min(mlo, (uint32_t)lo[q]);
      mhi = max(mhi, (uint32_t)hi[q]);
    }
  }
  if (mlo != 0xffffffffu) {
    atomicMin(&sh.elo, mlo);
    atomicMax(&sh.ehi, mhi);
  }
  __syncthreads();
  const uint32_t e0 = sh.elo, e1 = sh.ehi;
  const uint32_t E = e1 > e0 ? e1 - e0 : 0u;
  if (E > 0xffffu || (uint64_t)S * 4u + (uint64_t)E * 8u > a.lds_bytes) return 0;
  uint32_t *bnd = (uint32_t *)dyn;
  uint2 *ent = (uint2 *)(dyn + S * 4);
#pragma unroll
  for (int q = 0; q < R; q++)
    bnd[BT * q + threadIdx.x] = row[q] < a.n ? ((uint32_t)lo[q] - e0) | (((uint32_t)hi[q] - e0) << 16) : 0u;
  const int64_t cs = c * S;
  const uint32_t w0 = (uint32_t)(cs > HALO ? cs - HALO : 0);
  const uint32_t wn = (uint32_t)(cs + S + HALO < a.n ? cs + S + HALO : a.n) - w0;
  int outside = 0;
  for (uint32_t e = threadIdx.x; e < E; e += BT) {
    const uint32_t j = col_at(a, (int32_t)(e0 + e));
    outside |= j - w0 >= wn;
    ent[e] = make_uint2(j, __float_as_uint(a.val[e0 + e]));
  }
  return __syncthreads_or(outside) ? 1 : 2;
}

// p over chunk c's window when no block reads outside its window: the
// chunk's own rows from the registers (p_prev, r), the HALO rows on each
// side from the neighbours' stores; ends with a block barrier
template <int R, int W, class SH>
__device__ __forceinline__ int32_t cg_window_near(const CgArgs &a, int64_t c, bool first, float beta, const float *pp,
                                                  const float (&pv)[R], const float (&rv)[R], SH &sh, int32_t &wn) {
  constexpr int BT = 32 * W, S = BT * R;
  const int64_t lo = c * S;
  const int32_t w0 = (int32_t)(lo > HALO ? lo - HALO : 0);
  const int32_t w1 = (int32_t)(lo + S + HALO < a.n ? lo + S + HALO : a.n);
  const int t = threadIdx.x;
  if (t < 2 * HALO) {
    const int32_t j = t < HALO ? (int32_t)lo - HALO + t : (int32_t)(lo + S) + (t - HALO);
    if (j >= w0 && j < w1) {
      const float rj = ldcf(a.r + j);
      sh.win[j - w0] = first ? rj : __builtin_fmaf(beta, ldcf(pp + j), rj);
    }
  }
#pragma unroll
  for (int q = 0; q < R; q++) {
    const int32_t j = (int32_t)lo + BT * q + t;
    if (j < a.n) sh.win[j - w0] = first ? rv[q] : __builtin_fmaf(beta, pv[q], rv[q]);
  }
  __syncthreads();
  wn = w1 - w0;
  return w0;
}

// phase 1 of the resident kernel on staged rows; near: no block reads
// outside its window, so the window comes from registers and halos and
// only the halo rows of p are stored
template <int R, int W, class SH>
__device__ __forceinline__ void cg_phase1_chunk_lds(const CgArgs &a, int64_t c, int k, float beta, SH &sh,
                                                    const uint8_t *dyn, bool near, float (&pv)[R], float (&qv)[R],
                                                    const float (&rv)[R]) {
  constexpr int BT = 32 * W, S = BT * R;
  const bool first = k == 0;
  const float *pp = a.p[(k + 1) & 1];
  float *pn = a.p[k & 1];
  int32_t row[R];
  rows_of<R, W>(c, row);
  int32_t wn;
  const int32_t w0 = near ? cg_window_near<R, W>(a, c, first, beta, pp, pv, rv, sh, wn)
                          : cg_window<R, W>(a, c, first, beta, pp, sh, wn);
  const uint32_t *bnd = (const uint32_t *)dyn;
  const uint2 *ent = (const uint2 *)(dyn + S * 4);
#pragma unroll
  for (int q = 0; q < R; q++) {
    const uint32_t bq = bnd[BT * q + threadIdx.x];
    float acc = 0.0f;
    for (uint32_t e = bq & 0xffffu; e < (bq >> 16); e++) {
      const uint2 ev = ent[e];
      const uint32_t o = ev.x - (uint32_t)w0;
      float g;
      if (o < (uint32_t)wn) {
        g = sh.win[o];
      } else {
        const float rj = ldcf(a.r + ev.x);
        g = first ? rj : __builtin_fmaf(beta, ldcf(pp + ev.x), rj);
      }
      acc = __builtin_fmaf(__uint_as_float(ev.y), g, acc);
    }
    qv[q] = acc;
  }
  cg_phase1_tail<R, W>(a, c, row, w0, pn, sh, pv, qv, near);
}

// x = fmaf(alpha, p, x), r = fmaf(-alpha, q, r), partials of <r, r>
template <int R, int W, class SH>
__device__ __forceinline__ void cg_phase2_chunk(const CgArgs &a, int64_t c, float alpha, SH &sh, const float (&pv)[R],
                                                const float (&qv)[R], float (&xv)[R], float (&rv)[R],
                                                bool near = false) {
  int32_t row[R];
  rows_of<R, W>(c, row);
  double s = -0.0;
#pragma unroll
  for (int q = 0; q < R; q++) {
    if (row[q] < a.n) {
      xv[q] = __builtin_fmaf(alpha, pv[q], xv[q]);
      rv[q] = __builtin_fmaf(-alpha, qv[q], rv[q]);
      if (!near || halo_row(c, row[q], 32 * W * R)) stcf(a.r + row[q], rv[q]);
      s = s + (double)rv[q] * (double)rv[q];
    }
  }
  chunk_store<W>(s, a.prr, c, sh);
}

// streaming forms: per-row values through memory (x and q are only ever
// read back by the thread that wrote them)
template <int R, int W, class SH>
__device__ void cg_phase0(const CgArgs &a, SH &sh) {
  for (int64_t c = blockIdx.x; c < a.nch; c += gridDim.x) {
    float xv[R], rv[R];
    cg_phase0_chunk<R, W, su_stream<R>()>(a, c, sh, xv, rv);
  }
}

template <int R, int W, class SH>
__device__ void cg_phase1(const CgArgs &a, int k, float beta, SH &sh) {
  for (int64_t c = blockIdx.x; c < a.nch; c += gridDim.x) {
    float pv[R], qv[R];
    cg_phase1_chunk<R, W, su_stream<R>()>(a, c, k, beta, sh, pv, qv);
    int32_t row[R];
    rows_of<R, W>(c, row);
#pragma unroll
    for (int q = 0; q < R; q++)
      if (row[q] < a.n) a.q[row[q]] = qv[q];
  }
}

template <int R, int W, class SH>
__device__ void cg_phase2(const CgArgs &a, int k, float alpha, SH &sh) {
  const float *pn = a.p[k & 1];
  for (int64_t c = blockIdx.x; c < a.nch; c += gridDim.x) {
    int32_t row[R];
    rows_of<R, W>(c, row);
    float pv[R], qv[R], xv[R], rv[R];
#pragma unroll
    for (int q = 0; q < R; q++) {
      const bool ok = row[q] < a.n;
      const int32_t i = ok ? row[q] : 0;
      pv[q] = ok ? ldcf(pn + i) : 0.0f;
      rv[q] = ok ? ldcf(a.r + i) : 0.0f;
      qv[q] = ok ? a.q[i] : 0.0f;
      xv[q] = ok ? a.x[i] : 0.0f;
    }
    cg_phase2_chunk<R, W>(a, c, alpha, sh, pv, qv, xv, rv);
#pragma unroll
    for (int q = 0; q < R; q++)
      if (row[q] < a.n) a.x[row[q]] = xv[q];
  }
}

enum : int32_t { CG_CONVERGED = 0, CG_MAX_ITER = 1, CG_BREAKDOWN = 2, CG_ABORTED = 3 };

__device__ __forceinline__ bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }

// the whole solve in one cooperative launch, per-row values through memory
template <int R, int W>
__global__ __launch_bounds__(32 * W) void k_cg(CgArgs a) {
  __shared__ CgShared<R, W> sh;
  int32_t k = 0, reason = CG_ABORTED;
  cg_phase0<R, W>(a, sh);
  if (grid_sync(a.bar, a.hdr)) {
    double rr = final64(a.prr, a.nch, sh), rr_prev = 0.0;
    for (;; k++) {
      if (lead() && a.rr_hist) a.rr_hist[k] = rr;
      if (rr <= a.tol2) {
        reason = CG_CONVERGED;
        break;
      }
      if (k == a.max_iter) {
        reason = CG_MAX_ITER;
        break;
      }
      cg_phase1<R, W>(a, k, k ? (float)(rr / rr_prev) : 0.0f, sh);
      if (!grid_sync(a.bar, a.hdr)) break;
      const double pq = final64(a.ppq, a.nch, sh);
      if (!(pq > 0.0)) {
        reason = CG_BREAKDOWN;
        break;
      }
      cg_phase2<R, W>(a, k, (float)(rr / pq), sh);
      if (!grid_sync(a.bar, a.hdr)) break;
      rr_prev = rr;
      rr = final64(a.prr, a.nch, sh);
    }
  }
  if (lead()) {
    a.result[0] = k;
    a.result[1] = reason;
  }
}

// the same solve with at most one chunk per block (gridDim.x >= nch): the
// block's x, r, p and q stay in registers, its CSR rows in shared memory
// when they fit; x is stored once at the end
template <int R, int W>
__global__ __launch_bounds__(32 * W) void k_cg_res(CgArgs a) {
  __shared__ CgShared<R, W> sh;
  extern __shared__ __align__(16) uint8_t cg_dyn[];
  const int64_t c = blockIdx.x;
  const bool own = c < a.nch;  // uniform over the block
  float xv[R], rv[R], pv[R], qv[R];
  int32_t k = 0, reason = CG_ABORTED;
  const int stage = own ? cg_stage<R, W>(a, c, cg_dyn, sh) : 2;  // uniform over the block
  const bool staged = own && stage > 0;
  // a block that streams its rows or gathers outside its window needs
  // every row of r and p in memory
  if (stage < 2 && threadIdx.x == 0) __hip_atomic_fetch_or(&a.state->far, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (own) cg_phase0_chunk<R, W, su_resident<R>()>(a, c, sh, xv, rv);
  if (grid_sync(a.bar, a.hdr)) {
    // the same word for every thread, written before the barrier
    const bool near = staged && ldc32(&a.state->far) == 0u;
    double rr = final64(a.prr, a.nch, sh), rr_prev = 0.0;
    for (;; k++) {
      if (lead() && a.rr_hist) a.rr_hist[k] = rr;
      if (rr <= a.tol2) {
        reason = CG_CONVERGED;
        break;
      }
      if (k == a.max_iter) {
        reason = CG_MAX_ITER;
        break;
      }
      const float beta = k ? (float)(rr / rr_prev) : 0.0f;
      if (staged)
        cg_phase1_chunk_lds<R, W>(a, c, k, beta, sh, cg_dyn, near, pv, qv, rv);
      else if (own)
        cg_phase1_chunk<R, W, su_resident<R>()>(a, c, k, beta, sh, pv, qv);
      if (!grid_sync(a.bar, a.hdr)) break;
      const double pq = final64(a.ppq, a.nch, sh);
      if (!(pq > 0.0)) {
        reason = CG_BREAKDOWN;
        break;
      }
      if (own) cg_phase2_chunk<R, W>(a, c, (float)(rr / pq), sh, pv, qv, xv, rv, near);
      if (!grid_sync(a.bar, a.hdr)) break;
      rr_prev = rr;
      rr = final64(a.prr, a.nch, sh);
    }
  }
  if (own) {
    int32_t row[R];
    rows_of<R, W>(c, row);
#pragma unroll
    for (int q = 0; q < R; q++)
      if (row[q] < a.n) a.x[row[q]] = xv[q];
  }
  if (lead()) {
    a.result[0] = k;
    a.result[1] = reason;
  }
}

// the same phases as one launch each (the baseline without grid barriers);
// a stopped solve turns the remaining launches into no-ops
template <int R, int W>
__global__ __launch_bounds__(32 * W) void k_cg_p0(CgArgs a) {
  __shared__ CgShared<R, W> sh;
  cg_phase0<R, W>(a, sh);
}

template <int R, int W>
__global__ __launch_bounds__(32 * W) void k_cg_p1(CgArgs a, int32_t k) {
  __shared__ CgShared<R, W> sh;
  if (a.state->stop) return;
  const double rr = final64(a.prr, a.nch, sh);
  if (lead() && a.rr_hist) a.rr_hist[k] = rr;
  const int32_t reason = rr <= a.tol2 ? CG_CONVERGED : (k == a.max_iter ? CG_MAX_ITER : -1);
  if (reason >= 0) {
    if (lead()) {
      a.result[0] = k;
      a.result[1] = reason;
      a.state->stop = 1u;
    }
    return;
  }
  if (lead()) a.state->rr[k & 1] = rr;
  cg_phase1<R, W>(a, k, k ? (float)(rr / a.state->rr[(k + 1) & 1]) : 0.0f, sh);
}

template <int R, int W>
__global__ __launch_bounds__(32 * W) void k_cg_p2(CgArgs a, int32_t k) {
  __shared__ CgShared<R, W> sh;
  if (a.state->stop) return;
  const double pq = final64(a.ppq, a.nch, sh);
  if (!(pq > 0.0)) {
    if (lead()) {
      a.result[0] = k;
      a.result[1] = CG_BREAKDOWN;
      a.state->stop = 1u;
    }
    return;
  }
  cg_phase2<R, W>(a, k, (float)(a.state->rr[k & 1] / pq), sh);
}

// ---------------------------------------------------------------- host side
struct CgLayout {
  size_t bar, state, r, p0, p1, q, prr, ppq, total;
};

static size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

static CgLayout cg_layout(int64_t n, int R, int W) {
  const int64_t S = (int64_t)32 * W * R;
  const int64_t nch = (n + S - 1) / S;
  const size_t vec = up256((size_t)n * 4);
  CgLayout L;
  L.bar = WS_HEADER;
  L.state = L.bar + GB_BYTES;
  L.r = L.state + 256;
  L.p0 = L.r + vec;
  L.p1 = L.p0 + vec;
  L.q = L.p1 + vec;
  L.prr = L.q + vec;
  L.ppq = L.prr + up256((size_t)nch * 8);
  L.total = L.ppq + up256((size_t)nch * 8);
  return L;
}

size_t cg_workspace_bytes(int64_t n, int R, int W) { return cg_layout(n, R, W).total; }
size_t gx_workspace_bytes(int64_t G) { return WS_HEADER + GB_BYTES + (size_t)G * GX_BLOCK * 4; }

template <int R, int W>
struct CgKernels {
  static const void *coop() { return (const void *)k_cg<R, W>; }
  static const void *coop_res() { return (const void *)k_cg_res<R, W>; }
  static void per_phase(const CgArgs &a, int G, hipStream_t st) {
    hipLaunchKernelGGL((k_cg_p0<R, W>), dim3(G), dim3(32 * W), 0, st, a);
    for (int32_t k = 0; k <= a.max_iter; k++) {
      hipLaunchKernelGGL((k_cg_p1<R, W>), dim3(G), dim3(32 * W), 0, st, a, k);
      if (k < a.max_iter) hipLaunchKernelGGL((k_cg_p2<R, W>), dim3(G), dim3(32 * W), 0, st, a, k);
    }
  }
};

struct CgPick {
  const void *coop, *coop_res;
  void (*per_phase)(const CgArgs &, int, hipStream_t);
};

template <int W>
static bool pick_r(int R, CgPick *p) {
  switch (R) {
  case 1: *p = {CgKernels<1, W>::coop(), CgKernels<1, W>::coop_res(), CgKernels<1, W>::per_phase}; return true;
  case 2: *p = {CgKernels<2, W>::coop(), CgKernels<2, W>::coop_res(), CgKernels<2, W>::per_phase}; return true;
  case 4: *p = {CgKernels<4, W>::coop(), CgKernels<4, W>::coop_res(), CgKernels<4, W>::per_phase}; return true;
  case 8: *p = {CgKernels<8, W>::coop(), CgKernels<8, W>::coop_res(), CgKernels<8, W>::per_phase}; return true;
  }
  return false;
}

static bool cg_pick(int R, int W, CgPick *p) {
  switch (W) {
  case 8: return pick_r<8>(R, p);
  case 16: return pick_r<16>(R, p);
  case 32: return pick_r<32>(R, p);
  }
  return false;
}

static cox_status cg_run(const int32_t *row_ptr, const int32_t *col_idx, const float *val, int64_t n, int64_t nnz,
                         const float *b, float *x, int32_t max_iter, double tol, int32_t *result, double *rr_hist,
                         const cox_cfg *cfg, void *ws, size_t ws_bytes, void *stream, bool coop) {
  if (n < 0 || n > INT32_MAX - 8192 || nnz < 0 || nnz > INT32_MAX || max_iter < 0 || max_iter == INT32_MAX)
    return COX_ERR_INVALID;
  if (!result || (n > 0 && (!row_ptr || !val || !b || !x || (nnz > 0 && !col_idx)))) return COX_ERR_INVALID;
  Sigma sg;
  cox_status st = resolve_cfg(COX_OP_CG, COX_F32, cfg, &sg);
  if (st != COX_OK) return st;
  CgPick pk;
  if (!cg_pick(sg.k, sg.W, &pk)) return COX_ERR_UNSUPPORTED;
  const CgLayout L = cg_layout(n, sg.k, sg.W);
  if (!ws || ws_bytes < L.total) return COX_ERR_WORKSPACE;
  const int64_t S = (int64_t)32 * sg.W * sg.k;
  const int64_t nch = (n + S - 1) / S;
  const int block = 32 * sg.W;
  const int cap = std::min(blocks_per_cu(pk.coop, block), blocks_per_cu(pk.coop_res, block)) * device_cus();
  int G = sg.G;
  if (G == 0) G = device_cus();
  if (G > cap) {
    if (sg.G) return COX_ERR_INVALID;
    G = cap;
  }
  if (G > nch) G = (int)(nch > 0 ? nch : 1);
  if (G < 1) return COX_ERR_INVALID;
  char *w = (char *)ws;
  CgArgs a;
  a.rp = row_ptr;
  a.ci = col_idx;
  a.val = val;
  a.b = b;
  a.x = x;
  a.r = (float *)(w + L.r);
  a.p[0] = (float *)(w + L.p0);
  a.p[1] = (float *)(w + L.p1);
  a.q = (float *)(w + L.q);
  a.prr = (double *)(w + L.prr);
  a.ppq = (double *)(w + L.ppq);
  a.nch = nch;
  a.n = (int32_t)n;
  a.nnz = (int32_t)nnz;
  a.max_iter = max_iter;
  a.tol2 = tol * tol;
  a.result = result;
  a.rr_hist = rr_hist;
  a.bar = (uint32_t *)(w + L.bar);
  a.hdr = (uint32_t *)w;
  a.state = (CgState *)(w + L.state);
  a.lds_bytes = 0;
  hipStream_t hs = (hipStream_t)stream;
  const void *fn = G >= nch ? pk.coop_res : pk.coop;
  if (coop && G >= nch) {
    // the resident kernel stages CSR rows in what shared memory the grid
    // leaves: the compute unit's share per block less the static part
    hipFuncAttributes fa;
    const int cus = device_cus(), per_cu = (G + cus - 1) / cus;
    if (hipFuncGetAttributes(&fa, fn) == hipSuccess) {
      const size_t share = device_max_lds() / (size_t)per_cu, fixed = fa.sharedSizeBytes + 512;
      const size_t dyn = share > fixed ? (share - fixed) & ~(size_t)15 : 0;
      if (dyn >= (size_t)S * 4 + 1024 &&
          (dyn <= 65536 ||
           hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) == hipSuccess) &&
          (int64_t)blocks_per_cu(fn, block, dyn) * cus >= G)
        a.lds_bytes = (uint32_t)dyn;
    }
    (void)hipGetLastError();  // a refused attribute only means no staging
  }
  // barrier words and solver state start at zero on every call
  hipLaunchKernelGGL(k_grid_clear, dim3(1), dim3(256), 0, hs, a.bar, (int)((GB_BYTES + 256) / 4));
  if ((st = launch_status()) != COX_OK) return st;
  if (coop) {
    // one chunk per block at most: the register-resident kernel
    void *args[] = {&a};
    const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(block), args, a.lds_bytes, hs);
    if (e != hipSuccess) {
      set_hip_error(e);
      return COX_ERR_HIP;
    }
    return COX_OK;
  }
  pk.per_phase(a, G, hs);
  return launch_status();
}

}  // namespace cox

using namespace cox;

extern "C" {

cox_status cox_cg_solve(const int32_t *row_ptr, const int32_t *col_idx, const float *val, int64_t n, int64_t nnz,
                        const float *b, float *x, int32_t max_iter, double tol, int32_t *result, double *rr_hist,
                        const cox_cfg *cfg, void *ws, size_t ws_bytes, void *stream) {
  return cg_run(row_ptr, col_idx, val, n, nnz, b, x, max_iter, tol, result, rr_hist, cfg, ws, ws_bytes, stream,
                true);
}

cox_status cox_cg_solve_per_phase(const int32_t *row_ptr, const int32_t *col_idx, const float *val, int64_t n,
                                  int64_t nnz, const float *b, float *x, int32_t max_iter, double tol,
                                  int32_t *result, double *rr_hist, const cox_cfg *cfg, void *ws, size_t ws_bytes,
                                  void *stream) {
  return cg_run(row_ptr, col_idx, val, n, nnz, b, x, max_iter, tol, result, rr_hist, cfg, ws, ws_bytes, stream,
                false);
}

cox_status cox_grid_capacity(int32_t *max_blocks) {
  if (!max_blocks) return COX_ERR_INVALID;
  *max_blocks = blocks_per_cu((const void *)k_grid_exchange, GX_BLOCK) * device_cus();
  return launch_status();
}

static cox_status gx_run(int32_t grid_blocks, int32_t rounds, int absent, uint32_t spin_limit, uint32_t *out, void *ws,
                        size_t ws_bytes, void *stream) {
  if (grid_blocks < 1 || rounds < 0 || !out) return COX_ERR_INVALID;
  if (grid_blocks > blocks_per_cu((const void *)k_grid_exchange, GX_BLOCK) * device_cus()) return COX_ERR_INVALID;
  if (!ws || ws_bytes < gx_workspace_bytes(grid_blocks)) return COX_ERR_WORKSPACE;
  char *w = (char *)ws;
  uint32_t *bar = (uint32_t *)(w + WS_HEADER);
  uint32_t *slot = (uint32_t *)(w + WS_HEADER + GB_BYTES);
  uint32_t *hdr = (uint32_t *)w;
  hipStream_t hs = (hipStream_t)stream;
  hipLaunchKernelGGL(k_grid_clear, dim3(1), dim3(256), 0, hs, bar, (int)(GB_BYTES / 4));
  cox_status st = launch_status();
  if (st != COX_OK) return st;
  void *args[] = {&slot, &out, &rounds, &bar, &hdr, &absent, &spin_limit};
  const hipError_t e = hipLaunchCooperativeKernel((const void *)k_grid_exchange, dim3(grid_blocks), dim3(GX_BLOCK),
                                                  args, 0, hs);
  if (e != hipSuccess) {
    set_hip_error(e);
    return COX_ERR_HIP;
  }
  return COX_OK;
}

cox_status cox_grid_exchange(int32_t grid_blocks, int32_t rounds, uint32_t *out, void *ws, size_t ws_bytes,
                             void *stream) {
  return gx_run(grid_blocks, rounds, -1, GRID_MAX_SPIN, out, ws, ws_bytes, stream);
}

cox_status cox_grid_exchange_absent(int32_t grid_blocks, int32_t rounds, int32_t absent_block, uint32_t spin_limit,
                                    uint32_t *out, void *ws, size_t ws_bytes, void *stream) {
  if (absent_block < 0 || absent_block >= grid_blocks || spin_limit < 1 || spin_limit > GRID_MAX_SPIN)
    return COX_ERR_INVALID;
  return gx_run(grid_blocks, rounds, absent_block, spin_limit, out, ws, ws_bytes, stream);
}

}  // extern "C"
