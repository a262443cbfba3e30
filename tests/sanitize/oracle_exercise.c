/*
 * Sanitizer driver for the CPU oracle (test infrastructure).
 *
 * Linked with oracle/coxo.c into one executable that is built twice, with
 * AddressSanitizer + UndefinedBehaviorSanitizer and with ThreadSanitizer.
 * It calls every oracle entry point on seeded inputs that cover the edge
 * cases the kernels have (empty, ragged, single element, every tile width,
 * every legal schedule corner, masks with holes, empty segments, invalid
 * arguments), once on one worker thread and once on the block pool, and
 * checks that
 *   - every call returns the status the arguments call for;
 *   - sorted outputs are sorted and hold the input multiset;
 *   - the outputs are byte-identical for both thread counts (the oracle's
 *     blocks are independent, so the pool must not change a single bit;
 *     the one exception, the order of the warp-aggregated appends, is
 *     compared as a multiset).
 * Any sanitizer report aborts the program with a nonzero status.
 *
 * Usage: oracle_exercise [threads]   (default 8)
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* the oracle's C entry points */
int coxo_set_threads(int n);
int coxo_warp_shfl(const int32_t *v, int32_t *out, int64_t n, int op, int32_t arg, const int32_t *argv,
                   int width, const uint32_t *mask);
int coxo_warp_vote(const int32_t *pred, const uint32_t *mask, int64_t n, uint32_t *ballot, int32_t *anyall);
int coxo_tile_vote(const int32_t *pred, int64_t n, int T, uint32_t *ballot, int32_t *anyall);
int coxo_reduce_blocks_i32(const int32_t *x, int64_t n, int32_t *block_sums, int32_t *warp_pos);
int coxo_reduce(const void *x, int dtype, int64_t n, int acc, int k, int W, void *partials, void *total);
int coxo_dot(const void *a, const void *b, int dtype, int64_t n, int acc, int k, int W, void *partials,
             double *total);
int coxo_scan_i32(const int32_t *x, int32_t *y, int64_t n, int k, int W);
int coxo_compact_i32(const int32_t *x, int64_t n, int32_t *out, int64_t *count, int k, int W);
int coxo_tile_sort_u32(const uint32_t *keys, uint32_t *out, int64_t n, int G);
int coxo_group_sort_u32(const uint32_t *keys, uint32_t *out, int64_t n, int G);
int coxo_tile_sort_kv_u32(const uint32_t *keys, const uint32_t *vals, uint32_t *out_keys, uint32_t *out_vals,
                          int64_t n);
int coxo_tile_reduce_i32(const int32_t *x, int64_t n, int T, int32_t *out);
int coxo_warp_masked(const int32_t *x, int64_t n, int D, int32_t *out, uint32_t *rec);
int coxo_warp_dynamic(const int32_t *x, int64_t n, int D, uint32_t *mm, uint32_t *rank, uint32_t *rec,
                      int32_t *filt, int64_t *count);
int coxo_segmented(const void *x, int dtype, const int64_t *off, int64_t nseg, int k, int W, void *seg_total,
                   void *y, void *out_compact, int64_t *seg_count);
int coxo_exact_sum(const void *x, const void *y, int dtype, int64_t n, double *out);
int coxo_exact_sum_f64(const double *x, int64_t n, double *out);
int coxo_code5(const int32_t *a, const int32_t *b, int32_t *r1, int32_t *r2, int barriers);
int coxo_uniform_branch(const int32_t *cond, const int32_t *x, int64_t n, int32_t *out);
int coxo_integral_image_u8(const uint8_t *img, int64_t H, int64_t W, uint32_t *sat);
int coxo_grid_exchange(int G, int BT, int rounds, uint32_t *out);
int coxo_cg(const int32_t *rp, const int32_t *ci, const float *val, int64_t n, const float *b, float *x,
            int max_iter, double tol, int R, int W, int32_t *result, double *rr_hist);
void coxo_two_sum(float a, float b, float *s, float *e);
void coxo_two_prod(float a, float b, float *p, float *e);

enum { OK = 0, INVALID = 1, DTYPE = 2, UB = 8, DIVERGENT = 9 };
enum { I32 = 0, U32 = 1, F32 = 2, BF16 = 3 };

/* ---------------------------------------------------------------- inputs */
static uint64_t g_rng;
static void seed(uint64_t s) { g_rng = s * 0x9E3779B97F4A7C15ull + 0x1234567ull; }
static uint32_t rnd(void) { /* xorshift64* */
  g_rng ^= g_rng >> 12;
  g_rng ^= g_rng << 25;
  g_rng ^= g_rng >> 27;
  return (uint32_t)((g_rng * 0x2545F4914F6CDD1Dull) >> 32);
}
static float unif(float lo, float hi) { return lo + (hi - lo) * (float)(rnd() >> 8) * (1.0f / 16777216.0f); }

static void *xalloc(size_t bytes) {
  void *p = calloc(bytes ? bytes : 1, 1);
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(3);
  }
  return p;
}
static int32_t *rand_i32(int64_t n) {
  int32_t *a = (int32_t *)xalloc((size_t)n * 4);
  for (int64_t i = 0; i < n; i++) a[i] = (int32_t)rnd();
  return a;
}
static uint32_t *rand_u32(int64_t n, uint32_t mod) {
  uint32_t *a = (uint32_t *)xalloc((size_t)n * 4);
  for (int64_t i = 0; i < n; i++) a[i] = mod ? rnd() % mod : rnd();
  return a;
}
static float *rand_f32(int64_t n) {
  float *a = (float *)xalloc((size_t)n * 4);
  for (int64_t i = 0; i < n; i++) a[i] = unif(-1.0f, 1.0f) * (float)(1 + (rnd() & 7));
  return a;
}
static uint16_t *rand_bf16(int64_t n) {
  uint16_t *a = (uint16_t *)xalloc((size_t)n * 2);
  for (int64_t i = 0; i < n; i++) {
    float f = unif(-4.0f, 4.0f);
    uint32_t u;
    memcpy(&u, &f, 4);
    a[i] = (uint16_t)(u >> 16);
  }
  return a;
}

/* ---------------------------------------------------------------- record */
#define MAXREC 4096
typedef struct {
  uint64_t h[MAXREC];
  char what[MAXREC][48];
  int n;
} record;
static record *g_rec;
static uint64_t g_h;

static void hmix(const void *p, size_t bytes) { /* FNV-1a */
  const unsigned char *c = (const unsigned char *)p;
  for (size_t i = 0; i < bytes; i++) g_h = (g_h ^ c[i]) * 0x100000001B3ull;
}
static void begin(void) { g_h = 0xCBF29CE484222325ull; }
static void end(const char *what) {
  if (g_rec->n >= MAXREC) {
    fprintf(stderr, "too many cases\n");
    exit(3);
  }
  g_rec->h[g_rec->n] = g_h;
  snprintf(g_rec->what[g_rec->n], sizeof g_rec->what[0], "%s", what);
  g_rec->n++;
}

static void fail(const char *what, const char *detail) {
  fprintf(stderr, "FAIL %s: %s\n", what, detail);
  exit(1);
}
static void expect(int got, int want, const char *what) {
  if (got != want) {
    char d[64];
    snprintf(d, sizeof d, "status %d, expected %d", got, want);
    fail(what, d);
  }
  hmix(&got, sizeof got);
}

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return (x > y) - (x < y);
}
static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}
/* out holds, group by group of g keys, the keys of `in` sorted */
static void check_groups_sorted(const uint32_t *in, const uint32_t *out, int64_t n, int64_t g, const char *what) {
  uint32_t *t = (uint32_t *)xalloc((size_t)g * 4);
  for (int64_t s = 0; s < n; s += g) {
    int64_t m = n - s < g ? n - s : g;
    memcpy(t, in + s, (size_t)m * 4);
    qsort(t, (size_t)m, 4, cmp_u32);
    if (memcmp(t, out + s, (size_t)m * 4)) fail(what, "a group is not the sorted input group");
  }
  free(t);
}

/* ---------------------------------------------------------------- cases */
static void case_shfl(void) {
  static const int widths[] = {1, 2, 4, 8, 16, 32};
  const int64_t n = 32 * 9;
  for (int op = 0; op < 4; op++)
    for (int wi = 0; wi < 6; wi++) {
      char what[48];
      snprintf(what, sizeof what, "shfl op%d width%d", op, widths[wi]);
      seed(100 + op * 8 + wi);
      int32_t *v = rand_i32(n), *out = (int32_t *)xalloc(n * 4), *argv = (int32_t *)xalloc(n * 4);
      uint32_t *mask = rand_u32(n / 32, 0);
      mask[0] = 0xffffffffu;
      mask[1] = 0;
      mask[2] = 1u << 31;
      begin();
      int32_t arg = op == 0 ? (int32_t)(rnd() % 97) - 40 : (int32_t)(rnd() % 32);
      expect(coxo_warp_shfl(v, out, n, op, arg, NULL, widths[wi], NULL), OK, what);
      hmix(out, n * 4);
      for (int64_t i = 0; i < n; i++) argv[i] = (int32_t)(rnd() % 32);
      expect(coxo_warp_shfl(v, out, n, op, 0, argv, widths[wi], NULL), OK, what);
      hmix(out, n * 4);
      /* a partial mask may name an undefined read; only the status is fixed */
      int st = coxo_warp_shfl(v, out, n, op, arg, NULL, widths[wi], mask);
      if (st != OK && st != UB) fail(what, "masked shuffle status");
      hmix(&st, sizeof st);
      if (st == OK) hmix(out, n * 4);
      /* invalid arguments */
      expect(coxo_warp_shfl(v, out, n - 1, op, arg, NULL, widths[wi], NULL), INVALID, what);
      expect(coxo_warp_shfl(v, out, n, op, arg, NULL, 3, NULL), INVALID, what);
      if (op) expect(coxo_warp_shfl(v, out, n, op, 32, NULL, widths[wi], NULL), INVALID, what);
      end(what);
      free(v), free(out), free(argv), free(mask);
    }
}

static void case_vote(void) {
  const int64_t n = 32 * 40;
  seed(200);
  int32_t *pred = (int32_t *)xalloc(n * 4);
  for (int64_t i = 0; i < n; i++) pred[i] = (int32_t)(rnd() % 3) - 1;
  for (int64_t i = 0; i < 32; i++) pred[i] = 1; /* an all-true warp */
  uint32_t *mask = rand_u32(n / 32, 0), *bal = (uint32_t *)xalloc(n / 8);
  int32_t *aa = (int32_t *)xalloc(n / 8);
  mask[3] = 0, mask[4] = 0xffffffffu;
  begin();
  expect(coxo_warp_vote(pred, mask, n, bal, aa), OK, "vote");
  hmix(bal, n / 8), hmix(aa, n / 8);
  expect(coxo_warp_vote(pred, NULL, n, bal, aa), OK, "vote");
  hmix(bal, n / 8), hmix(aa, n / 8);
  expect(coxo_warp_vote(pred, NULL, 31, bal, aa), INVALID, "vote");
  uint32_t *tb = (uint32_t *)xalloc(n * 4);
  int32_t *ta = (int32_t *)xalloc(n * 4);
  for (int T = 1; T <= 32; T *= 2) {
    expect(coxo_tile_vote(pred, n, T, tb, ta), OK, "tile vote");
    hmix(tb, n / T * 4), hmix(ta, n / T * 4);
  }
  expect(coxo_tile_vote(pred, n, 3, tb, ta), INVALID, "tile vote");
  expect(coxo_tile_vote(pred, 31, 1, tb, ta), INVALID, "tile vote");
  end("vote");
  free(pred), free(mask), free(bal), free(aa), free(tb), free(ta);
}

static void case_reduce_blocks(void) {
  static const int64_t ns[] = {0, 1, 255, 256, 1000, 4097};
  for (int i = 0; i < 6; i++) {
    int64_t n = ns[i];
    seed(300 + i);
    int32_t *x = rand_i32(n), *bs = (int32_t *)xalloc(((n + 255) / 256) * 4),
            *wp = (int32_t *)xalloc(((n + 31) / 32) * 4);
    begin();
    expect(coxo_reduce_blocks_i32(x, n, bs, wp), OK, "reduce_blocks");
    hmix(bs, ((n + 255) / 256) * 4), hmix(wp, ((n + 31) / 32) * 4);
    end("reduce_blocks");
    free(x), free(bs), free(wp);
  }
}

static const int SIGMA[][2] = {{1, 1}, {1, 32}, {2, 3}, {4, 8}, {8, 32}, {32, 1}};
#define NSIGMA 6

static void case_reduce_dot_scan_compact(void) {
  static const int64_t ns[] = {0, 1, 33, 5000, 70001};
  for (int si = 0; si < NSIGMA; si++)
    for (int ni = 0; ni < 5; ni++) {
      const int k = SIGMA[si][0], W = SIGMA[si][1];
      const int64_t n = ns[ni], S = 32LL * W * k, nch = (n + S - 1) / S;
      char what[48];
      snprintf(what, sizeof what, "reduce k%d W%d n%lld", k, W, (long long)n);
      seed(400 + si * 8 + ni);
      int32_t *xi = rand_i32(n);
      float *xf = rand_f32(n), *yf = rand_f32(n);
      uint16_t *xb = rand_bf16(n), *yb = rand_bf16(n);
      void *part = xalloc((size_t)(nch + 1) * 8);
      double tot = 0;
      int64_t itot = 0;
      begin();
      expect(coxo_reduce(xi, I32, n, 0, k, W, part, &itot), OK, what);
      hmix(part, nch * 4), hmix(&itot, 8);
      expect(coxo_reduce(xi, I32, n, 1, k, W, part, &itot), DTYPE, what);
      for (int acc = 0; acc < 2; acc++) {
        const size_t pb = (size_t)nch * 4 * (acc + 1);
        expect(coxo_reduce(xf, F32, n, acc, k, W, part, &tot), OK, what);
        hmix(part, pb), hmix(&tot, 8);
        expect(coxo_reduce(xb, BF16, n, acc, k, W, part, &tot), OK, what);
        hmix(part, pb), hmix(&tot, 8);
        expect(coxo_dot(xf, yf, F32, n, acc, k, W, part, &tot), OK, what);
        hmix(part, pb), hmix(&tot, 8);
        expect(coxo_dot(xb, yb, BF16, n, acc, k, W, part, &tot), OK, what);
        hmix(part, pb), hmix(&tot, 8);
      }
      expect(coxo_dot(xi, xi, I32, n, 0, k, W, part, &tot), DTYPE, what);
      expect(coxo_reduce(xf, F32, n, 2, k, W, part, &tot), INVALID, what);
      int32_t *y = (int32_t *)xalloc((size_t)n * 4), *c = (int32_t *)xalloc((size_t)n * 4);
      int64_t cnt = -1;
      expect(coxo_scan_i32(xi, y, n, k, W), OK, what);
      hmix(y, (size_t)n * 4);
      expect(coxo_compact_i32(xi, n, c, &cnt, k, W), OK, what);
      if (cnt < 0 || cnt > n) fail(what, "compaction count out of range");
      hmix(&cnt, 8), hmix(c, (size_t)cnt * 4);
      expect(coxo_scan_i32(xi, y, n, 3, W), INVALID, what);
      expect(coxo_compact_i32(xi, n, c, &cnt, k, 33), INVALID, what);
      end(what);
      free(xi), free(xf), free(yf), free(xb), free(yb), free(part), free(y), free(c);
    }
}

static void case_sorts(void) {
  static const int64_t ns[] = {0, 1, 31, 32 * 50 + 7, 9000};
  for (int ni = 0; ni < 5; ni++) {
    const int64_t n = ns[ni];
    char what[48];
    snprintf(what, sizeof what, "sorts n%lld", (long long)n);
    seed(500 + ni);
    uint32_t *keys = rand_u32(n, ni & 1 ? 17 : 0), *vals = rand_u32(n, 0), *out = (uint32_t *)xalloc(n * 4),
             *ov = (uint32_t *)xalloc(n * 4);
    begin();
    for (int G = 2; G <= 32; G *= 2) {
      expect(coxo_tile_sort_u32(keys, out, n, G), OK, what);
      check_groups_sorted(keys, out, n, G, what);
      hmix(out, n * 4);
    }
    expect(coxo_tile_sort_u32(keys, out, n, 64), INVALID, what);
    for (int G = 2; G <= 4096; G *= 4) {
      expect(coxo_group_sort_u32(keys, out, n, G), OK, what);
      check_groups_sorted(keys, out, n, G, what);
      hmix(out, n * 4);
    }
    expect(coxo_group_sort_u32(keys, out, n, 8192), INVALID, what);
    expect(coxo_group_sort_u32(keys, out, n, 48), INVALID, what);
    expect(coxo_tile_sort_kv_u32(keys, vals, out, ov, n), OK, what);
    check_groups_sorted(keys, out, n, 32, what);
    for (int64_t i = 0; i < n; i++) /* stable: equal keys keep the order of their values' positions */
      if (i % 32 && out[i] == out[i - 1]) {
        int64_t a = -1, b = -1, s = i / 32 * 32;
        for (int64_t j = s; j < s + 32 && j < n; j++) {
          if (vals[j] == ov[i - 1] && keys[j] == out[i - 1] && a < 0) a = j;
          if (vals[j] == ov[i] && keys[j] == out[i]) b = j;
        }
        if (a < 0 || b < 0 || a >= b) fail(what, "key-value sort is not stable");
      }
    hmix(out, n * 4), hmix(ov, n * 4);
    for (int T = 2; T <= 32; T *= 2) {
      int32_t *tr = (int32_t *)xalloc(((n + T - 1) / T) * 4);
      expect(coxo_tile_reduce_i32((const int32_t *)vals, n, T, tr), OK, what);
      hmix(tr, ((n + T - 1) / T) * 4);
      free(tr);
    }
    end(what);
    free(keys), free(vals), free(out), free(ov);
  }
}

static void case_masked_dynamic(void) {
  static const int Ds[] = {0, 1, 17, 32, 1024};
  const int64_t n = 32 * 24;
  for (int di = 0; di < 5; di++) {
    const int D = Ds[di];
    char what[48];
    snprintf(what, sizeof what, "masked/dynamic D%d", D);
    seed(600 + di);
    int32_t *x = (int32_t *)xalloc(n * 4), *out = (int32_t *)xalloc(n * 4), *filt = (int32_t *)xalloc(n * 4);
    for (int64_t i = 0; i < n; i++) x[i] = (int32_t)(rnd() % 7) - 3;
    uint32_t *rec = (uint32_t *)xalloc(n), *mm = (uint32_t *)xalloc(n * 4), *rank = (uint32_t *)xalloc(n * 4);
    int64_t cnt = -1;
    begin();
    expect(coxo_warp_masked(x, n, D, out, rec), OK, what);
    hmix(out, n * 4), hmix(rec, (n / 32) * 16);
    expect(coxo_warp_dynamic(x, n, D, mm, rank, rec, filt, &cnt), OK, what);
    if (cnt < 0 || cnt > n) fail(what, "append count out of range");
    qsort(filt, (size_t)cnt, 4, cmp_i32); /* the order of the appends is the pool's */
    hmix(mm, n * 4), hmix(rank, n * 4), hmix(rec, (n / 32) * 32), hmix(&cnt, 8), hmix(filt, (size_t)cnt * 4);
    expect(coxo_warp_masked(x, n, 1025, out, rec), INVALID, what);
    expect(coxo_warp_dynamic(x, n - 5, D, mm, rank, rec, filt, &cnt), INVALID, what);
    end(what);
    free(x), free(out), free(filt), free(rec), free(mm), free(rank);
  }
}

static void case_segmented(void) {
  static const int64_t nsegs[] = {0, 1, 7, 40};
  for (int si = 0; si < NSIGMA; si += 2)
    for (int gi = 0; gi < 4; gi++) {
      const int k = SIGMA[si][0], W = SIGMA[si][1];
      const int64_t nseg = nsegs[gi];
      char what[48];
      snprintf(what, sizeof what, "segmented k%d W%d nseg%lld", k, W, (long long)nseg);
      seed(700 + si * 8 + gi);
      int64_t *off = (int64_t *)xalloc((size_t)(nseg + 1) * 8);
      for (int64_t s = 0; s < nseg; s++) {
        uint32_t r = rnd() % 4;
        off[s + 1] = off[s] + (r == 0 ? 0 : r == 1 ? rnd() % 40 : rnd() % 3000);
      }
      const int64_t n = off[nseg];
      int32_t *xi = rand_i32(n);
      float *xf = rand_f32(n);
      void *tot = xalloc((size_t)nseg * 8), *y = xalloc((size_t)n * 4), *oc = xalloc((size_t)n * 4);
      int64_t *cnt = (int64_t *)xalloc((size_t)nseg * 8);
      begin();
      expect(coxo_segmented(xi, I32, off, nseg, k, W, tot, y, oc, cnt), OK, what);
      hmix(tot, nseg * 8), hmix(y, n * 4), hmix(oc, n * 4), hmix(cnt, nseg * 8);
      memset(y, 0, (size_t)n * 4), memset(oc, 0, (size_t)n * 4);
      expect(coxo_segmented(xf, F32, off, nseg, k, W, tot, y, oc, cnt), OK, what);
      hmix(tot, nseg * 8), hmix(y, n * 4), hmix(oc, n * 4), hmix(cnt, nseg * 8);
      expect(coxo_segmented(xf, BF16, off, nseg, k, W, tot, y, oc, cnt), DTYPE, what);
      if (nseg > 1) {
        int64_t keep = off[1];
        off[1] = off[2] + 1; /* decreasing offsets */
        expect(coxo_segmented(xi, I32, off, nseg, k, W, tot, y, oc, cnt), INVALID, what);
        off[1] = keep;
      }
      end(what);
      free(off), free(xi), free(xf), free(tot), free(y), free(oc), free(cnt);
    }
}

static void case_exact_and_small(void) {
  static const int64_t ns[] = {0, 1, 1000, 70001};
  for (int ni = 0; ni < 4; ni++) {
    const int64_t n = ns[ni];
    seed(800 + ni);
    int32_t *xi = rand_i32(n);
    float *xf = rand_f32(n), *yf = rand_f32(n);
    uint16_t *xb = rand_bf16(n);
    double *xd = (double *)xalloc((size_t)n * 8), out = 0;
    for (int64_t i = 0; i < n; i++) xd[i] = (double)xf[i] * 1e10 + (double)yf[i];
    begin();
    expect(coxo_exact_sum(xf, NULL, F32, n, &out), OK, "exact");
    hmix(&out, 8);
    expect(coxo_exact_sum(xf, yf, F32, n, &out), OK, "exact");
    hmix(&out, 8);
    expect(coxo_exact_sum(xb, xb, BF16, n, &out), OK, "exact");
    hmix(&out, 8);
    expect(coxo_exact_sum(xi, NULL, I32, n, &out), OK, "exact");
    hmix(&out, 8);
    expect(coxo_exact_sum(xi, NULL, U32, n, &out), DTYPE, "exact");
    expect(coxo_exact_sum_f64(xd, n, &out), OK, "exact");
    hmix(&out, 8);
    end("exact");
    free(xi), free(xf), free(yf), free(xb), free(xd);
  }
  seed(850);
  int32_t *a = rand_i32(32), *b = rand_i32(32), r1[32], r2[32];
  for (int l = 0; l < 32; l++) a[l] &= 1, b[l] |= 1;
  begin();
  expect(coxo_code5(a, b, r1, r2, 1), OK, "code5");
  hmix(r1, sizeof r1), hmix(r2, sizeof r2);
  expect(coxo_code5(a, b, r1, r2, 0), UB, "code5 without barriers");
  float s, e;
  coxo_two_sum(1.0f, 1e-9f, &s, &e);
  hmix(&s, 4), hmix(&e, 4);
  coxo_two_prod(1.0f + 1e-7f, 3.0f, &s, &e);
  hmix(&s, 4), hmix(&e, 4);
  end("code5");
  free(a), free(b);
  const int64_t n = 32 * 12;
  int32_t *cond = (int32_t *)xalloc(n * 4), *x = rand_i32(n), *out = (int32_t *)xalloc(n * 4);
  for (int64_t w = 0; w < n / 32; w++)
    for (int l = 0; l < 32; l++) cond[32 * w + l] = (int32_t)(w % 3 == 0);
  begin();
  expect(coxo_uniform_branch(cond, x, n, out), OK, "uniform branch");
  hmix(out, n * 4);
  cond[32 * 5 + 7] ^= 1;
  expect(coxo_uniform_branch(cond, x, n, out), DIVERGENT, "divergent branch");
  end("uniform branch");
  free(cond), free(x), free(out);
}

static void case_image(void) {
  static const int64_t hw[][2] = {{0, 0}, {0, 5}, {5, 0}, {1, 1}, {1, 1500}, {37, 1001}, {130, 70}, {64, 2048}};
  for (int i = 0; i < 8; i++) {
    const int64_t H = hw[i][0], W = hw[i][1];
    seed(900 + i);
    uint8_t *img = (uint8_t *)xalloc((size_t)(H * W));
    for (int64_t j = 0; j < H * W; j++) img[j] = (uint8_t)rnd();
    uint32_t *sat = (uint32_t *)xalloc((size_t)(H * W) * 4);
    begin();
    expect(coxo_integral_image_u8(img, H, W, sat), OK, "image");
    if (H && W) { /* the corner holds the sum of all pixels */
      uint32_t s = 0;
      for (int64_t j = 0; j < H * W; j++) s += img[j];
      if (sat[H * W - 1] != s) fail("image", "corner is not the pixel sum");
    }
    hmix(sat, (size_t)(H * W) * 4);
    expect(coxo_integral_image_u8(img, -1, W, sat), INVALID, "image");
    end("image");
    free(img), free(sat);
  }
}

static void case_grid_exchange(void) {
  static const int cfg[][3] = {{1, 1, 3}, {3, 64, 5}, {17, 1024, 4}, {64, 256, 2}, {5, 32, 0}};
  for (int i = 0; i < 5; i++) {
    const int G = cfg[i][0], BT = cfg[i][1], R = cfg[i][2];
    uint32_t *out = (uint32_t *)xalloc((size_t)G * BT * 4);
    begin();
    expect(coxo_grid_exchange(G, BT, R, out), OK, "grid exchange");
    hmix(out, (size_t)G * BT * 4);
    end("grid exchange");
    free(out);
  }
  begin();
  expect(coxo_grid_exchange(0, 32, 1, NULL), INVALID, "grid exchange");
  expect(coxo_grid_exchange(4, 1025, 1, NULL), INVALID, "grid exchange");
  end("grid exchange args");
}

/* symmetric, strictly diagonally dominant band matrix with bands at 1 and
 * (when n > dist) at dist, columns ascending in every row */
static int64_t band_csr(int64_t n, int64_t dist, int32_t **rp, int32_t **ci, float **val) {
  float *lo1 = rand_f32(n), *lo2 = rand_f32(n);
  *rp = (int32_t *)xalloc((size_t)(n + 1) * 4);
  *ci = (int32_t *)xalloc((size_t)n * 5 * 4);
  *val = (float *)xalloc((size_t)n * 5 * 4);
  int64_t e = 0;
  for (int64_t i = 0; i < n; i++) {
    (*rp)[i] = (int32_t)e;
    const int64_t cols[5] = {i - dist, i - 1, i, i + 1, i + dist};
    for (int c = 0; c < 5; c++) {
      const int64_t j = cols[c];
      if (j < 0 || j >= n || (c != 2 && (j == i))) continue;
      if ((c == 0 || c == 4) && dist <= 1) continue;
      float v;
      if (c == 2) v = 9.0f + unif(0.0f, 1.0f);
      else if (c == 1 || c == 3) v = -0.25f * lo1[i < j ? i : j];
      else v = -0.25f * lo2[i < j ? i : j];
      (*ci)[e] = (int32_t)j;
      (*val)[e] = v;
      e++;
    }
  }
  (*rp)[n] = (int32_t)e;
  free(lo1), free(lo2);
  return e;
}

static void case_cg(void) {
  static const int64_t ns[] = {0, 1, 37, 3 * 4096 + 17, 20011};
  static const int sig[][2] = {{1, 8}, {4, 32}, {8, 16}, {2, 1}};
  for (int ni = 0; ni < 5; ni++)
    for (int si = 0; si < 4; si++) {
      const int64_t n = ns[ni];
      const int R = sig[si][0], W = sig[si][1];
      char what[48];
      snprintf(what, sizeof what, "cg n%lld R%d W%d", (long long)n, R, W);
      seed(1000 + ni * 8 + si);
      int32_t *rp, *ci;
      float *val;
      band_csr(n, ni & 1 ? 5 : 1, &rp, &ci, &val);
      float *b = rand_f32(n), *x = (float *)xalloc((size_t)n * 4);
      int32_t res[2];
      double hist[61];
      begin();
      for (int pass = 0; pass < 3; pass++) {
        const int max_iter = pass == 0 ? 0 : pass == 1 ? 12 : 60;
        const double tol = pass == 2 ? 1e-4 : 0.0;
        memset(x, 0, (size_t)n * 4);
        memset(hist, 0, sizeof hist);
        expect(coxo_cg(rp, ci, val, n, b, x, max_iter, tol, R, W, res, hist), OK, what);
        if (res[0] < 0 || res[0] > max_iter || res[1] < 0 || res[1] > 2) fail(what, "result out of range");
        hmix(res, sizeof res), hmix(x, (size_t)n * 4), hmix(hist, sizeof hist);
      }
      expect(coxo_cg(rp, ci, val, n, b, x, 5, 0.0, 16, W, res, hist), INVALID, what);
      expect(coxo_cg(rp, ci, val, n, b, x, -1, 0.0, R, W, res, hist), INVALID, what);
      if (n > 2) { /* a column index out of range is rejected before any pass */
        int32_t keep = ci[1];
        ci[1] = (int32_t)n;
        expect(coxo_cg(rp, ci, val, n, b, x, 5, 0.0, R, W, res, hist), INVALID, what);
        ci[1] = keep;
      }
      end(what);
      free(rp), free(ci), free(val), free(b), free(x);
    }
}

static void exercise(record *r) {
  g_rec = r;
  r->n = 0;
  case_shfl();
  case_vote();
  case_reduce_blocks();
  case_reduce_dot_scan_compact();
  case_sorts();
  case_masked_dynamic();
  case_segmented();
  case_exact_and_small();
  case_image();
  case_grid_exchange();
  case_cg();
}

int main(int argc, char **argv) {
  const int T = argc > 1 ? atoi(argv[1]) : 8;
  static record one, many;
  coxo_set_threads(1);
  exercise(&one);
  coxo_set_threads(T);
  exercise(&many);
  if (one.n != many.n) fail("driver", "case counts differ");
  for (int i = 0; i < one.n; i++)
    if (one.h[i] != many.h[i]) fail(one.what[i], "outputs differ between 1 and many threads");
  printf("ok %d cases, threads 1 and %d\n", one.n, T);
  return 0;
}
