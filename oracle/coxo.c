/*
 * CPU oracle for the warp-primitive hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source,
 * header, table or helper with the GPU library and includes nothing from it.
 *
 * Execution model: hierarchical collapsing (COX, Sec. 3; Code 3 in Sec. 2.3).
 * One CPU thread executes a whole thread block as a sequence of block-level
 * parallel regions.  A block-level region is an inter-warp loop over the
 * warps w of the block; inside it, warp-level regions are intra-warp loops
 * over the 32 lanes l.  Warp-level functions are builtins that read a
 * per-warp exchange array (the paper's warp_vote / shfl_arr, Sec. 3.2): every
 * lane first writes its operand (then a RAW warp barrier), then every lane
 * calls the builtin (then a WAR warp barrier, Code 5).  The WAR barrier here
 * poisons the array so that a builtin reading stale operands is caught.
 * Values that live across warp regions are [32] arrays and values that live
 * across block regions are [32*W] arrays (Sec. 3.6).  A branch that encloses
 * a barrier is evaluated by every lane, must be uniform (aligned barriers,
 * Sec. 2.2.3), and is then followed as lane 0 decides (loop peeling,
 * Sec. 3.3.1).  Blocks run on a pool of CPU threads, one block at a time per
 * thread, as the runtime maps a CUDA block to a CPU thread (Sec. 4).
 *
 * Warp-function semantics (shfl / shfl_up / shfl_down / shfl_xor with width,
 * ballot / any / all with masks) are the CUDA Programming Guide's, which the
 * paper refers to for them (Sec. 2.2.1).  Undefined uses (caller outside the
 * mask, a lane of the mask not executing the call, reading a lane outside the
 * mask) are reported as COXO_ERR_UB instead of producing a value.
 *
 * Floating point: binary32 with round-to-nearest-even, no contraction (build
 * with -ffp-contract=off), fmaf() only where a schedule names an FMA.  The
 * order of every floating-point operation is fixed by the schedule
 * sigma = (k, W) documented with each kernel below.
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------ */
/* status codes, dtypes, op codes (oracle's own copies)                */
/* ------------------------------------------------------------------ */
enum {
  COXO_OK = 0,
  COXO_ERR_INVALID = 1,
  COXO_ERR_DTYPE = 2,
  COXO_ERR_UB = 8,        /* undefined warp-function use */
  COXO_ERR_DIVERGENT = 9, /* a branch enclosing a barrier was not uniform */
  COXO_ERR_RANGE = 10,    /* exact accumulator range exceeded */
  COXO_ERR_NOMEM = 11
};
enum { DT_I32 = 0, DT_U32 = 1, DT_F32 = 2, DT_BF16 = 3 };
enum { ACC_PLAIN = 0, ACC_TWOSUM = 1 };
enum { OP_SUM = 0, OP_DOT = 1 };
enum { SH_IDX = 0, SH_UP = 1, SH_DOWN = 2, SH_XOR = 3 };

#define FULL 0xffffffffu
#define MAXW 32
#define MAXK 32

static __thread int t_err;
static void raise_err(int e) {
  if (!t_err) t_err = e;
}

/* ------------------------------------------------------------------ */
/* statement counters: the appendix invariant (every statement of the  */
/* input kernel runs once per thread; peeling conditions are extra)    */
/* ------------------------------------------------------------------ */
enum {
  ST_LOAD = 0,  /* per-thread load of the element */
  ST_SHFL,      /* per-thread shuffle-and-add of the warp tree */
  ST_VOTE,      /* per-thread ballot */
  ST_PEEL,      /* per-thread evaluation of a peeled branch condition */
  ST_BODY,      /* per-thread statement inside the peeled branch */
  ST_NUM
};
static __thread uint64_t t_cnt[ST_NUM];
#define CNT(s) (t_cnt[(s)]++)

void coxo_counts_reset(void) { memset(t_cnt, 0, sizeof t_cnt); }
int coxo_counts(uint64_t *out, int n) {
  for (int i = 0; i < n && i < ST_NUM; i++) out[i] = t_cnt[i];
  return ST_NUM;
}

/* ------------------------------------------------------------------ */
/* per-warp exchange array and the warp builtins                       */
/* ------------------------------------------------------------------ */
static const uint64_t POISON = 0xDEADBEEFDEADBEEFull;

typedef struct {
  uint64_t v[32];  /* operand bits supplied by each lane */
  uint32_t wrote;  /* lanes that supplied an operand since the last WAR barrier */
} xch_t;

static void xch_war(xch_t *x) {
  for (int l = 0; l < 32; l++) x->v[l] = POISON;
  x->wrote = 0;
}
static void xch_put(xch_t *x, int l, uint64_t bits) {
  x->v[l] = bits;
  x->wrote |= 1u << l;
}

/* a collective called by lane l with this mask is defined only if l is in
 * the mask and every lane of the mask has reached the call */
static int call_ok(const xch_t *x, int l, uint32_t mask) {
  if (!((mask >> l) & 1u) || (mask & ~x->wrote)) {
    raise_err(COXO_ERR_UB);
    return 0;
  }
  return 1;
}

/* source lane of a shuffle; the caller's own lane where CUDA returns the
 * caller's own value (b = first lane of the caller's width-segment) */
static int shfl_src(int op, int l, int arg, int w) {
  int b = l & ~(w - 1);
  switch (op) {
  case SH_IDX: return b + (arg & (w - 1));
  case SH_UP: return (l - b >= arg) ? l - arg : l;
  case SH_DOWN: return (l - b + arg < w) ? l + arg : l;
  case SH_XOR: {
    int j = l ^ arg; /* lanes of earlier segments are readable, later ones not */
    return (j < b + w) ? j : l;
  }
  }
  return l;
}

static uint64_t wf_shfl(const xch_t *x, int l, uint32_t mask, int op, int arg, int w) {
  if (!call_ok(x, l, mask)) return POISON;
  int j = shfl_src(op, l, arg, w);
  if (!((mask >> j) & 1u)) {
    raise_err(COXO_ERR_UB);
    return POISON;
  }
  return x->v[j];
}

/* votes: operands are predicate values, nonzero = true */
static uint32_t wf_ballot(const xch_t *x, int l, uint32_t mask) {
  if (!call_ok(x, l, mask)) return 0;
  uint32_t r = 0;
  for (int i = 0; i < 32; i++)
    if (((mask >> i) & 1u) && x->v[i] != 0) r |= 1u << i;
  return r;
}
static int wf_any(const xch_t *x, int l, uint32_t mask) { return wf_ballot(x, l, mask) != 0; }
static int wf_all(const xch_t *x, int l, uint32_t mask) {
  if (!call_ok(x, l, mask)) return 0;
  return wf_ballot(x, l, mask) == mask;
}

/* __match_any_sync: the lanes of the mask whose operand equals the
 * caller's; __match_all_sync: the mask if every lane of it holds the same
 * operand (pred = 1), else 0 (pred = 0) */
static uint32_t wf_match_any(const xch_t *x, int l, uint32_t mask) {
  if (!call_ok(x, l, mask)) return 0;
  uint32_t r = 0;
  for (int i = 0; i < 32; i++)
    if (((mask >> i) & 1u) && x->v[i] == x->v[l]) r |= 1u << i;
  return r;
}
static uint32_t wf_match_all(const xch_t *x, int l, uint32_t mask, int *pred) {
  *pred = 0;
  if (!call_ok(x, l, mask)) return 0;
  for (int i = 0; i < 32; i++)
    if (((mask >> i) & 1u) && x->v[i] != x->v[l]) return 0;
  *pred = 1;
  return mask;
}

/* __reduce_{add,min,max,and,or,xor}_sync over the lanes of the mask:
 * add / and / or / xor on unsigned operands (add wraps), min / max on
 * signed int operands */
enum { RD_ADD = 0, RD_MIN, RD_MAX, RD_AND, RD_OR, RD_XOR };
static uint32_t wf_reduce(const xch_t *x, int l, uint32_t mask, int op) {
  if (!call_ok(x, l, mask)) return 0;
  int first = 1;
  uint32_t r = 0;
  for (int i = 0; i < 32; i++) {
    if (!((mask >> i) & 1u)) continue;
    const uint32_t v = (uint32_t)x->v[i];
    if (first) {
      r = v;
      first = 0;
      continue;
    }
    switch (op) {
    case RD_ADD: r = r + v; break;
    case RD_MIN: r = (int32_t)v < (int32_t)r ? v : r; break;
    case RD_MAX: r = (int32_t)v > (int32_t)r ? v : r; break;
    case RD_AND: r &= v; break;
    case RD_OR: r |= v; break;
    case RD_XOR: r ^= v; break;
    }
  }
  return r;
}

/* loop peeling of a branch that encloses a barrier: every lane evaluated the
 * condition; it must agree across lanes; lane 0's outcome is followed */
static int peel(const int *flag, int nlanes) {
  for (int i = 1; i < nlanes; i++)
    if ((flag[i] != 0) != (flag[0] != 0)) raise_err(COXO_ERR_DIVERGENT);
  return flag[0] != 0;
}

/* bit helpers (value <-> operand bits) */
static uint64_t fbits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}
static float bitsf(uint64_t b) {
  uint32_t u = (uint32_t)b;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
static uint64_t dbits(double d) {
  uint64_t u;
  memcpy(&u, &d, 8);
  return u;
}
static double bitsd(uint64_t b) {
  double d;
  memcpy(&d, &b, 8);
  return d;
}
static uint64_t ibits(int32_t i) { return (uint32_t)i; }
static int32_t bitsi(uint64_t b) { return (int32_t)(uint32_t)b; }
/* CUDA int + lowers to a two's-complement wrapping add */
static int32_t wadd(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
static int popc32(uint32_t v) { return __builtin_popcount(v); }
static float bf16f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

/* ------------------------------------------------------------------ */
/* thread pool over blocks (one block per CPU thread at a time)        */
/* ------------------------------------------------------------------ */
static int g_threads = 1;

int coxo_set_threads(int n) {
  if (n <= 0) n = (int)sysconf(_SC_NPROCESSORS_ONLN);
  if (n < 1) n = 1;
  g_threads = n;
  return n;
}
int coxo_get_threads(void) { return g_threads; }

typedef void (*block_fn)(void *ctx, int64_t b);
typedef struct {
  block_fn fn;
  void *ctx;
  int64_t nblocks;
  int64_t next;
  int err;
} pool_job;

static void *pool_worker(void *p) {
  pool_job *j = (pool_job *)p;
  t_err = 0;
  for (;;) {
    int64_t b = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
    if (b >= j->nblocks) break;
    j->fn(j->ctx, b);
  }
  if (t_err) {
    int zero = 0;
    __atomic_compare_exchange_n(&j->err, &zero, t_err, 0, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
  }
  return NULL;
}

static int run_blocks(int64_t nblocks, block_fn fn, void *ctx) {
  int nt = g_threads;
  if (nblocks <= 0) return COXO_OK;
  if (nt > nblocks) nt = (int)nblocks;
  if (nt <= 1) {
    t_err = 0;
    for (int64_t b = 0; b < nblocks; b++) fn(ctx, b);
    return t_err;
  }
  pool_job job = {fn, ctx, nblocks, 0, 0};
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nt);
  if (!th) return COXO_ERR_NOMEM;
  pthread_attr_t attr;
  pthread_attr_init(&attr);
  pthread_attr_setstacksize(&attr, (size_t)16 << 20);
  int started = 0;
  for (int i = 0; i < nt; i++)
    if (pthread_create(&th[i], &attr, pool_worker, &job) == 0) started++;
    else break;
  pthread_attr_destroy(&attr);
  if (started == 0) {
    free(th);
    t_err = 0;
    for (int64_t b = 0; b < nblocks; b++) fn(ctx, b);
    return t_err;
  }
  for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
  free(th);
  return job.err;
}

static int sigma_ok(int k, int W) {
  return k >= 1 && k <= MAXK && (k & (k - 1)) == 0 && W >= 1 && W <= MAXW;
}
static int width_ok(int w) { return w >= 1 && w <= 32 && (w & (w - 1)) == 0; }

/* ================================================================== */
/* warp-function probes: one builtin applied to every 32-lane warp     */
/* ================================================================== */
typedef struct {
  const int32_t *v;
  int32_t *out;
  const int32_t *argv;
  int32_t arg;
  int op, width;
  const uint32_t *mask;
} shfl_ctx;

/* block b = one warp: lanes in mask[b] execute out = shfl_op(v, arg);
 * lanes outside the mask do not execute and copy their input */
static void shfl_block(void *p, int64_t g) {
  shfl_ctx *c = (shfl_ctx *)p;
  uint32_t m = c->mask ? c->mask[g] : FULL;
  xch_t X;
  xch_war(&X);
  for (int l = 0; l < 32; l++)
    if ((m >> l) & 1u) xch_put(&X, l, ibits(c->v[32 * g + l]));
  /* RAW warp barrier */
  for (int l = 0; l < 32; l++) {
    int64_t e = 32 * g + l;
    if ((m >> l) & 1u) {
      int a = c->argv ? c->argv[e] : c->arg;
      c->out[e] = bitsi(wf_shfl(&X, l, m, c->op, a, c->width));
    } else {
      c->out[e] = c->v[e];
    }
  }
  xch_war(&X); /* WAR warp barrier */
}

int coxo_warp_shfl(const int32_t *v, int32_t *out, int64_t n, int op, int32_t arg,
                   const int32_t *argv, int width, const uint32_t *mask) {
  if (n < 0 || n % 32 || !width_ok(width) || op < SH_IDX || op > SH_XOR) return COXO_ERR_INVALID;
  if (op != SH_IDX) {
    if (argv) {
      for (int64_t i = 0; i < n; i++)
        if (argv[i] < 0 || argv[i] > 31) return COXO_ERR_INVALID;
    } else if (arg < 0 || arg > 31) {
      return COXO_ERR_INVALID;
    }
  }
  shfl_ctx c = {v, out, argv, arg, op, width, mask};
  return run_blocks(n / 32, shfl_block, &c);
}

typedef struct {
  const int32_t *pred;
  const uint32_t *mask;
  uint32_t *ballot;
  int32_t *anyall;
} vote_ctx;

/* block g = one warp: lanes of mask[g] execute b = ballot(m, p),
 * a = any(m, p), l = all(m, p); the mask's lowest lane stores
 * ballot[g] = b and anyall[g] = a | l << 1; with an empty mask lane 0
 * stores zeros */
static void vote_block(void *p, int64_t g) {
  vote_ctx *c = (vote_ctx *)p;
  uint32_t m = c->mask ? c->mask[g] : FULL;
  xch_t X;
  xch_war(&X);
  uint32_t b[32];
  int a[32], al[32];
  for (int l = 0; l < 32; l++)
    if ((m >> l) & 1u) xch_put(&X, l, c->pred[32 * g + l] != 0);
  for (int l = 0; l < 32; l++)
    if ((m >> l) & 1u) {
      b[l] = wf_ballot(&X, l, m);
      a[l] = wf_any(&X, l, m);
      al[l] = wf_all(&X, l, m);
    }
  xch_war(&X);
  int lead = m ? __builtin_ctz(m) : 0;
  for (int l = 0; l < 32; l++) {
    if (l != lead) continue;
    if (m) {
      c->ballot[g] = b[l];
      c->anyall[g] = a[l] | (al[l] << 1);
    } else {
      c->ballot[g] = 0;
      c->anyall[g] = 0;
    }
  }
}

int coxo_warp_vote(const int32_t *pred, const uint32_t *mask, int64_t n, uint32_t *ballot,
                   int32_t *anyall) {
  if (n < 0 || n % 32) return COXO_ERR_INVALID;
  vote_ctx c = {pred, mask, ballot, anyall};
  return run_blocks(n / 32, vote_block, &c);
}

/* Tile-scoped votes of cooperative groups' thread_block_tile<T> (the
 * static groups of Sec. 2.2.2, with the votes of Sec. 2.2.1): a warp is
 * 32/T tiles of T consecutive lanes, each a whole group (no mask).  Every
 * lane supplies its predicate to the warp's exchange array; lane l of the
 * tile that starts at lane b reads the tile's T entries: tile.ballot has
 * bit i set iff lane b + i's predicate is nonzero, tile.any() is true iff
 * one is, tile.all() iff all T are.  The tile's rank-0 lane stores
 * ballot[tile] and anyall[tile] = any | all << 1. */
typedef struct {
  const int32_t *pred;
  int T;
  uint32_t *ballot;
  int32_t *anyall;
} tvote_ctx;

static uint32_t wf_tile_ballot(const xch_t *x, int l, int T) {
  const uint32_t tile = (T == 32 ? 0xFFFFFFFFu : ((1u << T) - 1u)) << (l - l % T);
  if (!call_ok(x, l, tile)) return 0;
  uint32_t r = 0;
  for (int i = 0; i < T; i++)
    if (x->v[l - l % T + i] != 0) r |= 1u << i;
  return r;
}

static void tvote_block(void *p, int64_t g) {
  tvote_ctx *c = (tvote_ctx *)p;
  const int T = c->T;
  const uint32_t full = T == 32 ? 0xFFFFFFFFu : (1u << T) - 1u;
  xch_t X;
  xch_war(&X);
  uint32_t b[32];
  int a[32], al[32];
  for (int l = 0; l < 32; l++) xch_put(&X, l, c->pred[32 * g + l] != 0);
  for (int l = 0; l < 32; l++) {
    b[l] = wf_tile_ballot(&X, l, T);
    a[l] = b[l] != 0;
    al[l] = b[l] == full;
  }
  xch_war(&X);
  for (int l = 0; l < 32; l += T) {
    c->ballot[(32 * g + l) / T] = b[l];
    c->anyall[(32 * g + l) / T] = a[l] | (al[l] << 1);
  }
}

int coxo_tile_vote(const int32_t *pred, int64_t n, int T, uint32_t *ballot, int32_t *anyall) {
  if (n < 0 || n % 32 || T < 1 || T > 32 || (T & (T - 1))) return COXO_ERR_INVALID;
  tvote_ctx c = {pred, T, ballot, anyall};
  return run_blocks(n / 32, tvote_block, &c);
}

/* ================================================================== */
/* K-R0: 256-thread blocks (8 warps), one element per thread:          */
/*   shfl_down tree (offsets 16..1) per warp, ballot(x > 0) per warp,  */
/*   shared-memory slot per warp, warp 0 combines the 8 slots.         */
/* ================================================================== */
typedef struct {
  const int32_t *x;
  int64_t n;
  int32_t *bsum;
  int32_t *wpos;
} r0_ctx;

static void r0_block(void *p, int64_t b) {
  r0_ctx *c = (r0_ctx *)p;
  enum { W = 8 };
  int32_t val[32 * W];
  int32_t slot[W];
  xch_t X;
  xch_war(&X);
  /* block region 1 */
  for (int w = 0; w < W; w++) {
    int pred[32];
    for (int l = 0; l < 32; l++) {
      int64_t e = b * 256 + 32 * w + l;
      CNT(ST_LOAD);
      val[32 * w + l] = e < c->n ? c->x[e] : 0;
      pred[l] = e < c->n && c->x[e] > 0;
    }
    for (int o = 16; o > 0; o >>= 1) {
      for (int l = 0; l < 32; l++) xch_put(&X, l, ibits(val[32 * w + l]));
      for (int l = 0; l < 32; l++) {
        CNT(ST_SHFL);
        val[32 * w + l] = wadd(val[32 * w + l], bitsi(wf_shfl(&X, l, FULL, SH_DOWN, o, 32)));
      }
      xch_war(&X);
    }
    uint32_t bal[32];
    for (int l = 0; l < 32; l++) xch_put(&X, l, (uint64_t)pred[l]);
    for (int l = 0; l < 32; l++) {
      CNT(ST_VOTE);
      bal[l] = wf_ballot(&X, l, FULL);
    }
    xch_war(&X);
    for (int l = 0; l < 32; l++) {
      if (l != 0) continue;
      int64_t g = b * W + w;
      if (32 * g < c->n) c->wpos[g] = popc32(bal[l]);
      slot[w] = val[32 * w];
    }
  }
  /* block barrier; block region 2: if (warp == 0) { tree over slots } */
  for (int w = 0; w < W; w++) {
    int flag[32];
    for (int l = 0; l < 32; l++) {
      CNT(ST_PEEL);
      flag[l] = (w == 0);
    }
    if (!peel(flag, 32)) continue;
    int32_t a[32];
    for (int l = 0; l < 32; l++) a[l] = l < W ? slot[l] : 0;
    for (int o = 16; o > 0; o >>= 1) {
      for (int l = 0; l < 32; l++) xch_put(&X, l, ibits(a[l]));
      for (int l = 0; l < 32; l++) {
        CNT(ST_BODY);
        a[l] = wadd(a[l], bitsi(wf_shfl(&X, l, FULL, SH_DOWN, o, 32)));
      }
      xch_war(&X);
    }
    for (int l = 0; l < 32; l++)
      if (l == 0) c->bsum[b] = a[0];
  }
}

int coxo_reduce_blocks_i32(const int32_t *x, int64_t n, int32_t *block_sums, int32_t *warp_pos) {
  if (n < 0) return COXO_ERR_INVALID;
  r0_ctx c = {x, n, block_sums, warp_pos};
  return run_blocks((n + 255) / 256, r0_block, &c);
}

/* ================================================================== */
/* element mapping of a chunk for schedule sigma = (k, W)              */
/*   T = 32W threads, S = T*k elements per chunk, V = min(k, 16 bytes  */
/*   / element size) elements per vector, R = k / V rows.  Thread      */
/*   (w, l) owns, for row i and vector slot v, chunk offset            */
/*       w*32k + (i*32 + l)*V + v                                      */
/*   and walks them in (i, v) order.  Offsets at or past the end of    */
/*   the data are padding: the additive identity (-0.0 for floats, 0   */
/*   for integers; a dot pads x with -0.0 and y with +0.0).            */
/* ================================================================== */
static int vec_of(int k, int dtype) {
  int v = dtype == DT_BF16 ? 8 : 4;
  return k < v ? k : v;
}
static int64_t chunk_off(int k, int V, int w, int i, int l, int v) {
  return (int64_t)w * 32 * k + ((int64_t)i * 32 + l) * V + v;
}

/* per-lane accumulator of the reductions */
typedef struct {
  float s, c;  /* sum (and compensation for ACC_TWOSUM) */
  int32_t i;   /* integer sum */
} lacc;

/* Knuth's TwoSum: s = fl(a + b) and e with a + b = s + e exactly */
static void two_sum(float a, float b, float *s, float *e) {
  float ss = a + b;
  float bb = ss - a;
  *e = (a - (ss - bb)) + (b - bb);
  *s = ss;
}

static float load_f(const void *x, int dt, int64_t e) {
  return dt == DT_BF16 ? bf16f(((const uint16_t *)x)[e]) : ((const float *)x)[e];
}

typedef struct {
  const void *x, *y; /* y only for dot */
  int dtype, op, acc;
  int k, W;
} red_kind;

/* one lane's step on one element (pads included) */
static void lane_step(const red_kind *rk, lacc *a, int64_t e, int64_t e1) {
  if (rk->dtype == DT_I32) {
    int32_t xv = e < e1 ? ((const int32_t *)rk->x)[e] : 0;
    a->i = wadd(a->i, xv);
    return;
  }
  float xv = e < e1 ? load_f(rk->x, rk->dtype, e) : -0.0f;
  if (rk->op == OP_SUM) {
    if (rk->acc == ACC_PLAIN) {
      a->s = a->s + xv;
    } else {
      float s, err;
      two_sum(a->s, xv, &s, &err);
      a->s = s;
      a->c = a->c + err;
    }
  } else {
    float yv = e < e1 ? load_f(rk->y, rk->dtype, e) : 0.0f;
    if (rk->acc == ACC_PLAIN) {
      a->s = fmaf(xv, yv, a->s);
    } else {
      float p = xv * yv;
      float pe = fmaf(xv, yv, -p); /* TwoProduct: p + pe = x*y exactly */
      float s, q;
      two_sum(a->s, p, &s, &q);
      a->s = s;
      a->c = a->c + (pe + q);
    }
  }
}

/* tree combine of own value a with the partner's b (own operand first) */
static lacc lane_combine(const red_kind *rk, lacc a, lacc b) {
  lacc r = a;
  if (rk->dtype == DT_I32) {
    r.i = wadd(a.i, b.i);
  } else if (rk->acc == ACC_PLAIN) {
    r.s = a.s + b.s;
  } else {
    float s, e;
    two_sum(a.s, b.s, &s, &e);
    r.s = s;
    r.c = (a.c + b.c) + e;
  }
  return r;
}

static lacc lacc_identity(void) {
  lacc a;
  a.s = -0.0f;
  a.c = -0.0f;
  a.i = 0;
  return a;
}

/* shfl_down tree (offsets 16, 8, 4, 2, 1) over one warp's 32 lanes of acc;
 * each component that the kind carries is one exchange round */
static void warp_tree(const red_kind *rk, lacc *acc /*[32]*/, xch_t *X) {
  for (int o = 16; o > 0; o >>= 1) {
    lacc part[32];
    for (int l = 0; l < 32; l++) part[l] = acc[l];
    if (rk->dtype == DT_I32) {
      for (int l = 0; l < 32; l++) xch_put(X, l, ibits(acc[l].i));
      for (int l = 0; l < 32; l++) part[l].i = bitsi(wf_shfl(X, l, FULL, SH_DOWN, o, 32));
      xch_war(X);
    } else {
      for (int l = 0; l < 32; l++) xch_put(X, l, fbits(acc[l].s));
      for (int l = 0; l < 32; l++) part[l].s = bitsf(wf_shfl(X, l, FULL, SH_DOWN, o, 32));
      xch_war(X);
      if (rk->acc == ACC_TWOSUM) {
        for (int l = 0; l < 32; l++) xch_put(X, l, fbits(acc[l].c));
        for (int l = 0; l < 32; l++) part[l].c = bitsf(wf_shfl(X, l, FULL, SH_DOWN, o, 32));
        xch_war(X);
      }
    }
    for (int l = 0; l < 32; l++) acc[l] = lane_combine(rk, acc[l], part[l]);
  }
}

/* Collapsed reduction of one chunk [e0, e0 + S) clipped at e1:
 *   block region 1: per warp, lane-serial accumulation (step a2), warp
 *     shfl_down tree (a3), lane 0 stores the warp's value in slot[w];
 *   block barrier;
 *   block region 2: warp 0 loads slot[l] for l < W (identity otherwise),
 *     runs the same tree, lane 0 holds the chunk partial (a5). */
static lacc reduce_chunk(const red_kind *rk, int64_t e0, int64_t e1) {
  const int k = rk->k, W = rk->W;
  const int V = vec_of(k, rk->dtype), R = k / V;
  lacc acc[32 * MAXW];
  lacc slot[MAXW];
  xch_t X;
  xch_war(&X);
  for (int w = 0; w < W; w++) {
    for (int l = 0; l < 32; l++) {
      lacc a = lacc_identity();
      for (int i = 0; i < R; i++)
        for (int v = 0; v < V; v++) lane_step(rk, &a, e0 + chunk_off(k, V, w, i, l, v), e1);
      acc[32 * w + l] = a;
    }
    warp_tree(rk, &acc[32 * w], &X);
    for (int l = 0; l < 32; l++)
      if (l == 0) slot[w] = acc[32 * w];
  }
  lacc res = lacc_identity();
  for (int w = 0; w < W; w++) {
    int flag[32];
    for (int l = 0; l < 32; l++) flag[l] = (w == 0);
    if (!peel(flag, 32)) continue;
    lacc a[32];
    for (int l = 0; l < 32; l++) a[l] = l < W ? slot[l] : lacc_identity();
    warp_tree(rk, a, &X);
    res = a[0];
  }
  return res;
}

/* chunk partial as a double for the FP64 final combine */
static double partial_f64(const red_kind *rk, lacc a) {
  if (rk->acc == ACC_TWOSUM) return (double)a.s + (double)a.c;
  return (double)a.s;
}

typedef struct {
  red_kind rk;
  int64_t n, S;
  lacc *part;
} red_ctx;

static void red_block(void *p, int64_t c) {
  red_ctx *r = (red_ctx *)p;
  r->part[c] = reduce_chunk(&r->rk, c * r->S, r->n);
}

/* FP64 final combine over nch chunk values (step a6), a fixed tree with the
 * shape of one 256-thread block: thread j sums values j, j+256, j+512, ...
 * serially from -0.0; each of the 8 warps runs the shfl_down tree (offsets
 * 16..1) in FP64; warp 0 runs the tree again over the 8 warp results
 * (lanes 8..31 hold -0.0); lane 0 holds the total. */
static double final_f64(const double *val, int64_t nch) {
  enum { F = 256, FW = 8 };
  double t[F];
  double slot[FW];
  xch_t X;
  xch_war(&X);
  for (int w = 0; w < FW; w++) {
    for (int l = 0; l < 32; l++) {
      double s = -0.0;
      for (int64_t c = 32 * w + l; c < nch; c += F) s = s + val[c];
      t[32 * w + l] = s;
    }
    for (int o = 16; o > 0; o >>= 1) {
      for (int l = 0; l < 32; l++) xch_put(&X, l, dbits(t[32 * w + l]));
      for (int l = 0; l < 32; l++)
        t[32 * w + l] = t[32 * w + l] + bitsd(wf_shfl(&X, l, FULL, SH_DOWN, o, 32));
      xch_war(&X);
    }
    slot[w] = t[32 * w];
  }
  double a[32];
  for (int l = 0; l < 32; l++) a[l] = l < FW ? slot[l] : -0.0;
  for (int o = 16; o > 0; o >>= 1) {
    for (int l = 0; l < 32; l++) xch_put(&X, l, dbits(a[l]));
    for (int l = 0; l < 32; l++) a[l] = a[l] + bitsd(wf_shfl(&X, l, FULL, SH_DOWN, o, 32));
    xch_war(&X);
  }
  return a[0];
}

/* reduce / dot over n elements with schedule (k, W).
 *   partials (nullable): per chunk; int32 for I32, float for plain FP,
 *     float pairs (s, c) for TWOSUM.
 *   total: int64 = sum of the int32 chunk partials (I32), or the FP64
 *     final combine (F32 / BF16). */
static int reduce_any(const void *x, const void *y, int dtype, int op, int64_t n, int acc, int k,
                      int W, void *partials, void *total) {
  if (n < 0 || !sigma_ok(k, W) || (acc != ACC_PLAIN && acc != ACC_TWOSUM)) return COXO_ERR_INVALID;
  if (dtype != DT_I32 && dtype != DT_F32 && dtype != DT_BF16) return COXO_ERR_DTYPE;
  if (dtype == DT_I32 && (acc != ACC_PLAIN || op != OP_SUM)) return COXO_ERR_DTYPE;
  const int64_t S = (int64_t)32 * W * k;
  const int64_t nch = (n + S - 1) / S;
  red_ctx r;
  r.rk.x = x;
  r.rk.y = y;
  r.rk.dtype = dtype;
  r.rk.op = op;
  r.rk.acc = acc;
  r.rk.k = k;
  r.rk.W = W;
  r.n = n;
  r.S = S;
  r.part = (lacc *)malloc(sizeof(lacc) * (size_t)(nch ? nch : 1));
  if (!r.part) return COXO_ERR_NOMEM;
  int err = run_blocks(nch, red_block, &r);
  if (dtype == DT_I32) {
    int64_t tot = 0;
    for (int64_t c = 0; c < nch; c++) {
      tot += (int64_t)r.part[c].i;
      if (partials) ((int32_t *)partials)[c] = r.part[c].i;
    }
    *(int64_t *)total = tot;
  } else {
    double *val = (double *)malloc(sizeof(double) * (size_t)(nch ? nch : 1));
    if (!val) {
      free(r.part);
      return COXO_ERR_NOMEM;
    }
    for (int64_t c = 0; c < nch; c++) {
      val[c] = partial_f64(&r.rk, r.part[c]);
      if (partials) {
        if (acc == ACC_TWOSUM) {
          ((float *)partials)[2 * c] = r.part[c].s;
          ((float *)partials)[2 * c + 1] = r.part[c].c;
        } else {
          ((float *)partials)[c] = r.part[c].s;
        }
      }
    }
    *(double *)total = final_f64(val, nch);
    free(val);
  }
  free(r.part);
  return err;
}

int coxo_reduce(const void *x, int dtype, int64_t n, int acc, int k, int W, void *partials,
                void *total) {
  return reduce_any(x, NULL, dtype, OP_SUM, n, acc, k, W, partials, total);
}

int coxo_dot(const void *a, const void *b, int dtype, int64_t n, int acc, int k, int W,
             void *partials, double *total) {
  if (dtype != DT_F32 && dtype != DT_BF16) return COXO_ERR_DTYPE;
  return reduce_any(a, b, dtype, OP_DOT, n, acc, k, W, partials, total);
}

/* ================================================================== */
/* chunk scan (steps a2, a3, a5): values q of the chunk-local inclusive */
/* scan, for int32 (wrapping) or binary32.                              */
/*   Per thread and row i: z_v = serial inclusive prefix of its V       */
/*   elements; r = z_{V-1}.  Per row, the warp scans r with             */
/*       for d in 1,2,4,8: t = shfl_up(r, d, 16); if ((l & 15) >= d)    */
/*           r = r + t;                                                 */
/*       t = shfl(r, 15, 32); if (l >= 16) r = r + t;                   */
/*   then ex = shfl_up(r, 1, 32) (used for l >= 1) and the row total    */
/*   rt = shfl(r, 31, 32).  The warp carry before row i is              */
/*   C_0 = none, C_{i+1} = C_i + rt_i (C_1 = rt_0).  Lane 0 stores the  */
/*   warp total C_R in slot[w]; block barrier; warp 0 scans the slots   */
/*   with the same tree and keeps E_w = shfl_up(., 1, 32) for w >= 1;  */
/*   block barrier; the element value is                                */
/*       q = ((E_w + C_i) + ex) + z_v                                   */
/*   evaluated left to right with absent terms (w = 0, i = 0, l = 0)    */
/*   skipped.                                                           */
/* ================================================================== */
typedef union {
  int32_t i;
  float f;
} sval;

static sval sadd(int isf, sval a, sval b) {
  sval r;
  if (isf) r.f = a.f + b.f;
  else r.i = wadd(a.i, b.i);
  return r;
}
static uint64_t sbits(int isf, sval a) { return isf ? fbits(a.f) : ibits(a.i); }
static sval bitss(int isf, uint64_t b) {
  sval r;
  if (isf) r.f = bitsf(b);
  else r.i = bitsi(b);
  return r;
}
static sval sident(int isf) {
  sval r;
  if (isf) r.f = -0.0f;
  else r.i = 0;
  return r;
}

/* 32-lane scan with the tree documented above; r[l] becomes inclusive,
 * ex[l] the exclusive value (valid for l >= 1), returns lane 31's total */
static sval warp_scan32(int isf, sval *r, sval *ex, xch_t *X) {
  for (int d = 1; d <= 8; d <<= 1) {
    sval t[32];
    for (int l = 0; l < 32; l++) xch_put(X, l, sbits(isf, r[l]));
    for (int l = 0; l < 32; l++) t[l] = bitss(isf, wf_shfl(X, l, FULL, SH_UP, d, 16));
    xch_war(X);
    for (int l = 0; l < 32; l++)
      if ((l & 15) >= d) r[l] = sadd(isf, r[l], t[l]);
  }
  {
    sval t[32];
    for (int l = 0; l < 32; l++) xch_put(X, l, sbits(isf, r[l]));
    for (int l = 0; l < 32; l++) t[l] = bitss(isf, wf_shfl(X, l, FULL, SH_IDX, 15, 32));
    xch_war(X);
    for (int l = 0; l < 32; l++)
      if (l >= 16) r[l] = sadd(isf, r[l], t[l]);
  }
  sval tot[32];
  for (int l = 0; l < 32; l++) xch_put(X, l, sbits(isf, r[l]));
  for (int l = 0; l < 32; l++) {
    ex[l] = bitss(isf, wf_shfl(X, l, FULL, SH_UP, 1, 32));
    tot[l] = bitss(isf, wf_shfl(X, l, FULL, SH_IDX, 31, 32));
  }
  xch_war(X);
  return tot[0];
}

typedef struct {
  int isf;        /* binary32 values, else int32 */
  const void *x;  /* input */
  int k, W;
} scan_kind;

static sval load_s(const scan_kind *sk, int64_t e, int64_t e1) {
  sval r;
  if (sk->isf) r.f = e < e1 ? ((const float *)sk->x)[e] : -0.0f;
  else r.i = e < e1 ? ((const int32_t *)sk->x)[e] : 0;
  return r;
}

/* writes q for every valid offset of chunk [e0, e0+S) (clipped at e1) into
 * q_out[e - e0] and returns the chunk total (q of the chunk's last slot) */
static sval scan_chunk(const scan_kind *sk, int64_t e0, int64_t e1, sval *q_out) {
  const int isf = sk->isf, k = sk->k, W = sk->W;
  const int V = vec_of(k, isf ? DT_F32 : DT_I32), R = k / V;
  const int64_t S = (int64_t)32 * W * k;
  sval *z = (sval *)malloc(sizeof(sval) * (size_t)S);        /* [T][R][V] */
  sval *ex = (sval *)malloc(sizeof(sval) * (size_t)(32 * W * R)); /* [T][R] */
  sval *carry = (sval *)malloc(sizeof(sval) * (size_t)(W * R));   /* [W][R] */
  sval slot[MAXW], ew[MAXW];
  sval total = sident(isf);
  if (!z || !ex || !carry) {
    raise_err(COXO_ERR_NOMEM);
    free(z);
    free(ex);
    free(carry);
    return total;
  }
  xch_t X;
  xch_war(&X);
  /* block region 1 */
  for (int w = 0; w < W; w++) {
    sval r[R][32];
    for (int l = 0; l < 32; l++) {
      int t = 32 * w + l;
      for (int i = 0; i < R; i++) {
        sval acc = sident(isf);
        for (int v = 0; v < V; v++) {
          sval xv = load_s(sk, e0 + chunk_off(k, V, w, i, l, v), e1);
          acc = v == 0 ? xv : sadd(isf, acc, xv);
          z[((int64_t)t * R + i) * V + v] = acc;
        }
        r[i][l] = acc;
      }
    }
    sval c = sident(isf);
    for (int i = 0; i < R; i++) {
      sval exr[32];
      sval rt = warp_scan32(isf, r[i], exr, &X);
      for (int l = 0; l < 32; l++) ex[(32 * w + l) * R + i] = exr[l];
      carry[w * R + i] = c; /* meaningful for i >= 1 */
      c = i == 0 ? rt : sadd(isf, c, rt);
    }
    for (int l = 0; l < 32; l++)
      if (l == 0) slot[w] = c;
  }
  /* block barrier; block region 2: warp 0 scans the warp totals */
  for (int w = 0; w < W; w++) {
    int flag[32];
    for (int l = 0; l < 32; l++) flag[l] = (w == 0);
    if (!peel(flag, 32)) continue;
    sval a[32], exw[32];
    for (int l = 0; l < 32; l++) a[l] = l < W ? slot[l] : sident(isf);
    warp_scan32(isf, a, exw, &X);
    for (int l = 0; l < 32; l++)
      if (l < W) ew[l] = exw[l];
  }
  /* block barrier; block region 3: element values */
  for (int w = 0; w < W; w++)
    for (int l = 0; l < 32; l++) {
      int t = 32 * w + l;
      for (int i = 0; i < R; i++)
        for (int v = 0; v < V; v++) {
          int have = 0;
          sval q = sident(isf);
          if (w >= 1) {
            q = ew[w];
            have = 1;
          }
          if (i >= 1) {
            q = have ? sadd(isf, q, carry[w * R + i]) : carry[w * R + i];
            have = 1;
          }
          if (l >= 1) {
            sval e = ex[t * R + i];
            q = have ? sadd(isf, q, e) : e;
            have = 1;
          }
          sval zz = z[((int64_t)t * R + i) * V + v];
          q = have ? sadd(isf, q, zz) : zz;
          int64_t off = chunk_off(k, V, w, i, l, v);
          if (e0 + off < e1) q_out[off] = q;
          if (w == W - 1 && l == 31 && i == R - 1 && v == V - 1) total = q;
        }
    }
  free(z);
  free(ex);
  free(carry);
  return total;
}

/* flat int32 inclusive scan: y_e = (sum_{j<=e} x_j) mod 2^32.  The chunk
 * carry is plain integer addition in chunk order. */
typedef struct {
  scan_kind sk;
  int64_t n, S;
  int32_t *y;
  int32_t *ctot; /* per chunk totals */
  const int32_t *carry;
} scan_ctx;

static void scan_pass1(void *p, int64_t c) {
  scan_ctx *s = (scan_ctx *)p;
  int64_t e0 = c * s->S;
  sval *q = (sval *)malloc(sizeof(sval) * (size_t)s->S);
  if (!q) {
    raise_err(COXO_ERR_NOMEM);
    return;
  }
  sval tot = scan_chunk(&s->sk, e0, s->n, q);
  for (int64_t o = 0; o < s->S && e0 + o < s->n; o++) s->y[e0 + o] = q[o].i;
  s->ctot[c] = tot.i;
  free(q);
}
static void scan_pass2(void *p, int64_t c) {
  scan_ctx *s = (scan_ctx *)p;
  int64_t e0 = c * s->S;
  int32_t cr = s->carry[c];
  for (int64_t o = 0; o < s->S && e0 + o < s->n; o++) s->y[e0 + o] = wadd(cr, s->y[e0 + o]);
}

int coxo_scan_i32(const int32_t *x, int32_t *y, int64_t n, int k, int W) {
  if (n < 0 || !sigma_ok(k, W)) return COXO_ERR_INVALID;
  const int64_t S = (int64_t)32 * W * k, nch = (n + S - 1) / S;
  scan_ctx s;
  s.sk.isf = 0;
  s.sk.x = x;
  s.sk.k = k;
  s.sk.W = W;
  s.n = n;
  s.S = S;
  s.y = y;
  s.ctot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nch + 1));
  int32_t *carry = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nch + 1));
  if (!s.ctot || !carry) {
    free(s.ctot);
    free(carry);
    return COXO_ERR_NOMEM;
  }
  int err = run_blocks(nch, scan_pass1, &s);
  int32_t run = 0;
  for (int64_t c = 0; c < nch; c++) {
    carry[c] = run;
    run = wadd(run, s.ctot[c]);
  }
  s.carry = carry;
  int err2 = run_blocks(nch, scan_pass2, &s);
  free(s.ctot);
  free(carry);
  return err ? err : err2;
}

/* ================================================================== */
/* ballot compaction of one chunk (keep x > 0, stable).                 */
/*   Per thread, row i, slot v: p = (x > 0).  Per row the warp takes    */
/*   B_v = ballot(FULL, p_v) for v = 0..V-1; the rank of (l, v) in the  */
/*   row is sum_v' popc(B_v' & lanemask_lt(l)) + sum_{v'<v} p_{l,v'};   */
/*   the row count is sum_v popc(B_v).  Warp counts go to slot[w]; the  */
/*   block exclusive scan of the slots gives warp offsets.              */
/* ================================================================== */
typedef struct {
  int isf;
  const void *x;
  int k, W;
} cmp_kind;

static int pos_pred(const cmp_kind *ck, int64_t e, int64_t e1) {
  if (e >= e1) return 0;
  return ck->isf ? (((const float *)ck->x)[e] > 0.0f) : (((const int32_t *)ck->x)[e] > 0);
}

/* returns the chunk's kept count; if dst is non-NULL writes the kept
 * elements at dst[rank] (element type of x) */
static int64_t compact_chunk(const cmp_kind *ck, int64_t e0, int64_t e1, void *dst) {
  const int k = ck->k, W = ck->W;
  const int V = vec_of(k, ck->isf ? DT_F32 : DT_I32), R = k / V;
  int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)(32 * W * k));
  int64_t slot[MAXW], woff[MAXW];
  if (!rank) {
    raise_err(COXO_ERR_NOMEM);
    return 0;
  }
  xch_t X;
  xch_war(&X);
  for (int w = 0; w < W; w++) {
    int64_t run = 0; /* warp-uniform running count over rows */
    for (int i = 0; i < R; i++) {
      uint32_t B[8];
      int p[32][8];
      for (int l = 0; l < 32; l++)
        for (int v = 0; v < V; v++) p[l][v] = pos_pred(ck, e0 + chunk_off(k, V, w, i, l, v), e1);
      for (int v = 0; v < V; v++) {
        uint32_t b[32];
        for (int l = 0; l < 32; l++) xch_put(&X, l, (uint64_t)p[l][v]);
        for (int l = 0; l < 32; l++) b[l] = wf_ballot(&X, l, FULL);
        xch_war(&X);
        B[v] = b[0];
      }
      int64_t rowcnt = 0;
      for (int v = 0; v < V; v++) rowcnt += popc32(B[v]);
      for (int l = 0; l < 32; l++) {
        uint32_t lt = (l == 0) ? 0u : (FULL >> (32 - l));
        int64_t base = 0;
        for (int v = 0; v < V; v++) base += popc32(B[v] & lt);
        int64_t own = 0;
        for (int v = 0; v < V; v++) {
          int64_t off = chunk_off(k, V, w, i, l, v);
          rank[off] = p[l][v] ? run + base + own : -1;
          own += p[l][v];
        }
      }
      run += rowcnt;
    }
    slot[w] = run;
  }
  /* block barrier; exclusive scan of warp counts (integer, any order) */
  int64_t tot = 0;
  for (int w = 0; w < W; w++) {
    woff[w] = tot;
    tot += slot[w];
  }
  if (dst) {
    for (int w = 0; w < W; w++)
      for (int l = 0; l < 32; l++)
        for (int i = 0; i < R; i++)
          for (int v = 0; v < V; v++) {
            int64_t off = chunk_off(k, V, w, i, l, v);
            if (rank[off] < 0) continue;
            int64_t r = woff[w] + rank[off];
            if (ck->isf) ((float *)dst)[r] = ((const float *)ck->x)[e0 + off];
            else ((int32_t *)dst)[r] = ((const int32_t *)ck->x)[e0 + off];
          }
  }
  free(rank);
  return tot;
}

typedef struct {
  cmp_kind ck;
  int64_t n, S;
  int64_t *cnt;
  const int64_t *off;
  int32_t *out;
} cmp_ctx;

static void cmp_pass1(void *p, int64_t c) {
  cmp_ctx *s = (cmp_ctx *)p;
  s->cnt[c] = compact_chunk(&s->ck, c * s->S, s->n, NULL);
}
static void cmp_pass2(void *p, int64_t c) {
  cmp_ctx *s = (cmp_ctx *)p;
  compact_chunk(&s->ck, c * s->S, s->n, s->out + s->off[c]);
}

int coxo_compact_i32(const int32_t *x, int64_t n, int32_t *out, int64_t *count, int k, int W) {
  if (n < 0 || !sigma_ok(k, W)) return COXO_ERR_INVALID;
  const int64_t S = (int64_t)32 * W * k, nch = (n + S - 1) / S;
  cmp_ctx s;
  s.ck.isf = 0;
  s.ck.x = x;
  s.ck.k = k;
  s.ck.W = W;
  s.n = n;
  s.S = S;
  s.out = out;
  s.cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nch + 1));
  int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nch + 1));
  if (!s.cnt || !off) {
    free(s.cnt);
    free(off);
    return COXO_ERR_NOMEM;
  }
  int err = run_blocks(nch, cmp_pass1, &s);
  int64_t run = 0;
  for (int64_t c = 0; c < nch; c++) {
    off[c] = run;
    run += s.cnt[c];
  }
  s.off = off;
  int err2 = run_blocks(nch, cmp_pass2, &s);
  *count = run;
  free(s.cnt);
  free(off);
  return err ? err : err2;
}

/* ================================================================== */
/* tile sort: each group of G keys (one per lane of a width-G tile)     */
/* sorted ascending as unsigned by the bitonic network                   */
/*   for k2 = 2, 4, .., G: for j = k2/2 .. 1:                            */
/*     o = shfl_xor(key, j, G); asc = ((lt & k2) == 0);                  */
/*     lower = ((lt & j) == 0); key = (lower == asc) ? min : max         */
/* (lt = lane within the tile).  A partial last group is padded with     */
/* UINT32_MAX, which sorts last and is not written.                      */
/* ================================================================== */
typedef struct {
  const uint32_t *keys;
  uint32_t *out;
  int64_t n;
  int G;
} sort_ctx;

static void sort_block(void *p, int64_t g) {
  sort_ctx *c = (sort_ctx *)p;
  const int G = c->G;
  uint32_t key[32];
  xch_t X;
  xch_war(&X);
  for (int l = 0; l < 32; l++) {
    int64_t e = 32 * g + l;
    key[l] = e < c->n ? c->keys[e] : 0xffffffffu;
  }
  for (int k2 = 2; k2 <= G; k2 <<= 1)
    for (int j = k2 >> 1; j > 0; j >>= 1) {
      uint32_t o[32];
      for (int l = 0; l < 32; l++) xch_put(&X, l, key[l]);
      for (int l = 0; l < 32; l++) o[l] = (uint32_t)wf_shfl(&X, l, FULL, SH_XOR, j, G);
      xch_war(&X);
      for (int l = 0; l < 32; l++) {
        int lt = l & (G - 1);
        int asc = (lt & k2) == 0, lower = (lt & j) == 0;
        uint32_t mn = key[l] < o[l] ? key[l] : o[l];
        uint32_t mx = key[l] < o[l] ? o[l] : key[l];
        key[l] = (lower == asc) ? mn : mx;
      }
    }
  for (int l = 0; l < 32; l++) {
    int64_t e = 32 * g + l;
    if (e < c->n) c->out[e] = key[l];
  }
}

int coxo_tile_sort_u32(const uint32_t *keys, uint32_t *out, int64_t n, int G) {
  if (n < 0 || G < 2 || !width_ok(G)) return COXO_ERR_INVALID;
  sort_ctx c = {keys, out, n, G};
  return run_blocks((n + 31) / 32, sort_block, &c);
}

/* group sort for groups larger than a warp (64 .. 4096 keys, sorted on the
 * GPU by a network whose wider exchanges cross the two halves of a wave or
 * go through shared memory): every group of G consecutive keys (a partial
 * last group: its valid keys) ascending as unsigned.  The result is unique,
 * so the oracle is the plain definition: a bottom-up merge sort per group. */
typedef struct {
  const uint32_t *keys;
  uint32_t *out;
  int64_t n;
  int G;
} gs_ctx;

static void gs_block(void *p, int64_t g) {
  gs_ctx *c = (gs_ctx *)p;
  const int64_t e0 = (int64_t)c->G * g;
  const int m = (int)(c->n - e0 < c->G ? c->n - e0 : c->G);
  uint32_t a[4096], b[4096];
  memcpy(a, c->keys + e0, (size_t)m * 4);
  uint32_t *src = a, *dst = b;
  for (int w = 1; w < m; w *= 2) {
    for (int lo = 0; lo < m; lo += 2 * w) {
      const int mid = lo + w < m ? lo + w : m, hi = lo + 2 * w < m ? lo + 2 * w : m;
      int i = lo, j = mid, k = lo;
      while (i < mid && j < hi) dst[k++] = src[i] <= src[j] ? src[i++] : src[j++];
      while (i < mid) dst[k++] = src[i++];
      while (j < hi) dst[k++] = src[j++];
    }
    uint32_t *t = src;
    src = dst;
    dst = t;
  }
  memcpy(c->out + e0, src, (size_t)m * 4);
}

int coxo_group_sort_u32(const uint32_t *keys, uint32_t *out, int64_t n, int G) {
  if (n < 0 || G < 2 || G > 4096 || (G & (G - 1))) return COXO_ERR_INVALID;
  gs_ctx c = {keys, out, n, G};
  return run_blocks((n + G - 1) / G, gs_block, &c);
}

/* key-value tile sort: every group of 32 consecutive (key, value) pairs
 * (a partial last group: its valid pairs) in ascending unsigned key order,
 * pairs with equal keys in their original order (a stable sort: sorting by
 * (key, position in the group), which makes the result unique).  The plain
 * definition, by insertion sort. */
typedef struct {
  const uint32_t *keys, *vals;
  uint32_t *ok, *ov;
  int64_t n;
} kv_ctx;

static void kv_block(void *p, int64_t g) {
  kv_ctx *c = (kv_ctx *)p;
  const int64_t e0 = 32 * g;
  const int m = (int)(c->n - e0 < 32 ? c->n - e0 : 32);
  uint32_t k[32], v[32];
  for (int i = 0; i < m; i++) {
    uint32_t kk = c->keys[e0 + i], vv = c->vals[e0 + i];
    int j = i;
    while (j > 0 && k[j - 1] > kk) {
      k[j] = k[j - 1];
      v[j] = v[j - 1];
      j--;
    }
    k[j] = kk;
    v[j] = vv;
  }
  for (int i = 0; i < m; i++) {
    c->ok[e0 + i] = k[i];
    c->ov[e0 + i] = v[i];
  }
}

int coxo_tile_sort_kv_u32(const uint32_t *keys, const uint32_t *vals, uint32_t *out_keys, uint32_t *out_vals,
                          int64_t n) {
  if (n < 0) return COXO_ERR_INVALID;
  kv_ctx c = {keys, vals, out_keys, out_vals, n};
  return run_blocks((n + 31) / 32, kv_block, &c);
}

/* ================================================================== */
/* tile<T> reduce: out[g] = wrap32 sum of x[gT .. gT+T-1] (zero pads)   */
/*   via tile.shfl_down(v, o) with o = T/2 .. 1 (width T); the tile's   */
/*   first lane stores.                                                 */
/* ================================================================== */
typedef struct {
  const int32_t *x;
  int64_t n;
  int T;
  int32_t *out;
} tred_ctx;

static void tred_block(void *p, int64_t g) {
  tred_ctx *c = (tred_ctx *)p;
  const int T = c->T;
  int32_t v[32];
  xch_t X;
  xch_war(&X);
  for (int l = 0; l < 32; l++) {
    int64_t e = 32 * g + l;
    v[l] = e < c->n ? c->x[e] : 0;
  }
  for (int o = T >> 1; o > 0; o >>= 1) {
    for (int l = 0; l < 32; l++) xch_put(&X, l, ibits(v[l]));
    for (int l = 0; l < 32; l++) v[l] = wadd(v[l], bitsi(wf_shfl(&X, l, FULL, SH_DOWN, o, T)));
    xch_war(&X);
  }
  for (int l = 0; l < 32; l++) {
    int64_t e = 32 * g + l;
    if ((l & (T - 1)) == 0 && e < c->n) c->out[e / T] = v[l];
  }
}

int coxo_tile_reduce_i32(const int32_t *x, int64_t n, int T, int32_t *out) {
  if (n < 0 || !width_ok(T) || T < 2) return COXO_ERR_INVALID;
  tred_ctx c = {x, n, T, out};
  return run_blocks((n + 31) / 32, tred_block, &c);
}

/* ================================================================== */
/* masked warp operations (divergent code; masks from a predicate).     */
/* For lane l of warp g (element e = 32g + l):                           */
/*   p = ((uint32)x & 1023) < D;  m = ballot(FULL, p);                   */
/*   if (p) {            // active lanes = m                             */
/*     b  = ballot(m, x > 0);                                            */
/*     A  = any(m, ((x >> 10) & 31) == 0);                               */
/*     L  = all(m, ((x >> 15) & 31) != 0);                               */
/*     src = next lane of m above l, wrapping to m's lowest lane;        */
/*     s  = shfl(m, x, src);  ld = ffs(m) - 1;  bc = shfl(m, x, ld);     */
/*     out[e] = s;  lane ld stores rec[g] = {m, b, A | L << 1, bc};      */
/*   } else out[e] = INT32_MIN;                                          */
/*   with m == 0 lane 0 stores rec[g] = {0, 0, 0, 0}.                    */
/* ================================================================== */
typedef struct {
  const int32_t *x;
  int D;
  int32_t *out;
  uint32_t *rec;
} mask_ctx;

static void mask_block(void *p, int64_t g) {
  mask_ctx *c = (mask_ctx *)p;
  const int32_t *x = c->x + 32 * g;
  int pr[32];
  uint32_t m[32];
  xch_t X;
  xch_war(&X);
  for (int l = 0; l < 32; l++) pr[l] = ((uint32_t)x[l] & 1023u) < (uint32_t)c->D;
  for (int l = 0; l < 32; l++) xch_put(&X, l, (uint64_t)pr[l]);
  for (int l = 0; l < 32; l++) m[l] = wf_ballot(&X, l, FULL);
  xch_war(&X);
  /* divergent branch (no barrier inside it encloses all lanes): the
   * intra-warp loops run only the lanes whose predicate holds */
  uint32_t b[32];
  int A[32], L[32];
  int32_t s[32], bc[32];
  for (int l = 0; l < 32; l++)
    if (pr[l]) xch_put(&X, l, (uint64_t)(x[l] > 0));
  for (int l = 0; l < 32; l++)
    if (pr[l]) b[l] = wf_ballot(&X, l, m[l]);
  xch_war(&X);
  for (int l = 0; l < 32; l++)
    if (pr[l]) xch_put(&X, l, (uint64_t)(((x[l] >> 10) & 31) == 0));
  for (int l = 0; l < 32; l++)
    if (pr[l]) A[l] = wf_any(&X, l, m[l]);
  xch_war(&X);
  for (int l = 0; l < 32; l++)
    if (pr[l]) xch_put(&X, l, (uint64_t)(((x[l] >> 15) & 31) != 0));
  for (int l = 0; l < 32; l++)
    if (pr[l]) L[l] = wf_all(&X, l, m[l]);
  xch_war(&X);
  for (int l = 0; l < 32; l++)
    if (pr[l]) xch_put(&X, l, ibits(x[l]));
  for (int l = 0; l < 32; l++)
    if (pr[l]) {
      uint32_t above = (l == 31) ? 0u : (m[l] & (FULL << (l + 1)));
      int src = above ? __builtin_ctz(above) : __builtin_ctz(m[l]);
      int ld = __builtin_ffs((int)m[l]) - 1;
      s[l] = bitsi(wf_shfl(&X, l, m[l], SH_IDX, src, 32));
      bc[l] = bitsi(wf_shfl(&X, l, m[l], SH_IDX, ld, 32));
    }
  xch_war(&X);
  for (int l = 0; l < 32; l++) {
    int64_t e = 32 * g + l;
    if (pr[l]) {
      c->out[e] = s[l];
      int ld = __builtin_ffs((int)m[l]) - 1;
      if (l == ld) {
        uint32_t *r = c->rec + 4 * g;
        r[0] = m[l];
        r[1] = b[l];
        r[2] = (uint32_t)(A[l] | (L[l] << 1));
        r[3] = (uint32_t)bc[l];
      }
    } else {
      c->out[e] = INT32_MIN;
    }
    if (l == 0 && m[l] == 0) {
      uint32_t *r = c->rec + 4 * g;
      r[0] = r[1] = r[2] = r[3] = 0;
    }
  }
}

int coxo_warp_masked(const int32_t *x, int64_t n, int D, int32_t *out, uint32_t *rec) {
  if (n < 0 || n % 32 || D < 0 || D > 1024) return COXO_ERR_INVALID;
  mask_ctx c = {x, D, out, rec};
  return run_blocks(n / 32, mask_block, &c);
}

/* ================================================================== */
/* dynamic groups: the lanes whose predicate holds form, inside the     */
/* divergent branch, the group coalesced_threads() returns (the dynamic */
/* cooperative group the paper's Table 1 lists as unsupported by COX,   */
/* filter_arr; Sec. 2.2.2-2.2.3).  Lane l of warp g, x = x[32g + l]:     */
/*   p = ((uint32)x & 1023) < D;                                         */
/*   if (p) { grp = coalesced_threads();  m = activemask();             */
/*     rank[e] = grp.thread_rank();  key = ((uint32)x >> 10) & 7;        */
/*     mm[e] = __match_any_sync(m, key);                                 */
/*     ma = __match_all_sync(m, key, &pred);                             */
/*     the six __reduce_*_sync(m, .) of x (add of x & 0xffff);           */
/*     filter: the rank-0 lane adds grp.size() to the counter, the base  */
/*     comes back by grp.shfl(base, 0), out[base + rank] = x;           */
/*     the rank-0 lane writes rec[g] = {m, ma, add, min, max, and, or,   */
/*     xor} }                                                           */
/*   else { mm[e] = 0; rank[e] = 0xffffffff; }                           */
/*   (m == 0: lane 0 writes rec[g] = 0).                                 */
/* The counter's order across warps is the order the atomics happen to  */
/* take; inside a warp the members are written in rank order.            */
/* ================================================================== */
typedef struct {
  const int32_t *x;
  int D;
  uint32_t *mm, *rank, *rec;
  int32_t *filt;
  int64_t *counter;
} dyn_ctx;

static void dyn_block(void *p, int64_t g) {
  dyn_ctx *c = (dyn_ctx *)p;
  const int32_t *x = c->x + 32 * g;
  int pr[32];
  uint32_t m[32], rk[32], mm[32], ma[32], red[6][32];
  int pred[32];
  int64_t base[32];
  xch_t X;
  xch_war(&X);
  for (int l = 0; l < 32; l++) pr[l] = ((uint32_t)x[l] & 1023u) < (uint32_t)c->D;
  /* divergent branch: the intra-warp loops run only the lanes with p */
  uint32_t active = 0;
  for (int l = 0; l < 32; l++)
    if (pr[l]) active |= 1u << l;
  for (int l = 0; l < 32; l++)
    if (pr[l]) {
      m[l] = active; /* activemask() inside the branch */
      rk[l] = (uint32_t)popc32(active & ((1u << l) - 1u));
    }
  for (int l = 0; l < 32; l++)
    if (pr[l]) xch_put(&X, l, ((uint32_t)x[l] >> 10) & 7u);
  for (int l = 0; l < 32; l++)
    if (pr[l]) mm[l] = wf_match_any(&X, l, m[l]);
  xch_war(&X);
  for (int l = 0; l < 32; l++)
    if (pr[l]) xch_put(&X, l, ((uint32_t)x[l] >> 10) & 7u);
  for (int l = 0; l < 32; l++)
    if (pr[l]) ma[l] = wf_match_all(&X, l, m[l], &pred[l]);
  xch_war(&X);
  for (int op = RD_ADD; op <= RD_XOR; op++) {
    for (int l = 0; l < 32; l++)
      if (pr[l]) xch_put(&X, l, op == RD_ADD ? ((uint32_t)x[l] & 0xffffu) : (uint32_t)x[l]);
    for (int l = 0; l < 32; l++)
      if (pr[l]) red[op][l] = wf_reduce(&X, l, m[l], op);
    xch_war(&X);
  }
  /* warp-aggregated append */
  for (int l = 0; l < 32; l++)
    if (pr[l] && rk[l] == 0)
      base[l] = __atomic_fetch_add(c->counter, (int64_t)popc32(m[l]), __ATOMIC_RELAXED);
  for (int l = 0; l < 32; l++)
    if (pr[l]) xch_put(&X, l, rk[l] == 0 ? (uint64_t)base[l] : 0u);
  for (int l = 0; l < 32; l++)
    if (pr[l]) {
      /* grp.shfl(v, 0): the member of rank 0 is the mask's first lane */
      const int ld = __builtin_ctz(m[l]);
      base[l] = (int64_t)wf_shfl(&X, l, m[l], SH_IDX, ld, 32);
    }
  xch_war(&X);
  for (int l = 0; l < 32; l++) {
    const int64_t e = 32 * g + l;
    if (pr[l]) {
      c->mm[e] = mm[l];
      c->rank[e] = rk[l];
      c->filt[base[l] + rk[l]] = x[l];
      if (rk[l] == 0) {
        uint32_t *r = c->rec + 8 * g;
        r[0] = m[l];
        r[1] = ma[l];
        for (int op = 0; op < 6; op++) r[2 + op] = red[op][l];
        (void)pred[l];
      }
    } else {
      c->mm[e] = 0;
      c->rank[e] = 0xffffffffu;
    }
    if (l == 0 && active == 0) {
      uint32_t *r = c->rec + 8 * g;
      for (int i = 0; i < 8; i++) r[i] = 0;
    }
  }
}

int coxo_warp_dynamic(const int32_t *x, int64_t n, int D, uint32_t *mm, uint32_t *rank, uint32_t *rec,
                      int32_t *filt, int64_t *count) {
  if (n < 0 || n % 32 || D < 0 || D > 1024) return COXO_ERR_INVALID;
  *count = 0;
  dyn_ctx c = {x, D, mm, rank, rec, filt, count};
  return run_blocks(n / 32, dyn_block, &c);
}

/* ================================================================== */
/* segmented reduce + scan + compaction over CSR segments               */
/* Segment s = [off[s], off[s+1]); chunks of S = 32Wk elements start at */
/* the segment's first element; the last chunk is padded.  Per chunk:   */
/*   partial P_j = reduce_chunk (same tree as the flat reduce),          */
/*   chunk-local scan q and chunk total T_j = scan_chunk,                */
/*   kept count and ranks = compact_chunk.                               */
/* Per segment:                                                          */
/*   int32: seg_total = sum_j (int64) P_j; y = wrap(carry_j + q) with    */
/*     carry_j the wrapped sum of earlier T_j;                           */
/*   binary32: seg_total = FP64 serial ascending sum of (double) P_j     */
/*     from -0.0; y = (float)(C_j + (double) q) with C_0 = -0.0 and      */
/*     C_{j+1} = C_j + (double) T_j (serial chain);                      */
/*   compaction: out[off[s] + r] = r-th element with x > 0 (in order),   */
/*     seg_count[s] = number kept.                                       */
/* An empty segment yields the identity total (0 / -0.0) and count 0.    */
/* ================================================================== */
typedef struct {
  int isf;
  const void *x;
  const int64_t *off;
  int k, W;
  void *seg_total;
  void *y;
  void *outc;
  int64_t *seg_count;
} seg_ctx;

static void seg_block(void *p, int64_t s) {
  seg_ctx *c = (seg_ctx *)p;
  const int isf = c->isf;
  const int64_t S = (int64_t)32 * c->W * c->k;
  const int64_t a = c->off[s], e1 = c->off[s + 1];
  red_kind rk;
  rk.x = c->x;
  rk.y = NULL;
  rk.dtype = isf ? DT_F32 : DT_I32;
  rk.op = OP_SUM;
  rk.acc = ACC_PLAIN;
  rk.k = c->k;
  rk.W = c->W;
  scan_kind sk = {isf, c->x, c->k, c->W};
  cmp_kind ck = {isf, c->x, c->k, c->W};
  sval *q = (sval *)malloc(sizeof(sval) * (size_t)S);
  if (!q) {
    raise_err(COXO_ERR_NOMEM);
    return;
  }
  int64_t itot = 0;
  double ftot = -0.0;
  int32_t icarry = 0;
  double fcarry = -0.0;
  int64_t kept = 0;
  for (int64_t e0 = a; e0 < e1; e0 += S) {
    lacc P = reduce_chunk(&rk, e0, e1);
    if (isf) ftot = ftot + (double)P.s;
    else itot += (int64_t)P.i;
    sval T = scan_chunk(&sk, e0, e1, q);
    for (int64_t o = 0; o < S && e0 + o < e1; o++) {
      if (isf) ((float *)c->y)[e0 + o] = (float)(fcarry + (double)q[o].f);
      else ((int32_t *)c->y)[e0 + o] = wadd(icarry, q[o].i);
    }
    if (isf) fcarry = fcarry + (double)T.f;
    else icarry = wadd(icarry, T.i);
    void *dst = isf ? (void *)((float *)c->outc + a + kept) : (void *)((int32_t *)c->outc + a + kept);
    kept += compact_chunk(&ck, e0, e1, dst);
  }
  if (isf) ((double *)c->seg_total)[s] = ftot;
  else ((int64_t *)c->seg_total)[s] = itot;
  c->seg_count[s] = kept;
  free(q);
}

int coxo_segmented(const void *x, int dtype, const int64_t *off, int64_t nseg, int k, int W,
                   void *seg_total, void *y, void *out_compact, int64_t *seg_count) {
  if (nseg < 0 || !sigma_ok(k, W)) return COXO_ERR_INVALID;
  if (dtype != DT_I32 && dtype != DT_F32) return COXO_ERR_DTYPE;
  for (int64_t s = 0; s < nseg; s++)
    if (off[s] < 0 || off[s + 1] < off[s]) return COXO_ERR_INVALID;
  seg_ctx c = {dtype == DT_F32, x, off, k, W, seg_total, y, out_compact, seg_count};
  return run_blocks(nseg, seg_block, &c);
}

/* ================================================================== */
/* exact sum (the "FP64 oracle" of the precision workload): the exact   */
/* value of sum x_i (or sum x_i*y_i) rounded once to binary64 (RNE).    */
/* Kulisch-style fixed-point accumulator: a 768-bit two's-complement    */
/* integer whose bit 0 weighs 2^-384.  Every binary32 value and every   */
/* product of two binary32 values is a multiple of 2^-298 below 2^256,  */
/* so it is added exactly; up to 2^60 terms fit.                        */
/* ================================================================== */
#define XL 12
#define XBIAS 384
typedef struct {
  uint64_t w[XL];
} xacc;

static void xacc_addsub(xacc *a, int pos, uint64_t m, int neg) {
  int li = pos >> 6, sh = pos & 63;
  uint64_t lo = m << sh, hi = sh ? (m >> (64 - sh)) : 0;
  uint64_t add[XL];
  memset(add, 0, sizeof add);
  add[li] = lo;
  if (li + 1 < XL) add[li + 1] = hi;
  if (!neg) {
    unsigned __int128 carry = 0;
    for (int i = 0; i < XL; i++) {
      unsigned __int128 t = (unsigned __int128)a->w[i] + add[i] + carry;
      a->w[i] = (uint64_t)t;
      carry = t >> 64;
    }
  } else {
    uint64_t borrow = 0;
    for (int i = 0; i < XL; i++) {
      unsigned __int128 t = (unsigned __int128)a->w[i] - add[i] - borrow;
      a->w[i] = (uint64_t)t;
      borrow = (uint64_t)(t >> 64) ? 1 : 0;
    }
  }
}

/* add an exact binary64 value */
static int xacc_add(xacc *a, double d) {
  if (d == 0.0) return 0;
  if (!isfinite(d)) return COXO_ERR_RANGE;
  int e;
  double f = frexp(fabs(d), &e);          /* |d| = f * 2^e, f in [0.5, 1) */
  uint64_t m = (uint64_t)ldexp(f, 53);    /* |d| = m * 2^(e-53), exact */
  int pos = e - 53 + XBIAS;
  while (pos < 0) {
    if (m & 1u) return COXO_ERR_RANGE;    /* below the accumulator's lsb */
    m >>= 1;
    pos++;
  }
  if (pos + 53 > XL * 64 - 64) return COXO_ERR_RANGE;
  xacc_addsub(a, pos, m, d < 0);
  return 0;
}

static void xacc_merge(xacc *a, const xacc *b) {
  unsigned __int128 carry = 0;
  for (int i = 0; i < XL; i++) {
    unsigned __int128 t = (unsigned __int128)a->w[i] + b->w[i] + carry;
    a->w[i] = (uint64_t)t;
    carry = t >> 64;
  }
}

static double xacc_round(const xacc *in) {
  xacc a = *in;
  int neg = (a.w[XL - 1] >> 63) & 1;
  if (neg) { /* negate */
    unsigned __int128 carry = 1;
    for (int i = 0; i < XL; i++) {
      unsigned __int128 t = (unsigned __int128)(~a.w[i]) + carry;
      a.w[i] = (uint64_t)t;
      carry = t >> 64;
    }
  }
  int top = -1;
  for (int i = XL - 1; i >= 0 && top < 0; i--)
    if (a.w[i]) top = i * 64 + 63 - __builtin_clzll(a.w[i]);
  if (top < 0) return neg ? -0.0 : 0.0;
  /* gather bits [top-63, top] into M and a sticky bit for everything below */
  uint64_t M = 0;
  int sticky = 0;
  for (int b = 0; b < 64; b++) {
    int pos = top - b;
    M <<= 1;
    if (pos >= 0 && ((a.w[pos >> 6] >> (pos & 63)) & 1u)) M |= 1u;
  }
  for (int pos = top - 64; pos >= 0 && !sticky; pos--)
    if ((a.w[pos >> 6] >> (pos & 63)) & 1u) sticky = 1;
  uint64_t q = M >> 11, rem = M & 0x7ffu;
  if (rem > 0x400u || (rem == 0x400u && (sticky || (q & 1u)))) q++;
  int scale = top - 52 - XBIAS;
  double r = ldexp((double)q, scale); /* q == 2^53 after rounding is exact too */
  return neg ? -r : r;
}

typedef struct {
  const void *x, *y;
  int dtype;
  int64_t n, per;
  xacc *acc;
  int *err;
} xs_ctx;

static void xs_block(void *p, int64_t b) {
  xs_ctx *c = (xs_ctx *)p;
  xacc a;
  memset(&a, 0, sizeof a);
  int64_t lo = b * c->per, hi = lo + c->per < c->n ? lo + c->per : c->n;
  for (int64_t i = lo; i < hi; i++) {
    double t;
    if (c->dtype == DT_I32) t = (double)((const int32_t *)c->x)[i];
    else {
      double xv = (double)load_f(c->x, c->dtype, i);
      t = c->y ? xv * (double)load_f(c->y, c->dtype, i) : xv; /* exact: 24+24 bits */
    }
    if (xacc_add(&a, t)) raise_err(COXO_ERR_RANGE);
  }
  c->acc[b] = a;
}

int coxo_exact_sum(const void *x, const void *y, int dtype, int64_t n, double *out) {
  if (n < 0) return COXO_ERR_INVALID;
  if (dtype != DT_F32 && dtype != DT_BF16 && dtype != DT_I32) return COXO_ERR_DTYPE;
  const int64_t per = 1 << 16, nb = (n + per - 1) / per;
  xacc *acc = (xacc *)calloc((size_t)(nb ? nb : 1), sizeof(xacc));
  if (!acc) return COXO_ERR_NOMEM;
  xs_ctx c = {x, y, dtype, n, per, acc, NULL};
  int err = run_blocks(nb, xs_block, &c);
  xacc tot;
  memset(&tot, 0, sizeof tot);
  for (int64_t b = 0; b < nb; b++) xacc_merge(&tot, &acc[b]);
  *out = xacc_round(&tot);
  free(acc);
  return err;
}

/* exact sum of arbitrary binary64 values (used to pin the accumulator) */
int coxo_exact_sum_f64(const double *x, int64_t n, double *out) {
  xacc a;
  memset(&a, 0, sizeof a);
  for (int64_t i = 0; i < n; i++)
    if (xacc_add(&a, x[i])) return COXO_ERR_RANGE;
  *out = xacc_round(&a);
  return 0;
}

/* the two halves of the compensated step, exposed so that tests can check
 * that they are error-free transformations */
void coxo_two_sum(float a, float b, float *s, float *e) { two_sum(a, b, s, e); }
void coxo_two_prod(float a, float b, float *p, float *e) {
  *p = a * b;
  *e = fmaf(a, b, -*p);
}

/* Two back-to-back warp votes (Sec. 3.2, Code 5): r1 = all(FULL, a),
 * r2 = all(FULL, b) for one warp.  With barriers = 1 the operand writes and
 * builtin reads of each vote are separate warp regions (RAW and WAR
 * barriers).  With barriers = 0 one intra-warp loop runs write, vote,
 * write, vote per lane, i.e. the barriers are missing; the exchange-array
 * checks must then report COXO_ERR_UB instead of returning values. */
int coxo_code5(const int32_t *a, const int32_t *b, int32_t *r1, int32_t *r2, int barriers) {
  xch_t X;
  xch_war(&X);
  t_err = 0;
  if (barriers) {
    for (int l = 0; l < 32; l++) xch_put(&X, l, (uint64_t)(a[l] != 0));
    for (int l = 0; l < 32; l++) r1[l] = wf_all(&X, l, FULL);
    xch_war(&X);
    for (int l = 0; l < 32; l++) xch_put(&X, l, (uint64_t)(b[l] != 0));
    for (int l = 0; l < 32; l++) r2[l] = wf_all(&X, l, FULL);
    xch_war(&X);
  } else {
    for (int l = 0; l < 32; l++) {
      xch_put(&X, l, (uint64_t)(a[l] != 0));
      r1[l] = wf_all(&X, l, FULL);
      xch_put(&X, l, (uint64_t)(b[l] != 0));
      r2[l] = wf_all(&X, l, FULL);
    }
  }
  return t_err;
}

/* A branch that encloses warp barriers (Sec. 3.3.1): per warp,
 *   if (cond) { out = x + shfl_down tree (offsets 16..1) } else out = x;
 * The condition is evaluated by every lane and must be uniform across the
 * warp (aligned barriers); lane 0's outcome is followed.  A non-uniform
 * condition reports COXO_ERR_DIVERGENT. */
typedef struct {
  const int32_t *cond, *x;
  int32_t *out;
} ub_ctx;

static void ub_block(void *p, int64_t g) {
  ub_ctx *c = (ub_ctx *)p;
  int flag[32];
  int32_t v[32];
  xch_t X;
  xch_war(&X);
  for (int l = 0; l < 32; l++) {
    flag[l] = c->cond[32 * g + l] != 0;
    v[l] = c->x[32 * g + l];
  }
  if (peel(flag, 32)) {
    for (int o = 16; o > 0; o >>= 1) {
      for (int l = 0; l < 32; l++) xch_put(&X, l, ibits(v[l]));
      for (int l = 0; l < 32; l++) v[l] = wadd(v[l], bitsi(wf_shfl(&X, l, FULL, SH_DOWN, o, 32)));
      xch_war(&X);
    }
  }
  for (int l = 0; l < 32; l++) c->out[32 * g + l] = v[l];
}

int coxo_uniform_branch(const int32_t *cond, const int32_t *x, int64_t n, int32_t *out) {
  if (n < 0 || n % 32) return COXO_ERR_INVALID;
  ub_ctx c = {cond, x, out};
  return run_blocks(n / 32, ub_block, &c);
}

/* ================================================================== */
/* integral image (summed-area table), the application of the shuffle    */
/* scans in Table 1 (shfl_intimage_rows, shfl_vertical_shfl):            */
/*   sat[y][x] = sum of img[y'][x'] over y' <= y, x' <= x  (mod 2^32)    */
/* The plain definition: an inclusive prefix along every row, then one   */
/* down every column, in uint32 arithmetic (exact modulo 2^32, so the    */
/* order of the additions does not matter).                              */
/* ================================================================== */
typedef struct {
  const uint8_t *img;
  uint32_t *sat;
  int64_t H, W;
} ii_ctx;

static void ii_rows(void *p, int64_t y) {
  ii_ctx *c = (ii_ctx *)p;
  uint32_t s = 0;
  for (int64_t x = 0; x < c->W; x++) {
    s += c->img[y * c->W + x];
    c->sat[y * c->W + x] = s;
  }
}
static void ii_cols(void *p, int64_t x) {
  ii_ctx *c = (ii_ctx *)p;
  uint32_t s = 0;
  for (int64_t y = 0; y < c->H; y++) {
    s += c->sat[y * c->W + x];
    c->sat[y * c->W + x] = s;
  }
}

int coxo_integral_image_u8(const uint8_t *img, int64_t H, int64_t W, uint32_t *sat) {
  if (H < 0 || W < 0) return COXO_ERR_INVALID;
  ii_ctx c = {img, sat, H, W};
  int st = run_blocks(H, ii_rows, &c);
  if (st == COXO_OK) st = run_blocks(W, ii_cols, &c);
  return st;
}

/* ================================================================== */
/* grid-wide barriers (this_grid().sync(), Sec. 2.2.2; COX could not run */
/* kernels that need one, Sec. 5.1 and Table 1)                         */
/*                                                                      */
/* A grid barrier is collapsed one level above the block barrier of     */
/* Sec. 3.5: the kernel is split at it into grid-level regions, and a   */
/* region runs for every block before the next one starts.  Here every  */
/* grid-level region is one run_blocks pass.                            */
/* ================================================================== */

/* MurmurHash3's 32-bit finaliser (Appleby), the payload mixer of the    */
/* exchange kernel                                                       */
static uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

/* Exchange kernel: G blocks of BT threads, `rounds` rounds; in round r
 *   region 1: thread t of block b writes fmix32(r << 20 ^ b << 10 ^ t) to
 *             slot[b][t];
 *   grid barrier;
 *   region 2: thread t of block b adds (mod 2^32) slot[(b + r + 1) % G][t]
 *             to its sum;
 *   grid barrier (the next round overwrites the slots).
 * out[b * BT + t] = the sum. */
typedef struct {
  int G, BT, r;
  uint32_t *slot, *out;
} gx_ctx;

static void gx_write(void *p, int64_t b) {
  gx_ctx *c = (gx_ctx *)p;
  for (int t = 0; t < c->BT; t++)
    c->slot[b * c->BT + t] = fmix32(((uint32_t)c->r << 20) ^ ((uint32_t)b << 10) ^ (uint32_t)t);
}
static void gx_read(void *p, int64_t b) {
  gx_ctx *c = (gx_ctx *)p;
  const int64_t src = (b + c->r + 1) % c->G;
  for (int t = 0; t < c->BT; t++) c->out[b * c->BT + t] += c->slot[src * c->BT + t];
}

int coxo_grid_exchange(int G, int BT, int rounds, uint32_t *out) {
  if (G < 1 || G > 1024 || BT < 1 || BT > 1024 || rounds < 0) return COXO_ERR_INVALID;
  uint32_t *slot = (uint32_t *)calloc((size_t)G * BT, 4);
  if (!slot) return COXO_ERR_NOMEM;
  memset(out, 0, (size_t)G * BT * 4);
  gx_ctx c = {G, BT, 0, slot, out};
  int st = COXO_OK;
  for (int r = 0; r < rounds && st == COXO_OK; r++) {
    c.r = r;
    st = run_blocks(G, gx_write, &c);
    if (st == COXO_OK) st = run_blocks(G, gx_read, &c);
  }
  free(slot);
  return st;
}

/* ------------------------------------------------------------------ */
/* Conjugate gradient (Hestenes and Stiefel, 1952) for a symmetric       */
/* positive definite A in CSR form: the solver of gpuConjugateGradient   */
/* (Table 1), whose iterations are separated by grid barriers.           */
/* Vectors are binary32, scalars binary64:                                */
/*   r = b - A x;  rr_0 = <r, r>                                          */
/*   for k = 0, 1, ...:                                                    */
/*     stop (reason 0) if rr_k <= tol^2, (reason 1) if k == max_iter       */
/*     p = r if k == 0, else fmaf(beta, p, r), beta = (float)(rr_k/rr_k-1) */
/*     q = A p;  pq = <p, q>;  stop (reason 2) unless pq > 0               */
/*     alpha = (float)(rr_k / pq)                                          */
/*     x = fmaf(alpha, p, x);  r = fmaf(-alpha, q, r);  rr_k+1 = <r, r>    */
/* (A v)_i = the row's entries in storage order accumulated from +0.0f as */
/* acc = fmaf(a_ij, v_j, acc).                                             */
/* <u, v> with schedule (R, W): chunk c is rows [cS, cS + S), S = 32 W R;  */
/* thread (w, l) adds the exact products (double) u_i * (double) v_i of    */
/* rows cS + 32 W q + 32 w + l, q = 0 .. R-1 (rows past n add nothing), in */
/* FP64 from -0.0; each warp runs the shfl_down tree, warp 0 runs it over  */
/* the W warp values (-0.0 beyond W): the chunk value; final_f64 combines  */
/* the chunk values.  Every grid-level region below is one pass.           */
/* ------------------------------------------------------------------ */
typedef struct {
  const int32_t *rp, *ci;
  const float *val, *b;
  float *x, *r, *p, *q;
  int64_t n, S;
  int R, W;
  float coef;   /* beta of the p pass, alpha of the x/r pass */
  int first;    /* p pass of iteration 0 */
  double *part; /* chunk values of the pass's inner product */
} cg_ctx;

static float cg_row(const cg_ctx *g, int64_t i, const float *v) {
  float acc = 0.0f;
  for (int64_t jj = g->rp[i]; jj < g->rp[i + 1]; jj++) acc = fmaf(g->val[jj], v[g->ci[jj]], acc);
  return acc;
}

static void tree_f64_shfl_down(double *a, xch_t *X) {
  for (int o = 16; o > 0; o >>= 1) {
    for (int l = 0; l < 32; l++) xch_put(X, l, dbits(a[l]));
    for (int l = 0; l < 32; l++) a[l] = a[l] + bitsd(wf_shfl(X, l, FULL, SH_DOWN, o, 32));
    xch_war(X);
  }
}

/* the chunk value of <u, v> */
static double cg_chunk_dot(const cg_ctx *g, int64_t c, const float *u, const float *v) {
  const int W = g->W, R = g->R;
  double t[32 * MAXW];
  double slot[MAXW];
  xch_t X;
  xch_war(&X);
  for (int w = 0; w < W; w++) {
    for (int l = 0; l < 32; l++) {
      double s = -0.0;
      for (int q = 0; q < R; q++) {
        const int64_t i = c * g->S + (int64_t)32 * W * q + 32 * w + l;
        if (i < g->n) s = s + (double)u[i] * (double)v[i];
      }
      t[32 * w + l] = s;
    }
    tree_f64_shfl_down(&t[32 * w], &X);
    slot[w] = t[32 * w];
  }
  double a[32];
  for (int l = 0; l < 32; l++) a[l] = l < W ? slot[l] : -0.0;
  tree_f64_shfl_down(a, &X);
  return a[0];
}

static int64_t cg_lo(const cg_ctx *g, int64_t c) { return c * g->S; }
static int64_t cg_hi(const cg_ctx *g, int64_t c) {
  const int64_t e = (c + 1) * g->S;
  return e < g->n ? e : g->n;
}

/* r = b - A x, chunk values of <r, r> */
static void cg_pass_r0(void *p, int64_t c) {
  cg_ctx *g = (cg_ctx *)p;
  for (int64_t i = cg_lo(g, c); i < cg_hi(g, c); i++) g->r[i] = g->b[i] - cg_row(g, i, g->x);
  g->part[c] = cg_chunk_dot(g, c, g->r, g->r);
}
/* p = r or fmaf(beta, p, r) */
static void cg_pass_p(void *p, int64_t c) {
  cg_ctx *g = (cg_ctx *)p;
  for (int64_t i = cg_lo(g, c); i < cg_hi(g, c); i++) g->p[i] = g->first ? g->r[i] : fmaf(g->coef, g->p[i], g->r[i]);
}
/* q = A p, chunk values of <p, q> */
static void cg_pass_q(void *p, int64_t c) {
  cg_ctx *g = (cg_ctx *)p;
  for (int64_t i = cg_lo(g, c); i < cg_hi(g, c); i++) g->q[i] = cg_row(g, i, g->p);
  g->part[c] = cg_chunk_dot(g, c, g->p, g->q);
}
/* x += alpha p, r -= alpha q, chunk values of <r, r> */
static void cg_pass_xr(void *p, int64_t c) {
  cg_ctx *g = (cg_ctx *)p;
  for (int64_t i = cg_lo(g, c); i < cg_hi(g, c); i++) {
    g->x[i] = fmaf(g->coef, g->p[i], g->x[i]);
    g->r[i] = fmaf(-g->coef, g->q[i], g->r[i]);
  }
  g->part[c] = cg_chunk_dot(g, c, g->r, g->r);
}

/* rp: int32[n+1] with rp[0] = 0, nondecreasing, rp[n] = nnz; ci: int32[nnz]
 * column indices in [0, n); val: float[nnz]; b: float[n]; x: float[n], the
 * start on entry and the result on return.  result[0] = iterations k,
 * result[1] = reason; rr_hist[0 .. k] = rr_0 .. rr_k (max_iter + 1
 * entries). */
int coxo_cg(const int32_t *rp, const int32_t *ci, const float *val, int64_t n, const float *b, float *x,
            int max_iter, double tol, int R, int W, int32_t *result, double *rr_hist) {
  if (n < 0 || max_iter < 0 || !sigma_ok(R, W) || R > 8) return COXO_ERR_INVALID;
  if (n > 0 && rp[0] != 0) return COXO_ERR_INVALID;
  for (int64_t i = 0; i < n; i++) {
    if (rp[i + 1] < rp[i]) return COXO_ERR_INVALID;
    for (int64_t jj = rp[i]; jj < rp[i + 1]; jj++)
      if (ci[jj] < 0 || ci[jj] >= n) return COXO_ERR_INVALID;
  }
  const int64_t S = (int64_t)32 * W * R;
  const int64_t nch = (n + S - 1) / S;
  const size_t nb = (size_t)(n > 0 ? n : 1) * sizeof(float);
  float *r = (float *)malloc(nb), *pv = (float *)malloc(nb), *q = (float *)malloc(nb);
  double *part = (double *)malloc((size_t)(nch > 0 ? nch : 1) * sizeof(double));
  int st = COXO_OK;
  if (!r || !pv || !q || !part) st = COXO_ERR_NOMEM;
  cg_ctx g = {rp, ci, val, b, x, r, pv, q, n, S, R, W, 0.0f, 1, part};
  const double tol2 = tol * tol;
  int k = 0, reason = 0;
  double rr = 0.0, rr_prev = 0.0;
  if (st == COXO_OK) st = run_blocks(nch, cg_pass_r0, &g);
  if (st == COXO_OK) rr = final_f64(part, nch);
  for (; st == COXO_OK; k++) {
    rr_hist[k] = rr;
    if (rr <= tol2) {
      reason = 0;
      break;
    }
    if (k == max_iter) {
      reason = 1;
      break;
    }
    g.first = k == 0;
    g.coef = k == 0 ? 0.0f : (float)(rr / rr_prev);
    st = run_blocks(nch, cg_pass_p, &g);
    if (st == COXO_OK) st = run_blocks(nch, cg_pass_q, &g);
    if (st != COXO_OK) break;
    const double pq = final_f64(part, nch);
    if (!(pq > 0.0)) {
      reason = 2;
      break;
    }
    g.coef = (float)(rr / pq);
    st = run_blocks(nch, cg_pass_xr, &g);
    if (st != COXO_OK) break;
    rr_prev = rr;
    rr = final_f64(part, nch);
  }
  result[0] = k;
  result[1] = reason;
  free(r);
  free(pv);
  free(q);
  free(part);
  return st;
}
