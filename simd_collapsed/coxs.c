/*
 * coxs.c -- a SIMD-collapsed CPU executor of the warp-level kernels.
 *
 * Hierarchical collapsing (COX, Sec. 3.5-3.6): a CUDA block runs as one
 * CPU task; the code between block barriers is a loop over the block's
 * warps, and the code between warp-level collectives is a loop over the 32
 * lanes of a warp.  Here each warp's 32 lanes are held as one SIMD value,
 * so an intra-warp loop is a few vector instructions, and the warp
 * builtins -- ballot / any / all and the four shuffles -- take and return
 * whole warps, the way COX implements its warp_vote / warp_all runtime
 * functions with AVX over the per-warp array (Sec. 3.2; the vote any / all
 * timings with and without AVX, Table 2 of Sec. 5.2).
 *
 * One source, three builds:
 *   COXS_ISA = 512 : AVX-512 (F, BW, DQ, VL, CD): a warp is two zmm
 *                    registers; shuffles are vpermt2d, votes are mask
 *                    registers;
 *   COXS_ISA = 256 : AVX2 + FMA: a warp is four ymm registers;
 *   COXS_ISA = 0   : the lane loops written out, compiled without
 *                    auto-vectorisation (the "without SIMD" build).
 *
 * Every lane does the schedule's arithmetic in the schedule's order (the
 * element mapping of sigma = (k, W), the shfl_down trees, the scan tree,
 * TwoSum / TwoProduct), so integer and binary32 results are those of the
 * plain collapsed executor bit for bit.  Built with -ffp-contract=off:
 * fused multiply-adds only where a schedule names one.
 *
 * This is a CPU executor and baseline.  The GPU library never links or
 * calls it.
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#if COXS_ISA == 512 || COXS_ISA == 256
#include <immintrin.h>
#endif

#ifndef COXS_ISA
#error "COXS_ISA must be 512, 256 or 0"
#endif

enum {
  COXS_OK = 0,
  COXS_ERR_INVALID = 1,
  COXS_ERR_DTYPE = 2,
  COXS_ERR_UB = 8, /* a masked shuffle reading a lane outside its mask */
  COXS_ERR_NOMEM = 11
};
enum { DT_I32 = 0, DT_U32 = 1, DT_F32 = 2, DT_BF16 = 3 };
enum { ACC_PLAIN = 0, ACC_TWOSUM = 1 };
enum { SH_IDX = 0, SH_UP = 1, SH_DOWN = 2, SH_XOR = 3 };

#define ALL32 0xffffffffu
#define NEG0 0x80000000u /* -0.0f, the additive identity of binary32 */

static uint32_t f2u(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}
static float u2f(uint32_t u) {
  float f;
  memcpy(&f, &u, 4);
  return f;
}
static int popc(uint32_t m) { return __builtin_popcount(m); }

/* ================================================================== */
/* one warp as one SIMD value: 32 lanes of 32-bit words                 */
/* ================================================================== */
#if COXS_ISA == 512
/* named members, no arrays: the struct stays in registers */
typedef struct {
  __m512i lo, hi; /* lanes 0-15, 16-31 */
} wv;
#define WV_INLINE static inline __attribute__((always_inline))
#define MAP1(r, x, F) ((r).lo = F((x).lo), (r).hi = F((x).hi))
#define MAP2(r, x, y, F) ((r).lo = F((x).lo, (y).lo), (r).hi = F((x).hi, (y).hi))
#define MASK2(x, y, F) ((uint32_t)F((x).lo, (y).lo) | ((uint32_t)F((x).hi, (y).hi) << 16))
WV_INLINE wv wv_load(const void *p) {
  wv r;
  r.lo = _mm512_loadu_si512(p);
  r.hi = _mm512_loadu_si512((const char *)p + 64);
  return r;
}
WV_INLINE void wv_store(void *p, wv a) {
  _mm512_storeu_si512(p, a.lo);
  _mm512_storeu_si512((char *)p + 64, a.hi);
}
WV_INLINE wv wv_splat(uint32_t x) {
  wv r;
  r.lo = r.hi = _mm512_set1_epi32((int)x);
  return r;
}
#define WV_BIN(name, intr)        \
  WV_INLINE wv name(wv a, wv b) { \
    wv r;                         \
    MAP2(r, a, b, intr);          \
    return r;                     \
  }
WV_BIN(wv_add, _mm512_add_epi32)
WV_BIN(wv_and, _mm512_and_si512)
WV_BIN(wv_or, _mm512_or_si512)
WV_BIN(wv_xor, _mm512_xor_si512)
WV_BIN(wv_minu, _mm512_min_epu32)
WV_BIN(wv_maxu, _mm512_max_epu32)
#define F512(intr) static inline __attribute__((always_inline)) __m512i intr##_i(__m512i a, __m512i b) { \
    return _mm512_castps_si512(intr(_mm512_castsi512_ps(a), _mm512_castsi512_ps(b)));               \
  }
F512(_mm512_add_ps)
F512(_mm512_sub_ps)
F512(_mm512_mul_ps)
WV_BIN(wv_fadd, _mm512_add_ps_i)
WV_BIN(wv_fsub, _mm512_sub_ps_i)
WV_BIN(wv_fmul, _mm512_mul_ps_i)
WV_INLINE __m512i fma512(__m512i a, __m512i b, __m512i c) {
  return _mm512_castps_si512(
      _mm512_fmadd_ps(_mm512_castsi512_ps(a), _mm512_castsi512_ps(b), _mm512_castsi512_ps(c)));
}
WV_INLINE wv wv_ffma(wv a, wv b, wv c) {
  wv r;
  r.lo = fma512(a.lo, b.lo, c.lo);
  r.hi = fma512(a.hi, b.hi, c.hi);
  return r;
}
/* ballot of (lane != 0) */
WV_INLINE uint32_t wv_nz(wv a) { return MASK2(a, a, _mm512_test_epi32_mask); }
WV_INLINE __mmask16 gt0_i(__m512i a, __m512i z) { return _mm512_cmpgt_epi32_mask(a, z); }
WV_INLINE __mmask16 gt0_f(__m512i a, __m512i z) {
  return _mm512_cmp_ps_mask(_mm512_castsi512_ps(a), _mm512_castsi512_ps(z), _CMP_GT_OQ);
}
WV_INLINE uint32_t wv_gt0_i32(wv a) {
  const wv z = wv_splat(0);
  return MASK2(a, z, gt0_i);
}
WV_INLINE uint32_t wv_gt0_f32(wv a) {
  const wv z = wv_splat(0);
  return MASK2(a, z, gt0_f);
}
WV_INLINE uint32_t wv_ltu(wv a, wv b) { return MASK2(a, b, _mm512_cmplt_epu32_mask); }
WV_INLINE uint32_t wv_eq(wv a, wv b) { return MASK2(a, b, _mm512_cmpeq_epi32_mask); }
/* lane l: bit l of m ? a : b */
WV_INLINE wv wv_sel(uint32_t m, wv a, wv b) {
  wv r;
  r.lo = _mm512_mask_blend_epi32((__mmask16)(m & 0xffffu), b.lo, a.lo);
  r.hi = _mm512_mask_blend_epi32((__mmask16)(m >> 16), b.hi, a.hi);
  return r;
}
/* lane l: a[idx[l]], idx in [0, 31] */
WV_INLINE wv wv_perm(wv a, wv idx) {
  wv r;
  r.lo = _mm512_permutex2var_epi32(a.lo, idx.lo, a.hi);
  r.hi = _mm512_permutex2var_epi32(a.lo, idx.hi, a.hi);
  return r;
}
/* lane l: 32-bit word at byte offset 4 * idx[l] from base */
WV_INLINE wv wv_gather(const void *base, wv idx) {
  wv r;
  r.lo = _mm512_i32gather_epi32(idx.lo, base, 4);
  r.hi = _mm512_i32gather_epi32(idx.hi, base, 4);
  return r;
}
/* 32-bit words at byte offset 2 * idx[l] (bfloat16 elements in the low half) */
WV_INLINE wv wv_gather_h(const void *base, wv idx) {
  wv r;
  r.lo = _mm512_i32gather_epi32(idx.lo, base, 2);
  r.hi = _mm512_i32gather_epi32(idx.hi, base, 2);
  return r;
}
WV_INLINE void wv_scatter(void *base, wv idx, wv a) {
  _mm512_i32scatter_epi32(base, idx.lo, a.lo, 4);
  _mm512_i32scatter_epi32(base, idx.hi, a.hi, 4);
}
WV_INLINE __m512i sl16(__m512i a) { return _mm512_slli_epi32(a, 16); }
WV_INLINE wv wv_slli16(wv a) {
  wv r;
  MAP1(r, a, sl16);
  return r;
}
/* (float)(C + (double)q) per lane */
WV_INLINE __m512i carry16(__m512i q, __m512d c) {
  const __m512 f = _mm512_castsi512_ps(q);
  const __m512d lo = _mm512_add_pd(c, _mm512_cvtps_pd(_mm512_castps512_ps256(f)));
  const __m512d hi = _mm512_add_pd(c, _mm512_cvtps_pd(_mm256_castpd_ps(_mm512_extractf64x4_pd(_mm512_castps_pd(f), 1))));
  return _mm512_castps_si512(_mm512_insertf32x8(_mm512_castps256_ps512(_mm512_cvtpd_ps(lo)), _mm512_cvtpd_ps(hi), 1));
}
WV_INLINE wv wv_carry_f64(wv q, double C) {
  const __m512d c = _mm512_set1_pd(C);
  wv r;
  r.lo = carry16(q.lo, c);
  r.hi = carry16(q.hi, c);
  return r;
}
/* stores the lanes of a whose bit is set in m, in lane order, at dst;
 * returns how many */
WV_INLINE int wv_compress_store(void *dst, uint32_t m, wv a) {
  _mm512_mask_compressstoreu_epi32(dst, (__mmask16)(m & 0xffffu), a.lo);
  const int c0 = popc(m & 0xffffu);
  _mm512_mask_compressstoreu_epi32((char *)dst + 4 * c0, (__mmask16)(m >> 16), a.hi);
  return popc(m);
}

#elif COXS_ISA == 256
/* named members, no arrays: the struct stays in registers */
typedef struct {
  __m256i q0, q1, q2, q3; /* lanes 0-7, 8-15, 16-23, 24-31 */
} wv;
#define WV_INLINE static inline __attribute__((always_inline))
#define MAP1(r, x, F) ((r).q0 = F((x).q0), (r).q1 = F((x).q1), (r).q2 = F((x).q2), (r).q3 = F((x).q3))
#define MAP2(r, x, y, F) \
  ((r).q0 = F((x).q0, (y).q0), (r).q1 = F((x).q1, (y).q1), (r).q2 = F((x).q2, (y).q2), (r).q3 = F((x).q3, (y).q3))
WV_INLINE wv wv_load(const void *p) {
  const char *c = (const char *)p;
  wv r;
  r.q0 = _mm256_loadu_si256((const __m256i *)c);
  r.q1 = _mm256_loadu_si256((const __m256i *)(c + 32));
  r.q2 = _mm256_loadu_si256((const __m256i *)(c + 64));
  r.q3 = _mm256_loadu_si256((const __m256i *)(c + 96));
  return r;
}
WV_INLINE void wv_store(void *p, wv a) {
  char *c = (char *)p;
  _mm256_storeu_si256((__m256i *)c, a.q0);
  _mm256_storeu_si256((__m256i *)(c + 32), a.q1);
  _mm256_storeu_si256((__m256i *)(c + 64), a.q2);
  _mm256_storeu_si256((__m256i *)(c + 96), a.q3);
}
WV_INLINE wv wv_splat(uint32_t x) {
  wv r;
  r.q0 = r.q1 = r.q2 = r.q3 = _mm256_set1_epi32((int)x);
  return r;
}
#define WV_BIN(name, intr)        \
  WV_INLINE wv name(wv a, wv b) { \
    wv r;                         \
    MAP2(r, a, b, intr);          \
    return r;                     \
  }
WV_BIN(wv_add, _mm256_add_epi32)
WV_BIN(wv_and, _mm256_and_si256)
WV_BIN(wv_or, _mm256_or_si256)
WV_BIN(wv_xor, _mm256_xor_si256)
WV_BIN(wv_minu, _mm256_min_epu32)
WV_BIN(wv_maxu, _mm256_max_epu32)
#define F256(intr) static inline __attribute__((always_inline)) __m256i intr##_i(__m256i a, __m256i b) { \
    return _mm256_castps_si256(intr(_mm256_castsi256_ps(a), _mm256_castsi256_ps(b)));               \
  }
F256(_mm256_add_ps)
F256(_mm256_sub_ps)
F256(_mm256_mul_ps)
WV_BIN(wv_fadd, _mm256_add_ps_i)
WV_BIN(wv_fsub, _mm256_sub_ps_i)
WV_BIN(wv_fmul, _mm256_mul_ps_i)
WV_INLINE __m256i fma256(__m256i a, __m256i b, __m256i c) {
  return _mm256_castps_si256(
      _mm256_fmadd_ps(_mm256_castsi256_ps(a), _mm256_castsi256_ps(b), _mm256_castsi256_ps(c)));
}
WV_INLINE wv wv_ffma(wv a, wv b, wv c) {
  wv r;
  r.q0 = fma256(a.q0, b.q0, c.q0);
  r.q1 = fma256(a.q1, b.q1, c.q1);
  r.q2 = fma256(a.q2, b.q2, c.q2);
  r.q3 = fma256(a.q3, b.q3, c.q3);
  return r;
}
/* 8-lane all-ones / zero lanes -> 8 bits */
WV_INLINE uint32_t m8(__m256i m) { return (uint32_t)_mm256_movemask_ps(_mm256_castsi256_ps(m)); }
#define MASK4(x, y, F) (m8(F((x).q0, (y).q0)) | (m8(F((x).q1, (y).q1)) << 8) | (m8(F((x).q2, (y).q2)) << 16) | \
                        (m8(F((x).q3, (y).q3)) << 24))
WV_INLINE uint32_t wv_nz(wv a) {
  const wv z = wv_splat(0);
  return ~MASK4(a, z, _mm256_cmpeq_epi32);
}
WV_INLINE uint32_t wv_gt0_i32(wv a) {
  const wv z = wv_splat(0);
  return MASK4(a, z, _mm256_cmpgt_epi32);
}
WV_INLINE __m256i gt0f(__m256i a, __m256i z) {
  return _mm256_castps_si256(_mm256_cmp_ps(_mm256_castsi256_ps(a), _mm256_castsi256_ps(z), _CMP_GT_OQ));
}
WV_INLINE uint32_t wv_gt0_f32(wv a) {
  const wv z = wv_splat(0);
  return MASK4(a, z, gt0f);
}
/* unsigned a < b as signed compare of the sign-flipped values */
WV_INLINE __m256i ltu8(__m256i a, __m256i b) {
  const __m256i s = _mm256_set1_epi32((int)0x80000000);
  return _mm256_cmpgt_epi32(_mm256_xor_si256(b, s), _mm256_xor_si256(a, s));
}
WV_INLINE uint32_t wv_ltu(wv a, wv b) { return MASK4(a, b, ltu8); }
WV_INLINE uint32_t wv_eq(wv a, wv b) { return MASK4(a, b, _mm256_cmpeq_epi32); }
/* bits 8j .. 8j+7 of m -> per-lane all-ones / zeros */
WV_INLINE __m256i lanes8(uint32_t m, int j) {
  const __m256i bit = _mm256_setr_epi32(1, 2, 4, 8, 16, 32, 64, 128);
  const __m256i b = _mm256_set1_epi32((int)((m >> (8 * j)) & 0xffu));
  return _mm256_cmpeq_epi32(_mm256_and_si256(b, bit), bit);
}
WV_INLINE wv wv_sel(uint32_t m, wv a, wv b) {
  wv r;
  r.q0 = _mm256_blendv_epi8(b.q0, a.q0, lanes8(m, 0));
  r.q1 = _mm256_blendv_epi8(b.q1, a.q1, lanes8(m, 1));
  r.q2 = _mm256_blendv_epi8(b.q2, a.q2, lanes8(m, 2));
  r.q3 = _mm256_blendv_epi8(b.q3, a.q3, lanes8(m, 3));
  return r;
}
/* 8 output lanes: a[idx], idx in [0, 31], from the four source registers */
WV_INLINE __m256i perm8(wv a, __m256i idx) {
  const __m256i lo = _mm256_and_si256(idx, _mm256_set1_epi32(7));
  const __m256i reg = _mm256_srli_epi32(idx, 3);
  __m256i r = _mm256_permutevar8x32_epi32(a.q0, lo);
  r = _mm256_blendv_epi8(r, _mm256_permutevar8x32_epi32(a.q1, lo), _mm256_cmpeq_epi32(reg, _mm256_set1_epi32(1)));
  r = _mm256_blendv_epi8(r, _mm256_permutevar8x32_epi32(a.q2, lo), _mm256_cmpeq_epi32(reg, _mm256_set1_epi32(2)));
  r = _mm256_blendv_epi8(r, _mm256_permutevar8x32_epi32(a.q3, lo), _mm256_cmpeq_epi32(reg, _mm256_set1_epi32(3)));
  return r;
}
WV_INLINE wv wv_perm(wv a, wv idx) {
  wv r;
  r.q0 = perm8(a, idx.q0);
  r.q1 = perm8(a, idx.q1);
  r.q2 = perm8(a, idx.q2);
  r.q3 = perm8(a, idx.q3);
  return r;
}
WV_INLINE wv wv_gather(const void *base, wv idx) {
  wv r;
  r.q0 = _mm256_i32gather_epi32((const int *)base, idx.q0, 4);
  r.q1 = _mm256_i32gather_epi32((const int *)base, idx.q1, 4);
  r.q2 = _mm256_i32gather_epi32((const int *)base, idx.q2, 4);
  r.q3 = _mm256_i32gather_epi32((const int *)base, idx.q3, 4);
  return r;
}
WV_INLINE wv wv_gather_h(const void *base, wv idx) {
  wv r;
  r.q0 = _mm256_i32gather_epi32((const int *)base, idx.q0, 2);
  r.q1 = _mm256_i32gather_epi32((const int *)base, idx.q1, 2);
  r.q2 = _mm256_i32gather_epi32((const int *)base, idx.q2, 2);
  r.q3 = _mm256_i32gather_epi32((const int *)base, idx.q3, 2);
  return r;
}
WV_INLINE void wv_scatter(void *base, wv idx, wv a) {
  int32_t i[32], v[32];
  wv_store(i, idx);
  wv_store(v, a);
  for (int l = 0; l < 32; l++) ((int32_t *)base)[i[l]] = v[l];
}
WV_INLINE __m256i sl16(__m256i a) { return _mm256_slli_epi32(a, 16); }
WV_INLINE wv wv_slli16(wv a) {
  wv r;
  MAP1(r, a, sl16);
  return r;
}
WV_INLINE __m256i carry8(__m256i q, __m256d c) {
  const __m256 f = _mm256_castsi256_ps(q);
  const __m128 lo = _mm256_cvtpd_ps(_mm256_add_pd(c, _mm256_cvtps_pd(_mm256_castps256_ps128(f))));
  const __m128 hi = _mm256_cvtpd_ps(_mm256_add_pd(c, _mm256_cvtps_pd(_mm256_extractf128_ps(f, 1))));
  return _mm256_castps_si256(_mm256_insertf128_ps(_mm256_castps128_ps256(lo), hi, 1));
}
WV_INLINE wv wv_carry_f64(wv q, double C) {
  const __m256d c = _mm256_set1_pd(C);
  wv r;
  r.q0 = carry8(q.q0, c);
  r.q1 = carry8(q.q1, c);
  r.q2 = carry8(q.q2, c);
  r.q3 = carry8(q.q3, c);
  return r;
}
WV_INLINE int wv_compress_store(void *dst, uint32_t m, wv a) {
  int32_t v[32];
  wv_store(v, a);
  int c = 0;
  for (int l = 0; l < 32; l++)
    if ((m >> l) & 1u) ((int32_t *)dst)[c++] = v[l];
  return c;
}

#else /* scalar lane loops */
typedef struct {
  uint32_t l[32];
} wv;
#define WV_INLINE static inline
WV_INLINE wv wv_load(const void *p) {
  wv r;
  memcpy(r.l, p, 128);
  return r;
}
WV_INLINE void wv_store(void *p, wv a) { memcpy(p, a.l, 128); }
WV_INLINE wv wv_splat(uint32_t x) {
  wv r;
  for (int i = 0; i < 32; i++) r.l[i] = x;
  return r;
}
#define WV_BIN(name, expr)                              \
  WV_INLINE wv name(wv a, wv b) {                       \
    wv r;                                               \
    for (int i = 0; i < 32; i++) {                      \
      const uint32_t x = a.l[i], y = b.l[i];            \
      r.l[i] = (expr);                                  \
    }                                                   \
    return r;                                           \
  }
WV_BIN(wv_add, x + y)
WV_BIN(wv_and, x & y)
WV_BIN(wv_or, x | y)
WV_BIN(wv_xor, x ^ y)
WV_BIN(wv_minu, x < y ? x : y)
WV_BIN(wv_maxu, x < y ? y : x)
WV_BIN(wv_fadd, f2u(u2f(x) + u2f(y)))
WV_BIN(wv_fsub, f2u(u2f(x) - u2f(y)))
WV_BIN(wv_fmul, f2u(u2f(x) * u2f(y)))
WV_INLINE wv wv_ffma(wv a, wv b, wv c) {
  wv r;
  for (int i = 0; i < 32; i++) r.l[i] = f2u(fmaf(u2f(a.l[i]), u2f(b.l[i]), u2f(c.l[i])));
  return r;
}
#define WV_PRED(name, expr)                             \
  WV_INLINE uint32_t name(wv a) {                       \
    uint32_t r = 0;                                     \
    for (int i = 0; i < 32; i++) {                      \
      const uint32_t x = a.l[i];                        \
      if (expr) r |= 1u << i;                           \
    }                                                   \
    return r;                                           \
  }
WV_PRED(wv_nz, x != 0)
WV_PRED(wv_gt0_i32, (int32_t)x > 0)
WV_PRED(wv_gt0_f32, u2f(x) > 0.0f)
WV_INLINE uint32_t wv_ltu(wv a, wv b) {
  uint32_t r = 0;
  for (int i = 0; i < 32; i++)
    if (a.l[i] < b.l[i]) r |= 1u << i;
  return r;
}
WV_INLINE uint32_t wv_eq(wv a, wv b) {
  uint32_t r = 0;
  for (int i = 0; i < 32; i++)
    if (a.l[i] == b.l[i]) r |= 1u << i;
  return r;
}
WV_INLINE wv wv_sel(uint32_t m, wv a, wv b) {
  wv r;
  for (int i = 0; i < 32; i++) r.l[i] = ((m >> i) & 1u) ? a.l[i] : b.l[i];
  return r;
}
WV_INLINE wv wv_perm(wv a, wv idx) {
  wv r;
  for (int i = 0; i < 32; i++) r.l[i] = a.l[idx.l[i] & 31u];
  return r;
}
WV_INLINE wv wv_gather(const void *base, wv idx) {
  wv r;
  for (int i = 0; i < 32; i++) memcpy(&r.l[i], (const char *)base + 4 * (int64_t)(int32_t)idx.l[i], 4);
  return r;
}
WV_INLINE wv wv_gather_h(const void *base, wv idx) {
  wv r;
  for (int i = 0; i < 32; i++) {
    uint16_t h;
    memcpy(&h, (const char *)base + 2 * (int64_t)(int32_t)idx.l[i], 2);
    r.l[i] = h;
  }
  return r;
}
WV_INLINE void wv_scatter(void *base, wv idx, wv a) {
  for (int i = 0; i < 32; i++) ((uint32_t *)base)[(int32_t)idx.l[i]] = a.l[i];
}
WV_INLINE wv wv_slli16(wv a) {
  wv r;
  for (int i = 0; i < 32; i++) r.l[i] = a.l[i] << 16;
  return r;
}
WV_INLINE wv wv_carry_f64(wv q, double C) {
  wv r;
  for (int i = 0; i < 32; i++) r.l[i] = f2u((float)(C + (double)u2f(q.l[i])));
  return r;
}
WV_INLINE int wv_compress_store(void *dst, uint32_t m, wv a) {
  int c = 0;
  for (int l = 0; l < 32; l++)
    if ((m >> l) & 1u) ((uint32_t *)dst)[c++] = a.l[l];
  return c;
}
#endif

WV_INLINE uint32_t wv_lane(wv a, int l) {
  uint32_t t[32];
  wv_store(t, a);
  return t[l];
}
WV_INLINE wv wv_fneg(wv a) { return wv_xor(a, wv_splat(NEG0)); }

/* ---------------------------------------------------------------- shuffle index tables */
/* g_src[op][log2 width][arg & 31][l]: the source lane of lane l under the
 * CUDA rules (b = l & ~(width-1)): IDX b + (arg & (width-1)); UP l - arg
 * if l - b >= arg else l; DOWN l + arg if l - b + arg < width else l; XOR
 * l ^ arg if (l ^ arg) < b + width else l. */
static int32_t g_src[4][6][32][32] __attribute__((aligned(64)));
static int32_t g_iota[32] __attribute__((aligned(64)));

static int src_lane(int op, int l, int a, int w) {
  const int b = l & ~(w - 1);
  switch (op) {
  case SH_IDX: return b + (a & (w - 1));
  case SH_UP: return (l - b >= a) ? l - a : l;
  case SH_DOWN: return (l - b + a < w) ? l + a : l;
  default: {
    const int j = l ^ a;
    return j < b + w ? j : l;
  }
  }
}

__attribute__((constructor)) static void coxs_tables(void) {
  for (int op = 0; op < 4; op++)
    for (int lw = 0; lw < 6; lw++)
      for (int a = 0; a < 32; a++)
        for (int l = 0; l < 32; l++) g_src[op][lw][a][l] = src_lane(op, l, a, 1 << lw);
  for (int l = 0; l < 32; l++) g_iota[l] = l;
}

static int log2w(int w) { return __builtin_ctz((unsigned)w); }

/* the warp builtins: every lane reads its source lane (CUDA's own-value
 * rule is in the table); ballot is one bit per lane */
WV_INLINE wv shfl(wv v, int op, int arg, int w) { return wv_perm(v, wv_load(g_src[op][log2w(w)][arg & 31])); }
WV_INLINE uint32_t ballot(wv pred) { return wv_nz(pred); }
WV_INLINE wv iota(void) { return wv_load(g_iota); }
/* lanes l with (l & (w - 1)) >= d (the lanes a Kogge-Stone step adds into) */
static uint32_t lanes_ge(int d, int w) {
  uint32_t m = 0;
  for (int l = 0; l < 32; l++)
    if ((l & (w - 1)) >= d) m |= 1u << l;
  return m;
}

/* ================================================================== */
/* block pool: blocks of a launch spread over the host threads          */
/* ================================================================== */
static int g_threads = 1;

int coxs_set_threads(int n) {
  g_threads = n < 1 ? 1 : (n > 256 ? 256 : n);
  return g_threads;
}
int coxs_get_threads(void) { return g_threads; }
int coxs_isa(void) { return COXS_ISA; }

typedef void (*block_fn)(void *ctx, int64_t b);
typedef struct {
  block_fn fn;
  void *ctx;
  int64_t nblocks, next;
} pool_t;

static void *pool_run(void *p) {
  pool_t *q = (pool_t *)p;
  for (;;) {
    const int64_t b = __atomic_fetch_add(&q->next, 1, __ATOMIC_RELAXED);
    if (b >= q->nblocks) break;
    q->fn(q->ctx, b);
  }
  return NULL;
}

static int launch(int64_t nblocks, block_fn fn, void *ctx) {
  if (nblocks <= 0) return COXS_OK;
  int nt = g_threads;
  if (nt > nblocks) nt = (int)nblocks;
  pool_t q = {fn, ctx, nblocks, 0};
  if (nt <= 1) {
    pool_run(&q);
    return COXS_OK;
  }
  pthread_t th[256];
  int started = 0;
  for (int i = 0; i < nt - 1; i++)
    if (pthread_create(&th[i], NULL, pool_run, &q) == 0) started++;
  pool_run(&q);
  for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
  return COXS_OK;
}

static int sigma_ok(int k, int W) {
  return k >= 1 && k <= 32 && !(k & (k - 1)) && W >= 1 && W <= 32 && !(W & (W - 1));
}
static int width_ok(int w) { return w >= 1 && w <= 32 && !(w & (w - 1)); }

/* ================================================================== */
/* warp builtins applied to arrays                                      */
/* ================================================================== */
typedef struct {
  const int32_t *v, *argv;
  int32_t *out;
  const uint32_t *mask;
  int op, arg, width;
  int ub;
} shfl_job;

static void shfl_warp(void *p, int64_t g) {
  shfl_job *j = (shfl_job *)p;
  const uint32_t m = j->mask ? j->mask[g] : ALL32;
  const wv v = wv_load(j->v + 32 * g);
  wv idx;
  if (j->argv) {
    int32_t s[32] __attribute__((aligned(64)));
    for (int l = 0; l < 32; l++) s[l] = src_lane(j->op, l, j->argv[32 * g + l], j->width);
    idx = wv_load(s);
  } else {
    idx = wv_load(g_src[j->op][log2w(j->width)][j->arg & 31]);
  }
  /* a lane of the mask reading a lane outside it is undefined */
  int32_t s[32];
  wv_store(s, idx);
  for (int l = 0; l < 32; l++)
    if (((m >> l) & 1u) && !((m >> s[l]) & 1u)) __atomic_store_n(&j->ub, 1, __ATOMIC_RELAXED);
  wv_store(j->out + 32 * g, wv_sel(m, wv_perm(v, idx), v));
}

int coxs_warp_shfl(const int32_t *v, int32_t *out, int64_t n, int op, int32_t arg, const int32_t *argv, int width,
                   const uint32_t *mask) {
  if (n < 0 || n % 32 || !width_ok(width) || op < SH_IDX || op > SH_XOR) return COXS_ERR_INVALID;
  if (op != SH_IDX) {
    if (argv) {
      for (int64_t i = 0; i < n; i++)
        if (argv[i] < 0 || argv[i] > 31) return COXS_ERR_INVALID;
    } else if (arg < 0 || arg > 31) {
      return COXS_ERR_INVALID;
    }
  }
  shfl_job j = {v, argv, out, mask, op, arg, width, 0};
  launch(n / 32, shfl_warp, &j);
  return j.ub ? COXS_ERR_UB : COXS_OK;
}

typedef struct {
  const int32_t *pred;
  const uint32_t *mask;
  uint32_t *ballot;
  int32_t *anyall;
} vote_job;

static void vote_warp(void *p, int64_t g) {
  vote_job *j = (vote_job *)p;
  const uint32_t m = j->mask ? j->mask[g] : ALL32;
  const uint32_t b = ballot(wv_load(j->pred + 32 * g)) & m;
  j->ballot[g] = m ? b : 0u;
  j->anyall[g] = m ? ((b != 0) | ((b == m) << 1)) : 0;
}

int coxs_warp_vote(const int32_t *pred, const uint32_t *mask, int64_t n, uint32_t *ballot_out, int32_t *anyall) {
  if (n < 0 || n % 32) return COXS_ERR_INVALID;
  vote_job j = {pred, mask, ballot_out, anyall};
  return launch(n / 32, vote_warp, &j);
}

/* ================================================================== */
/* 256-thread block reduce (8 warps, one element per lane)             */
/* ================================================================== */
typedef struct {
  const int32_t *x;
  int64_t n;
  int32_t *bsum, *wpos;
} r0_job;

static wv load_i32_tail(const int32_t *x, int64_t e, int64_t n, uint32_t pad) {
  if (e + 32 <= n) return wv_load(x + e);
  uint32_t t[32] __attribute__((aligned(64)));
  for (int l = 0; l < 32; l++) t[l] = e + l < n ? (uint32_t)x[e + l] : pad;
  return wv_load(t);
}

static void r0_block(void *p, int64_t b) {
  r0_job *j = (r0_job *)p;
  uint32_t slot[32] __attribute__((aligned(64)));
  memset(slot, 0, sizeof slot);
  for (int w = 0; w < 8; w++) {
    const int64_t e = 256 * b + 32 * w;
    wv v = load_i32_tail(j->x, e, j->n, 0u);
    const uint32_t pos = wv_gt0_i32(v);
    for (int o = 16; o > 0; o >>= 1) v = wv_add(v, shfl(v, SH_DOWN, o, 32));
    if (e < j->n) j->wpos[8 * b + w] = popc(pos);
    slot[w] = wv_lane(v, 0);
  }
  wv a = wv_load(slot);
  for (int o = 16; o > 0; o >>= 1) a = wv_add(a, shfl(a, SH_DOWN, o, 32));
  j->bsum[b] = (int32_t)wv_lane(a, 0);
}

int coxs_reduce_blocks_i32(const int32_t *x, int64_t n, int32_t *block_sums, int32_t *warp_pos) {
  if (n < 0) return COXS_ERR_INVALID;
  r0_job j = {x, n, block_sums, warp_pos};
  return launch((n + 255) / 256, r0_block, &j);
}

/* ================================================================== */
/* element mapping of sigma = (k, W): thread (w, l), row i < k / V,      */
/* slot v < V (V = min(k, 16 bytes / element)) owns chunk offset         */
/*   w * 32k + (i * 32 + l) * V + v.                                    */
/* One (w, i, v) is a warp-wide load: lane l at stride V.               */
/* ================================================================== */
static int vec_width(int k, int dt) {
  const int v = dt == DT_BF16 ? 8 : 4;
  return k < v ? k : v;
}

/* lane offsets l * V for V = 1, 2, 4, 8 */
static int32_t g_lv[4][32] __attribute__((aligned(64)));
__attribute__((constructor)) static void coxs_lane_offsets(void) {
  for (int j = 0; j < 4; j++)
    for (int l = 0; l < 32; l++) g_lv[j][l] = l << j;
}

/* the 32 lanes' binary32 bits (bfloat16 widened) or int32 values at
 * element positions base + l * V; with `full` every position is in range
 * (a gather), else positions at or past `lim` read `pad` */
static wv load_lanes(const void *x, int dt, int64_t base, int V, int64_t lim, uint32_t pad, int full) {
  if (full) {
    const wv li = wv_load(g_lv[log2w(V)]);
    if (dt == DT_BF16) return wv_slli16(wv_gather_h((const uint16_t *)x + base, li));
    return wv_gather((const uint32_t *)x + base, li);
  }
  uint32_t t[32] __attribute__((aligned(64)));
  for (int l = 0; l < 32; l++) {
    const int64_t e = base + (int64_t)l * V;
    if (e >= lim) t[l] = pad;
    else if (dt == DT_BF16) t[l] = (uint32_t)((const uint16_t *)x)[e] << 16;
    else t[l] = ((const uint32_t *)x)[e];
  }
  return wv_load(t);
}

/* ================================================================== */
/* chunked reduce / dot                                                 */
/* ================================================================== */
typedef struct {
  wv s, c; /* binary32 sum and compensation bits, or int32 sum in s */
} acc_t;

typedef struct {
  const void *x, *y;
  int dt, dot, acc, k, W;
  int64_t n, S;
  uint32_t *ps, *pc; /* per chunk: s bits (int32 for I32), c bits */
} red_job;

WV_INLINE void two_sum(wv a, wv b, wv *s, wv *e) {
  const wv ss = wv_fadd(a, b);
  const wv bb = wv_fsub(ss, a);
  *e = wv_fadd(wv_fsub(a, wv_fsub(ss, bb)), wv_fsub(b, bb));
  *s = ss;
}

WV_INLINE acc_t combine(const red_job *j, acc_t a, acc_t b) {
  if (j->dt == DT_I32) {
    a.s = wv_add(a.s, b.s);
  } else if (j->acc == ACC_PLAIN) {
    a.s = wv_fadd(a.s, b.s);
  } else {
    wv s, e;
    two_sum(a.s, b.s, &s, &e);
    a.c = wv_fadd(wv_fadd(a.c, b.c), e);
    a.s = s;
  }
  return a;
}

/* shfl_down tree, offsets 16 .. 1 (lane 0 holds the warp's value) */
WV_INLINE acc_t red_tree(const red_job *j, acc_t a) {
  for (int o = 16; o > 0; o >>= 1) {
    acc_t b;
    b.s = shfl(a.s, SH_DOWN, o, 32);
    b.c = j->acc == ACC_TWOSUM ? shfl(a.c, SH_DOWN, o, 32) : a.c;
    a = combine(j, a, b);
  }
  return a;
}

static void red_chunk(void *p, int64_t c) {
  red_job *j = (red_job *)p;
  const int k = j->k, W = j->W, V = vec_width(k, j->dt), R = k / V;
  const int64_t e0 = c * j->S;
  /* bf16 gathers read 4 bytes at an element's address: stay 1 element
   * short of the end */
  const int full = j->dt == DT_BF16 ? (e0 + j->S < j->n) : (e0 + j->S <= j->n);
  const uint32_t id = j->dt == DT_I32 ? 0u : NEG0;
  uint32_t slot_s[32] __attribute__((aligned(64))), slot_c[32] __attribute__((aligned(64)));
  for (int l = 0; l < 32; l++) slot_s[l] = slot_c[l] = id;
  for (int w = 0; w < W; w++) {
    acc_t a;
    a.s = a.c = wv_splat(id);
    for (int i = 0; i < R; i++)
      for (int v = 0; v < V; v++) {
        const int64_t base = e0 + (int64_t)w * 32 * k + (int64_t)i * 32 * V + v;
        const wv x = load_lanes(j->x, j->dt, base, V, j->n, j->dt == DT_I32 ? 0u : NEG0, full);
        if (j->dt == DT_I32) {
          a.s = wv_add(a.s, x);
        } else if (!j->dot) {
          if (j->acc == ACC_PLAIN) {
            a.s = wv_fadd(a.s, x);
          } else {
            wv s, e;
            two_sum(a.s, x, &s, &e);
            a.s = s;
            a.c = wv_fadd(a.c, e);
          }
        } else {
          const wv y = load_lanes(j->y, j->dt, base, V, j->n, 0u, full); /* y pads +0.0 */
          if (j->acc == ACC_PLAIN) {
            a.s = wv_ffma(x, y, a.s);
          } else {
            const wv pr = wv_fmul(x, y);
            const wv pe = wv_ffma(x, y, wv_fneg(pr)); /* TwoProduct */
            wv s, q;
            two_sum(a.s, pr, &s, &q);
            a.s = s;
            a.c = wv_fadd(a.c, wv_fadd(pe, q));
          }
        }
      }
    a = red_tree(j, a);
    slot_s[w] = wv_lane(a.s, 0);
    slot_c[w] = wv_lane(a.c, 0);
  }
  acc_t b;
  b.s = wv_load(slot_s);
  b.c = wv_load(slot_c);
  b = red_tree(j, b);
  j->ps[c] = wv_lane(b.s, 0);
  j->pc[c] = wv_lane(b.c, 0);
}

/* FP64 final combine shaped like a 256-thread block: thread t sums values
 * t, t + 256, ... serially from -0.0; the shfl_down tree (16 .. 1) in each
 * of the 8 warps; the same tree over the 8 warp values (-0.0 beyond). */
static double final_tree(const double *val, int64_t nch) {
  double t[256];
  for (int th = 0; th < 256; th++) t[th] = -0.0;
  for (int64_t c0 = 0; c0 < nch; c0 += 256) {
    const int64_t m = nch - c0 < 256 ? nch - c0 : 256;
    for (int th = 0; th < m; th++) t[th] = t[th] + val[c0 + th];
  }
  double top[32];
  for (int w = 0; w < 32; w++) top[w] = -0.0;
  for (int w = 0; w < 8; w++) {
    double *a = t + 32 * w;
    for (int o = 16; o > 0; o >>= 1)
      for (int l = 0; l < o; l++) a[l] = a[l] + a[l + o];
    top[w] = a[0];
  }
  for (int o = 16; o > 0; o >>= 1)
    for (int l = 0; l < o; l++) top[l] = top[l] + top[l + o];
  return top[0];
}

static int reduce_any(const void *x, const void *y, int dt, int dot, int64_t n, int acc, int k, int W,
                      void *partials, void *total) {
  if (n < 0 || !sigma_ok(k, W) || (acc != ACC_PLAIN && acc != ACC_TWOSUM)) return COXS_ERR_INVALID;
  if (dt != DT_I32 && dt != DT_F32 && dt != DT_BF16) return COXS_ERR_DTYPE;
  if (dt == DT_I32 && (acc != ACC_PLAIN || dot)) return COXS_ERR_DTYPE;
  const int64_t S = (int64_t)32 * W * k, nch = (n + S - 1) / S;
  uint32_t *ps = (uint32_t *)malloc(8 * (size_t)(nch + 1));
  if (!ps) return COXS_ERR_NOMEM;
  red_job j = {x, y, dt, dot, acc, k, W, n, S, ps, ps + nch + 1};
  launch(nch, red_chunk, &j);
  if (dt == DT_I32) {
    int64_t tot = 0;
    for (int64_t c = 0; c < nch; c++) {
      tot += (int64_t)(int32_t)ps[c];
      if (partials) ((uint32_t *)partials)[c] = ps[c];
    }
    *(int64_t *)total = tot;
  } else {
    double *val = (double *)malloc(8 * (size_t)(nch + 1));
    if (!val) {
      free(ps);
      return COXS_ERR_NOMEM;
    }
    for (int64_t c = 0; c < nch; c++) {
      const uint32_t pcv = (j.pc)[c];
      val[c] = acc == ACC_TWOSUM ? (double)u2f(ps[c]) + (double)u2f(pcv) : (double)u2f(ps[c]);
      if (partials) {
        if (acc == ACC_TWOSUM) {
          ((uint32_t *)partials)[2 * c] = ps[c];
          ((uint32_t *)partials)[2 * c + 1] = pcv;
        } else {
          ((uint32_t *)partials)[c] = ps[c];
        }
      }
    }
    *(double *)total = final_tree(val, nch);
    free(val);
  }
  free(ps);
  return COXS_OK;
}

int coxs_reduce(const void *x, int dtype, int64_t n, int acc, int k, int W, void *partials, void *total) {
  return reduce_any(x, NULL, dtype, 0, n, acc, k, W, partials, total);
}

int coxs_dot(const void *a, const void *b, int dtype, int64_t n, int acc, int k, int W, void *partials,
             double *total) {
  if (dtype != DT_F32 && dtype != DT_BF16) return COXS_ERR_DTYPE;
  return reduce_any(a, b, dtype, 1, n, acc, k, W, partials, total);
}


/* ================================================================== */
/* chunk scan (int32 wrapping or binary32) by the schedule's tree:       */
/*   per warp and row i: z_v = the lane's inclusive prefix of its V      */
/*   elements, r = z_{V-1}; Kogge-Stone shfl_up(r, d, width 16) for      */
/*   d = 1, 2, 4, 8 into lanes (l & 15) >= d; lanes 16-31 add lane 15    */
/*   (shfl index 15); ex = shfl_up(r, 1) for lanes >= 1; the row total   */
/*   rt is lane 31; the warp carry is C_0 = none, C_{i+1} = C_i + rt_i.  */
/*   Warp 0 scans the warp totals with the same tree and E_w is its      */
/*   shfl_up(., 1) (w >= 1).  q = ((E_w + C_i) + ex) + z_v.              */
/* Absent terms are the identity: 0, or -0.0 for binary32, which leaves  */
/* every value unchanged, so adding it is skipping it.                   */
/* ================================================================== */
WV_INLINE wv sadd(int isf, wv a, wv b) { return isf ? wv_fadd(a, b) : wv_add(a, b); }

/* inclusive scan of *r over the warp; *ex = shfl_up(r, 1) with the
 * identity in lane 0; returns lane 31 */
static uint32_t scan32(int isf, wv *r, wv *ex, uint32_t id) {
  for (int d = 1; d <= 8; d <<= 1) {
    const wv t = shfl(*r, SH_UP, d, 16);
    *r = wv_sel(lanes_ge(d, 16), sadd(isf, *r, t), *r);
  }
  const wv t = shfl(*r, SH_IDX, 15, 32);
  *r = wv_sel(0xffff0000u, sadd(isf, *r, t), *r);
  *ex = wv_sel(0xfffffffeu, shfl(*r, SH_UP, 1, 32), wv_splat(id));
  return wv_lane(*r, 31);
}

typedef struct {
  int isf;
  const void *x;
  int k, W;
} scan_kind;

/* per-call scratch of a chunk scan: z[S], ex[S / V], carries [W * R] */
typedef struct {
  uint32_t *z, *ex, *carry;
} scan_tmp;

static int scan_tmp_alloc(scan_tmp *t, int64_t S) {
  t->z = (uint32_t *)aligned_alloc(64, 4 * (size_t)S * 2 + 4 * 1024 + 64);
  if (!t->z) return 0;
  t->ex = t->z + S;
  t->carry = t->z + 2 * S;
  return 1;
}

/* q at every slot of chunk [e0, e0 + S) (clipped loads past e1) into
 * q_out[0 .. S); returns q at the chunk's last slot */
static uint32_t scan_chunk(const scan_kind *sk, int64_t e0, int64_t e1, uint32_t *q_out, scan_tmp *tmp) {
  const int isf = sk->isf, k = sk->k, W = sk->W;
  const int dt = isf ? DT_F32 : DT_I32;
  const int V = vec_width(k, dt), R = k / V;
  const uint32_t id = isf ? NEG0 : 0u;
  const int64_t S = (int64_t)32 * W * k;
  const int full = e0 + S <= e1;
  uint32_t slot[32] __attribute__((aligned(64)));
  for (int l = 0; l < 32; l++) slot[l] = id;
  /* block region 1: z, ex and the row carries of every warp */
  for (int w = 0; w < W; w++) {
    wv C = wv_splat(id);
    for (int i = 0; i < R; i++) {
      const int64_t base = (int64_t)w * 32 * k + (int64_t)i * 32 * V;
      wv z = wv_splat(id);
      for (int v = 0; v < V; v++) {
        const wv x = load_lanes(sk->x, dt, e0 + base + v, V, e1, id, full);
        z = v == 0 ? x : sadd(isf, z, x);
        wv_store(tmp->z + base + 32 * v, z); /* [w][i][v][lane] */
      }
      wv r = z, ex;
      const uint32_t rt = scan32(isf, &r, &ex, id);
      wv_store(tmp->ex + (int64_t)(w * R + i) * 32, ex);
      tmp->carry[w * R + i] = wv_lane(C, 0);
      C = sadd(isf, C, wv_splat(rt));
    }
    slot[w] = wv_lane(C, 0);
  }
  /* block barrier; region 2: warp 0 scans the warp totals */
  wv a = wv_load(slot), exw;
  scan32(isf, &a, &exw, id);
  uint32_t E[32] __attribute__((aligned(64)));
  wv_store(E, exw); /* E[0] is the identity */
  /* block barrier; region 3: element values, written at their offsets */
  uint32_t total = id;
  for (int w = 0; w < W; w++)
    for (int i = 0; i < R; i++) {
      const int64_t base = (int64_t)w * 32 * k + (int64_t)i * 32 * V;
      const wv head = sadd(isf, sadd(isf, wv_splat(E[w]), wv_splat(tmp->carry[w * R + i])),
                           wv_load(tmp->ex + (int64_t)(w * R + i) * 32));
      for (int v = 0; v < V; v++) {
        const wv q = sadd(isf, head, wv_load(tmp->z + base + 32 * v));
        wv_scatter(q_out + base + v, wv_load(g_lv[log2w(V)]), q);
        if (w == W - 1 && i == R - 1 && v == V - 1) total = wv_lane(q, 31);
      }
    }
  return total;
}

/* flat int32 inclusive scan: chunk scans, then the chunk carries (wrapping
 * sums of the earlier chunk totals, in chunk order) added */
typedef struct {
  scan_kind sk;
  int64_t n, S;
  int32_t *y;
  uint32_t *ctot;
  const uint32_t *carry;
  int err;
} scan_job;

static void scan_pass1(void *p, int64_t c) {
  scan_job *j = (scan_job *)p;
  const int64_t e0 = c * j->S;
  scan_tmp t;
  uint32_t *q = (uint32_t *)aligned_alloc(64, 4 * (size_t)j->S);
  if (!q || !scan_tmp_alloc(&t, j->S)) {
    free(q);
    j->err = COXS_ERR_NOMEM;
    return;
  }
  j->ctot[c] = scan_chunk(&j->sk, e0, j->n, q, &t);
  const int64_t m = j->n - e0 < j->S ? j->n - e0 : j->S;
  memcpy(j->y + e0, q, 4 * (size_t)m);
  free(t.z);
  free(q);
}

static void scan_pass2(void *p, int64_t c) {
  scan_job *j = (scan_job *)p;
  const int64_t e0 = c * j->S;
  const int64_t m = j->n - e0 < j->S ? j->n - e0 : j->S;
  const wv cr = wv_splat(j->carry[c]);
  int64_t o = 0;
  for (; o + 32 <= m; o += 32) wv_store(j->y + e0 + o, wv_add(cr, wv_load(j->y + e0 + o)));
  for (; o < m; o++) j->y[e0 + o] = (int32_t)(j->carry[c] + (uint32_t)j->y[e0 + o]);
}

int coxs_scan_i32(const int32_t *x, int32_t *y, int64_t n, int k, int W) {
  if (n < 0 || !sigma_ok(k, W)) return COXS_ERR_INVALID;
  const int64_t S = (int64_t)32 * W * k, nch = (n + S - 1) / S;
  uint32_t *ctot = (uint32_t *)malloc(8 * (size_t)(nch + 1));
  if (!ctot) return COXS_ERR_NOMEM;
  uint32_t *carry = ctot + nch + 1;
  scan_job j = {{0, x, k, W}, n, S, y, ctot, carry, 0};
  launch(nch, scan_pass1, &j);
  uint32_t run = 0;
  for (int64_t c = 0; c < nch; c++) {
    carry[c] = run;
    run += ctot[c];
  }
  launch(nch, scan_pass2, &j);
  free(ctot);
  return j.err;
}

/* ================================================================== */
/* ballot compaction (keep x > 0, stable).  Per warp and row the V       */
/* ballots B_v = ballot(x_v > 0) give the row count sum_v popc(B_v) and  */
/* lane l's rank sum_v popc(B_v & lanemask_lt(l)) plus its own earlier   */
/* slots: the kept elements of a row in the order of their offsets,     */
/* which is how they are written (a compress store of the row).         */
/* ================================================================== */
typedef struct {
  int isf;
  const void *x;
  int k, W;
} cmp_kind;

/* kept elements of one row (32 V consecutive elements at p, m of them
 * valid) written at dst in order; returns how many */
static int64_t compact_row(int isf, const uint32_t *p, int64_t m, uint32_t *dst) {
  int64_t c = 0, o = 0;
  for (; o + 32 <= m; o += 32) {
    const wv v = wv_load(p + o);
    const uint32_t keep = isf ? wv_gt0_f32(v) : wv_gt0_i32(v);
    if (dst) wv_compress_store(dst + c, keep, v);
    c += popc(keep);
  }
  for (; o < m; o++) {
    const uint32_t u = p[o];
    const int keep = isf ? u2f(u) > 0.0f : (int32_t)u > 0;
    if (keep) {
      if (dst) dst[c] = u;
      c++;
    }
  }
  return c;
}

/* the chunk's kept count (per warp and row: the ballots' popcounts); with
 * dst, the kept elements written from dst[0] */
static int64_t compact_chunk(const cmp_kind *ck, int64_t e0, int64_t e1, uint32_t *dst) {
  const int k = ck->k, W = ck->W;
  const int dt = ck->isf ? DT_F32 : DT_I32;
  const int V = vec_width(k, dt), R = k / V;
  const int64_t S = (int64_t)32 * W * k;
  const int full = e0 + S <= e1;
  int64_t kept = 0;
  for (int w = 0; w < W; w++)
    for (int i = 0; i < R; i++) {
      const int64_t base = e0 + (int64_t)w * 32 * k + (int64_t)i * 32 * V;
      if (base >= e1) continue;
      if (dst) {
        const int64_t m = e1 - base < 32 * V ? e1 - base : 32 * V;
        kept += compact_row(ck->isf, (const uint32_t *)ck->x + base, m, dst + kept);
      } else {
        for (int v = 0; v < V; v++) {
          const wv x = load_lanes(ck->x, dt, base + v, V, e1, 0u, full);
          kept += popc(ck->isf ? wv_gt0_f32(x) : wv_gt0_i32(x));
        }
      }
    }
  return kept;
}

typedef struct {
  cmp_kind ck;
  int64_t n, S;
  int64_t *cnt;
  const int64_t *off;
  int32_t *out;
} cmp_job;

static void cmp_pass1(void *p, int64_t c) {
  cmp_job *j = (cmp_job *)p;
  j->cnt[c] = compact_chunk(&j->ck, c * j->S, j->n, NULL);
}
static void cmp_pass2(void *p, int64_t c) {
  cmp_job *j = (cmp_job *)p;
  compact_chunk(&j->ck, c * j->S, j->n, (uint32_t *)j->out + j->off[c]);
}

int coxs_compact_i32(const int32_t *x, int64_t n, int32_t *out, int64_t *count, int k, int W) {
  if (n < 0 || !sigma_ok(k, W)) return COXS_ERR_INVALID;
  const int64_t S = (int64_t)32 * W * k, nch = (n + S - 1) / S;
  int64_t *cnt = (int64_t *)malloc(16 * (size_t)(nch + 1));
  if (!cnt) return COXS_ERR_NOMEM;
  int64_t *off = cnt + nch + 1;
  cmp_job j = {{0, x, k, W}, n, S, cnt, off, out};
  launch(nch, cmp_pass1, &j);
  int64_t run = 0;
  for (int64_t c = 0; c < nch; c++) {
    off[c] = run;
    run += cnt[c];
  }
  launch(nch, cmp_pass2, &j);
  *count = run;
  free(cnt);
  return COXS_OK;
}

/* ================================================================== */
/* tile sort: groups of G keys (G lanes of a width-G tile) ascending,    */
/* unsigned, by the bitonic network: for k2 = 2 .. G, j = k2/2 .. 1:     */
/* o = shfl_xor(key, j, G); lanes with ((lt & j) == 0) == ((lt & k2) ==  */
/* 0) keep min(key, o), the others max (lt = lane within the tile).     */
/* A partial last warp is padded with UINT32_MAX, which sorts last and   */
/* is not written.                                                      */
/* ================================================================== */
typedef struct {
  const uint32_t *keys;
  uint32_t *out;
  int64_t n;
  int G;
} sort_job;

static void sort_warp(void *p, int64_t g) {
  sort_job *j = (sort_job *)p;
  const int G = j->G;
  const int64_t e = 32 * g;
  wv key = load_i32_tail((const int32_t *)j->keys, e, j->n, 0xffffffffu);
  for (int k2 = 2; k2 <= G; k2 <<= 1)
    for (int jj = k2 >> 1; jj > 0; jj >>= 1) {
      const wv o = shfl(key, SH_XOR, jj, G);
      uint32_t keep_min = 0;
      for (int l = 0; l < 32; l++) {
        const int lt = l & (G - 1);
        if (((lt & jj) == 0) == ((lt & k2) == 0)) keep_min |= 1u << l;
      }
      key = wv_sel(keep_min, wv_minu(key, o), wv_maxu(key, o));
    }
  if (e + 32 <= j->n) {
    wv_store(j->out + e, key);
  } else {
    uint32_t t[32];
    wv_store(t, key);
    for (int l = 0; e + l < j->n; l++) j->out[e + l] = t[l];
  }
}

int coxs_tile_sort_u32(const uint32_t *keys, uint32_t *out, int64_t n, int G) {
  if (n < 0 || G < 2 || !width_ok(G)) return COXS_ERR_INVALID;
  sort_job j = {keys, out, n, G};
  return launch((n + 31) / 32, sort_warp, &j);
}

/* ================================================================== */
/* tile<T> reduce: out[g] = wrap32 sum of x[gT .. gT+T-1] (zero pads) by */
/* tile.shfl_down(v, o), o = T/2 .. 1; the tile's first lane stores.    */
/* ================================================================== */
typedef struct {
  const int32_t *x;
  int64_t n;
  int T;
  int32_t *out;
} tred_job;

static void tred_warp(void *p, int64_t g) {
  tred_job *j = (tred_job *)p;
  const int T = j->T;
  const int64_t e = 32 * g;
  wv v = load_i32_tail(j->x, e, j->n, 0u);
  for (int o = T >> 1; o > 0; o >>= 1) v = wv_add(v, shfl(v, SH_DOWN, o, T));
  uint32_t t[32];
  wv_store(t, v);
  const int64_t nt = (j->n + T - 1) / T;
  for (int l = 0; l < 32; l += T) {
    const int64_t tile = (e + l) / T;
    if (tile < nt) j->out[tile] = (int32_t)t[l];
  }
}

int coxs_tile_reduce_i32(const int32_t *x, int64_t n, int T, int32_t *out) {
  if (n < 0 || T < 2 || !width_ok(T)) return COXS_ERR_INVALID;
  tred_job j = {x, n, T, out};
  return launch((n + 31) / 32, tred_warp, &j);
}

/* ================================================================== */
/* masked warp operations with predicate-derived masks; lane l of warp g:*/
/*   p = ((uint32)x & 1023) < D;  m = ballot(p);                        */
/*   lanes of m: b = ballot(m, x > 0); A = any(m, ((x >> 10) & 31) == 0);*/
/*   L = all(m, ((x >> 15) & 31) != 0); s = shfl(m, x, the next lane of  */
/*   m above l, wrapping); bc = shfl(m, x, ffs(m) - 1); out = s;         */
/*   lane ffs(m) - 1 stores rec[g] = {m, b, A | L << 1, bc};            */
/*   other lanes out = INT32_MIN; with m == 0 rec[g] = {0, 0, 0, 0}.     */
/* The divergent region is the lanes of m: the votes see only them (the */
/* ballot is masked by m) and only they keep the shuffle's result.      */
/* ================================================================== */
typedef struct {
  const int32_t *x;
  int D;
  int32_t *out;
  uint32_t *rec;
} mask_job;

static void mask_warp(void *p, int64_t g) {
  mask_job *j = (mask_job *)p;
  const wv x = wv_load(j->x + 32 * g);
  const uint32_t m = wv_ltu(wv_and(x, wv_splat(1023u)), wv_splat((uint32_t)j->D));
  uint32_t *r = j->rec + 4 * g;
  if (!m) {
    wv_store(j->out + 32 * g, wv_splat(0x80000000u));
    r[0] = r[1] = r[2] = r[3] = 0;
    return;
  }
  const uint32_t b = wv_gt0_i32(x) & m;
  const wv f10 = wv_and(x, wv_splat(31u << 10)), f15 = wv_and(x, wv_splat(31u << 15));
  const uint32_t A = (~wv_nz(f10) & m) != 0; /* some lane of m has bits 10-14 zero */
  const uint32_t L = (wv_nz(f15) & m) == m;  /* every lane of m has bits 15-19 nonzero */
  int32_t src[32] __attribute__((aligned(64)));
  const int lead = __builtin_ctz(m);
  for (int l = 0; l < 32; l++) {
    const uint32_t above = l == 31 ? 0u : (m & (ALL32 << (l + 1)));
    src[l] = above ? __builtin_ctz(above) : lead;
  }
  const wv s = wv_perm(x, wv_load(src));
  wv_store(j->out + 32 * g, wv_sel(m, s, wv_splat(0x80000000u)));
  r[0] = m;
  r[1] = b;
  r[2] = A | (L << 1);
  r[3] = (uint32_t)j->x[32 * g + lead];
}

int coxs_warp_masked(const int32_t *x, int64_t n, int D, int32_t *out, uint32_t *rec) {
  if (n < 0 || n % 32 || D < 0 || D > 1024) return COXS_ERR_INVALID;
  mask_job j = {x, D, out, rec};
  return launch(n / 32, mask_warp, &j);
}

/* ================================================================== */
/* segmented reduce + scan + compaction over CSR segments: chunks of    */
/* S = 32 W k elements from each segment's first element (the last one  */
/* padded); per chunk the reduce partial P_j (the reduce tree), the     */
/* chunk scan q with its total T_j (the scan tree) and the compaction.  */
/* int32: total = sum of (int64) P_j; y = carry_j + q (wrapping).        */
/* binary32: total = FP64 serial sum of P_j from -0.0; y = (float)(C_j + */
/* (double) q), C_0 = -0.0, C_{j+1} = C_j + (double) T_j.                */
/* Compaction: the kept elements (x > 0) of segment s from out[off[s]];  */
/* seg_count[s] their number.  Empty segments: identity total, count 0. */
/* ================================================================== */
typedef struct {
  int isf;
  const void *x;
  const int64_t *off;
  int k, W;
  void *seg_total, *y, *outc;
  int64_t *seg_count;
  int err;
} seg_job;

static void seg_one(void *p, int64_t s) {
  seg_job *j = (seg_job *)p;
  const int isf = j->isf;
  const int64_t S = (int64_t)32 * j->W * j->k;
  const int64_t a = j->off[s], e1 = j->off[s + 1];
  uint32_t part_s, part_c;
  red_job rj = {j->x, NULL, isf ? DT_F32 : DT_I32, 0, ACC_PLAIN, j->k, j->W, e1, S, &part_s, &part_c};
  const scan_kind sk = {isf, j->x, j->k, j->W};
  const cmp_kind ck = {isf, j->x, j->k, j->W};
  uint32_t *q = (uint32_t *)aligned_alloc(64, 4 * (size_t)S);
  scan_tmp t;
  if (!q || !scan_tmp_alloc(&t, S)) {
    free(q);
    j->err = COXS_ERR_NOMEM;
    return;
  }
  int64_t itot = 0, kept = 0;
  double ftot = -0.0, fcarry = -0.0;
  uint32_t icarry = 0;
  for (int64_t e0 = a; e0 < e1; e0 += S) {
    /* the reduce of chunk [e0, e0 + S) clipped at e1: red_chunk indexes
     * chunks from 0, so shift its base by e0 */
    red_job rc = rj;
    rc.x = isf ? (const void *)((const float *)j->x + e0) : (const void *)((const int32_t *)j->x + e0);
    rc.n = e1 - e0;
    red_chunk(&rc, 0);
    if (isf) ftot = ftot + (double)u2f(part_s);
    else itot += (int64_t)(int32_t)part_s;
    const uint32_t T = scan_chunk(&sk, e0, e1, q, &t);
    const int64_t m = e1 - e0 < S ? e1 - e0 : S;
    int64_t o = 0;
    if (isf) {
      float *y = (float *)j->y + e0;
      for (; o + 32 <= m; o += 32) wv_store(y + o, wv_carry_f64(wv_load(q + o), fcarry));
      for (; o < m; o++) y[o] = (float)(fcarry + (double)u2f(q[o]));
      fcarry = fcarry + (double)u2f(T);
    } else {
      int32_t *y = (int32_t *)j->y + e0;
      const wv cr = wv_splat(icarry);
      for (; o + 32 <= m; o += 32) wv_store(y + o, wv_add(cr, wv_load(q + o)));
      for (; o < m; o++) y[o] = (int32_t)(icarry + q[o]);
      icarry += T;
    }
    kept += compact_chunk(&ck, e0, e1, (uint32_t *)j->outc + a + kept);
  }
  if (isf) ((double *)j->seg_total)[s] = ftot;
  else ((int64_t *)j->seg_total)[s] = itot;
  j->seg_count[s] = kept;
  free(t.z);
  free(q);
}

int coxs_segmented(const void *x, int dtype, const int64_t *off, int64_t nseg, int k, int W, void *seg_total,
                   void *y, void *out_compact, int64_t *seg_count) {
  if (nseg < 0 || !sigma_ok(k, W)) return COXS_ERR_INVALID;
  if (dtype != DT_I32 && dtype != DT_F32) return COXS_ERR_DTYPE;
  for (int64_t s = 0; s < nseg; s++)
    if (off[s] < 0 || off[s + 1] < off[s]) return COXS_ERR_INVALID;
  seg_job j = {dtype == DT_F32, x, off, k, W, seg_total, y, out_compact, seg_count, 0};
  launch(nseg, seg_one, &j);
  return j.err;
}

/* ================================================================== */
/* the vote builtins alone: warp_any / warp_all over a 32-entry flag     */
/* array, the runtime functions whose time per call with and without    */
/* AVX the paper reports (Table 2).  The calls walk 256 prepared flag   */
/* arrays (32 KiB, cache resident; no store just before a load of the   */
/* same array); returns nanoseconds per call.                           */
/* ================================================================== */
__attribute__((noinline)) static int warp_any(const int32_t *flags) { return wv_nz(wv_load(flags)) != 0; }
__attribute__((noinline)) static int warp_all(const int32_t *flags) { return wv_nz(wv_load(flags)) == ALL32; }

int coxs_vote_bench(int op, int64_t iters, double *ns_per_call, int64_t *checksum) {
  enum { NSET = 256 };
  if (iters <= 0 || (op != 0 && op != 1) || !ns_per_call) return COXS_ERR_INVALID;
  int32_t *flags = (int32_t *)aligned_alloc(64, sizeof(int32_t) * 32 * NSET);
  if (!flags) return COXS_ERR_NOMEM;
  /* any: mostly-false flags; all: mostly-true flags (the slow cases of the
   * votes: every lane has to be looked at) */
  uint32_t h = 2112100340u;
  for (int i = 0; i < 32 * NSET; i++) {
    h = h * 1664525u + 1013904223u;
    const int rare = (h >> 24) < 8; /* about 1 in 32 */
    flags[i] = op == 0 ? rare : !rare;
  }
  int64_t sum = 0;
  struct timespec t0, t1;
  clock_gettime(CLOCK_MONOTONIC, &t0);
  for (int64_t it = 0; it < iters; it++) {
    const int32_t *f = flags + 32 * (it & (NSET - 1));
    sum += op == 0 ? warp_any(f) : warp_all(f);
  }
  clock_gettime(CLOCK_MONOTONIC, &t1);
  *ns_per_call = ((double)(t1.tv_sec - t0.tv_sec) * 1e9 + (double)(t1.tv_nsec - t0.tv_nsec)) / (double)iters;
  if (checksum) *checksum = sum;
  free(flags);
  return COXS_OK;
}
