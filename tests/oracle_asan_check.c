/*
 * Runs every oracle entry point on small random inputs with buffers of exactly
 * the documented sizes, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py builds and runs
 * it).  Also checks facts that need no reference: noiseless input decodes to
 * the message (full frame), the 16-bit modulo decoder agrees with the exact
 * integer one, the blocked decoder's bits do not depend on the thread count,
 * and de-puncturing rejects a wrong input count.
 * Exit status 0 and "OK" on stdout when every call returned 0 and every check
 * held.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "vref.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64(void) { /* xorshift64* */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return rng_state * 0x2545f4914f6cdd1dull;
}
static double uniform(void) { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

static int failures = 0;
#define CHECK(cond, ...)                  \
  do {                                    \
    if (!(cond)) {                        \
      printf("FAIL: " __VA_ARGS__);       \
      printf("\n");                       \
      ++failures;                         \
    }                                     \
  } while (0)

static void *xmalloc(size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p) {
    printf("FAIL: out of memory\n");
    exit(2);
  }
  return p;
}

typedef struct {
  int k, beta;
  uint32_t gen[4];
} code_def;

static const code_def codes[] = {
    {3, 2, {05, 07}},     {4, 4, {013, 015, 017, 011}}, {5, 2, {023, 035}},
    {6, 2, {053, 075}},   {7, 2, {0171, 0133}},         {7, 3, {0133, 0171, 0165}},
    {8, 2, {0247, 0371}}, {9, 2, {0561, 0753}},
};

static void run_code(const code_def *cd, int64_t n, int terminated) {
  vref_code c;
  memset(&c, 0, sizeof(c));
  c.k = cd->k;
  c.beta = cd->beta;
  for (int b = 0; b < cd->beta; ++b) c.gen[b] = cd->gen[b];
  const int64_t N = n + (terminated ? c.k - 1 : 0);
  const int64_t cnt = N * c.beta;

  uint8_t *bits = xmalloc((size_t)n);
  for (int64_t i = 0; i < n; ++i) bits[i] = (uint8_t)(next_u64() & 1u);
  uint8_t *coded = xmalloc((size_t)cnt);
  CHECK(vref_encode(&c, bits, n, terminated, coded) == 0, "encode k=%d", c.k);

  float *lf = xmalloc(sizeof(float) * (size_t)cnt);
  float *lclean = xmalloc(sizeof(float) * (size_t)cnt);
  double *ld = xmalloc(sizeof(double) * (size_t)cnt);
  int8_t *lq = xmalloc((size_t)cnt);
  for (int64_t i = 0; i < cnt; ++i) {
    const double s = coded[i] ? -1.0 : 1.0;
    lclean[i] = (float)(2.0 * s);
    lf[i] = (float)(s + 3.0 * (uniform() - 0.5));
    ld[i] = lf[i];
  }
  CHECK(vref_quantize_i8(lf, cnt, 20.0f, lq) == 0, "quantize");

  uint8_t *o1 = xmalloc((size_t)n), *o2 = xmalloc((size_t)n);
  float mf;
  double md;
  int64_t mi;
  int16_t m16;
  /* full frame: noiseless input gives the message back */
  CHECK(vref_decode_full_f32(&c, lclean, n, terminated, o1, &mf) == 0, "full f32");
  CHECK(memcmp(o1, bits, (size_t)n) == 0, "noiseless full frame k=%d n=%lld", c.k, (long long)n);
  CHECK(vref_decode_full_f32(&c, lf, n, terminated, o1, &mf) == 0, "full f32 noisy");
  CHECK(vref_decode_full_f64(&c, ld, n, terminated, o1, &md) == 0, "full f64");
  CHECK(vref_decode_full_i8(&c, lq, n, terminated, o1, &mi) == 0, "full i8");
  CHECK(vref_decode_full_i16mod(&c, lq, n, terminated, o2, &m16) == 0, "full i16mod");
  CHECK(memcmp(o1, o2, (size_t)n) == 0, "i16mod != i8 k=%d", c.k);

  /* blocked, several geometries; thread count does not change the bits */
  const int64_t Ls[] = {1, 7, 64, n};
  const int64_t vs[][2] = {{0, 0}, {0, 9}, {5, 0}, {3, 17}, {40, 40}};
  for (size_t a = 0; a < sizeof(Ls) / sizeof(Ls[0]); ++a)
    for (size_t b = 0; b < sizeof(vs) / sizeof(vs[0]); ++b) {
      const int64_t L = Ls[a], v1 = vs[b][0], v2 = vs[b][1];
      CHECK(vref_decode_blocked_f32(&c, lf, n, terminated, L, v1, v2, o1, 1) == 0, "blocked f32");
      CHECK(vref_decode_blocked_f32(&c, lf, n, terminated, L, v1, v2, o2, 3) == 0, "blocked f32 mt");
      CHECK(memcmp(o1, o2, (size_t)n) == 0, "thread count changed the bits");
      CHECK(vref_decode_blocked_f64(&c, ld, n, terminated, L, v1, v2, o1, 2) == 0, "blocked f64");
      CHECK(vref_decode_blocked_i8(&c, lq, n, terminated, L, v1, v2, o1, 2) == 0, "blocked i8");
      const int64_t FW[][2] = {{1, 0}, {1, 1}, {3, 2}, {8, 25}, {1000, 2}};
      for (size_t f = 0; f < sizeof(FW) / sizeof(FW[0]); ++f)
        for (int rule = VREF_PT_STORED; rule <= VREF_PT_RANDOM; ++rule) {
          CHECK(vref_decode_blocked_pt_f32(&c, lf, n, terminated, L, v1, v2, FW[f][0], FW[f][1], rule, 7u, o1, 2) ==
                    0,
                "pt f32");
          CHECK(vref_decode_blocked_pt_i8(&c, lq, n, terminated, L, v1, v2, FW[f][0], FW[f][1], rule, 7u, o2, 1) == 0,
                "pt i8");
        }
    }
  /* one window with an emit range inside it */
  if (N >= 4) {
    const int64_t s = 1, e = N - 1, lo = 2, hi = N - 2;
    uint8_t *ow = xmalloc((size_t)(hi - lo));
    CHECK(vref_window_f64(&c, ld, s, e, 0, 0, lo, hi, ow, &md) == 0, "window f64");
    free(ow);
  }
  /* exhaustive search over a small window */
  if (N >= 10) {
    uint8_t ob[10];
    CHECK(vref_bruteforce_window(&c, ld, N - 10, N, 0, terminated, ob, &md) == 0, "bruteforce");
  }
  /* de-puncturing: a period-3 pattern keeping about two thirds of the slots */
  {
    const int period = 3;
    uint8_t *mask = xmalloc((size_t)period * (size_t)c.beta);
    for (int p = 0; p < period * c.beta; ++p) mask[p] = (uint8_t)(p % 3 != 2 || p == 2);
    int64_t kept = 0;
    for (int64_t t = 0; t < N; ++t)
      for (int b = 0; b < c.beta; ++b) kept += mask[(t % period) * c.beta + b];
    float *inf = xmalloc(sizeof(float) * (size_t)kept);
    int8_t *inq = xmalloc((size_t)kept);
    for (int64_t i = 0; i < kept; ++i) {
      inf[i] = lf[i];
      inq[i] = lq[i];
    }
    float *outf = xmalloc(sizeof(float) * (size_t)cnt);
    int8_t *outq = xmalloc((size_t)cnt);
    CHECK(vref_depuncture_f32(inf, kept, mask, period, c.beta, N, outf) == 0, "depuncture f32");
    CHECK(vref_depuncture_i8(inq, kept, mask, period, c.beta, N, outq) == 0, "depuncture i8");
    CHECK(vref_depuncture_f32(inf, kept - 1, mask, period, c.beta, N, outf) == -1, "depuncture count check");
    free(mask);
    free(inf);
    free(inq);
    free(outf);
    free(outq);
  }
  free(bits);
  free(coded);
  free(lf);
  free(lclean);
  free(ld);
  free(lq);
  free(o1);
  free(o2);
}

int main(void) {
  const int64_t ns[] = {1, 2, 9, 63, 200};
  for (size_t i = 0; i < sizeof(codes) / sizeof(codes[0]); ++i)
    for (size_t j = 0; j < sizeof(ns) / sizeof(ns[0]); ++j)
      for (int term = 0; term < 2; ++term) run_code(&codes[i], ns[j], term);
  if (failures) {
    printf("%d checks failed\n", failures);
    return 1;
  }
  printf("OK\n");
  return 0;
}
