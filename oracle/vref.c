/*
 * vref.c -- plain CPU oracle for soft-decision Viterbi decoding.
 *
 * TEST INFRASTRUCTURE ONLY (see vref.h).  Written to be read against the
 * paper, not to be fast: one state at a time, one branch at a time, in the
 * order of Algorithm 1 and Algorithm 2.  No blocking, no fusion, no tricks.
 *
 * Build: cc -std=c11 -O2 -ffp-contract=off -fopenmp -shared -fPIC vref.c
 * (-ffp-contract=off keeps every sum rounded once, as written.)
 */
#include "vref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define VREF_MAX_K 9
#define VREF_MAX_S (1 << (VREF_MAX_K - 1))

static int parity32(uint32_t x) {
  int p = 0;
  while (x) {
    p ^= (int)(x & 1u);
    x >>= 1;
  }
  return p;
}

static int code_ok(const vref_code *c) {
  if (!c || c->k < 3 || c->k > VREF_MAX_K || c->beta < 2 || c->beta > 4) return 0;
  for (int b = 0; b < c->beta; ++b)
    if (c->gen[b] == 0 || c->gen[b] >= (1u << c->k)) return 0;
  return 1;
}

/* Sec. II-A, eq. (1).  The encoder register holds in_t in bit k-1 and
 * in_{t-k+1} in bit 0, so output bit b = XOR of the register bits selected
 * by gen[b] = parity(gen[b] & register). */
static unsigned register_output(const vref_code *c, uint32_t reg) {
  unsigned a = 0;
  for (int b = 0; b < c->beta; ++b) a |= (unsigned)parity32(c->gen[b] & reg) << b;
  return a;
}

int vref_encode(const vref_code *code, const uint8_t *bits, int64_t n,
                int32_t terminated, uint8_t *coded) {
  if (!code_ok(code) || n < 0 || (n > 0 && (!bits || !coded))) return -1;
  const int64_t N = n + (terminated ? code->k - 1 : 0);
  uint32_t reg = 0;
  for (int64_t t = 0; t < N; ++t) {
    const uint32_t in = (t < n) ? (bits[t] & 1u) : 0u; /* tail inputs are 0 */
    reg = (reg >> 1) | (in << (code->k - 1));          /* newest input enters at the top */
    const unsigned a = register_output(code, reg);
    for (int b = 0; b < code->beta; ++b) coded[t * code->beta + b] = (uint8_t)((a >> b) & 1u);
  }
  return 0;
}

/* The encoder FSM (Sec. II-A): a state is the k-1 previous inputs, newest in
 * the MSB.  Taking input u from state i leads to state
 *   j = (u << (k-2)) | (i >> 1),
 * so state j has the two predecessors i = ((j << 1) & (S-1)) | b, b in {0,1},
 * both entered with branch input alpha_in = u = j >> (k-2), and the branch
 * output alpha_out is eq. (1) applied to the register (u << (k-1)) | i. */
typedef struct {
  int S;
  unsigned pred[VREF_MAX_S][2];
  unsigned aout[VREF_MAX_S][2];
} trellis;

static void build_trellis(const vref_code *c, trellis *tr) {
  tr->S = 1 << (c->k - 1);
  for (int j = 0; j < tr->S; ++j) {
    const unsigned u = (unsigned)j >> (c->k - 2);
    for (unsigned b = 0; b < 2; ++b) {
      const unsigned i = (((unsigned)j << 1) & (unsigned)(tr->S - 1)) | b;
      tr->pred[j][b] = i;
      tr->aout[j][b] = register_output(c, (u << (c->k - 1)) | i);
    }
  }
}

/* eq. (2): delta = sum over b of (-1)^alpha_out[b] * llr_t[b], summed in the
 * order b = 0, 1, ..., beta-1. */
static float bm_f32(const float *l, int beta, unsigned a) {
  float acc = (a & 1u) ? -l[0] : l[0];
  for (int b = 1; b < beta; ++b) acc = acc + (((a >> b) & 1u) ? -l[b] : l[b]);
  return acc;
}
static double bm_f64(const double *l, int beta, unsigned a) {
  double acc = (a & 1u) ? -l[0] : l[0];
  for (int b = 1; b < beta; ++b) acc = acc + (((a >> b) & 1u) ? -l[b] : l[b]);
  return acc;
}
static int64_t bm_i8(const int8_t *l, int beta, unsigned a) {
  int64_t acc = 0;
  for (int b = 0; b < beta; ++b) acc += ((a >> b) & 1u) ? -(int64_t)l[b] : (int64_t)l[b];
  return acc;
}

/* "minus infinity" for the metric of a state that cannot have been reached.
 * The integer path uses INT64_MIN as that value and never adds to it. */
#define I64_NEG_INF INT64_MIN
static float add_f32(float a, float d) { return a + d; }
static double add_f64(double a, double d) { return a + d; }
static int64_t add_i64(int64_t a, int64_t d) { return a == I64_NEG_INF ? a : a + d; }

/*
 * One window of the decoder: the forward procedure (Algorithm 1, eqs. 2-4)
 * over stages [s, e), then the backward procedure (Algorithm 2) from the last
 * stage, writing the decoded bits of stages [emit_lo, emit_hi) only.
 *
 * Initial path metrics: if the window starts where the encoder is known to be
 * in state 0, state 0 gets 0 and every other state minus infinity; otherwise
 * every state gets 0 (no knowledge of the starting state).
 *
 * ACS (eqs. 3-4): m_b = sigma[i_b] + delta(i_b -> j); the survivor is i_1 only
 * if m_1 > m_0 strictly, so ties go to the lower predecessor i_0.  One
 * decision bit per state and stage records which predecessor survived.
 *
 * Traceback start: state 0 if the window ends where the encoder is known to be
 * back in state 0 (terminated stream), else the state with the largest path
 * metric, lowest index on ties.  Each step back emits alpha_in = j >> (k-2)
 * and moves to the surviving predecessor.
 */
#define DEFINE_WINDOW(NAME, T, LT, NEG_INF, ADD, BM)                                          \
  static int NAME(const vref_code *c, const LT *llr, int64_t s, int64_t e, int start_known,   \
                  int end_zero, int64_t emit_lo, int64_t emit_hi, uint8_t *out,              \
                  T *final_metric) {                                                         \
    trellis tr;                                                                              \
    build_trellis(c, &tr);                                                                   \
    const int S = tr.S, kk = c->k, beta = c->beta;                                           \
    const int words = (S + 63) / 64;                                                         \
    const int64_t nst = e - s;                                                               \
    T *pm = (T *)malloc(sizeof(T) * (size_t)S);                                              \
    T *nm = (T *)malloc(sizeof(T) * (size_t)S);                                              \
    uint64_t *dec = (uint64_t *)calloc((size_t)(nst > 0 ? nst : 1) * (size_t)words,          \
                                       sizeof(uint64_t));                                    \
    if (!pm || !nm || !dec) {                                                                \
      free(pm);                                                                              \
      free(nm);                                                                              \
      free(dec);                                                                             \
      return -2;                                                                             \
    }                                                                                        \
    for (int j = 0; j < S; ++j) pm[j] = start_known ? (j == 0 ? (T)0 : NEG_INF) : (T)0;     \
    for (int64_t t = s; t < e; ++t) {                                                        \
      const LT *l = llr + t * beta;                                                          \
      uint64_t *dt = dec + (t - s) * words;                                                  \
      for (int j = 0; j < S; ++j) {                                                          \
        const T m0 = ADD(pm[tr.pred[j][0]], BM(l, beta, tr.aout[j][0]));                     \
        const T m1 = ADD(pm[tr.pred[j][1]], BM(l, beta, tr.aout[j][1]));                     \
        const int d = m1 > m0;                                                               \
        nm[j] = d ? m1 : m0;                                                                 \
        if (d) dt[j >> 6] |= 1ull << (j & 63);                                               \
      }                                                                                      \
      T *tmp = pm;                                                                           \
      pm = nm;                                                                               \
      nm = tmp;                                                                              \
    }                                                                                        \
    int jstar = 0;                                                                           \
    if (!end_zero)                                                                           \
      for (int j = 1; j < S; ++j)                                                            \
        if (pm[j] > pm[jstar]) jstar = j;                                                    \
    if (final_metric) *final_metric = pm[jstar];                                             \
    const int64_t stop = emit_lo > s ? emit_lo : s;                                          \
    for (int64_t t = e - 1; t >= stop; --t) {                                                \
      if (t < emit_hi) out[t - emit_lo] = (uint8_t)(jstar >> (kk - 2));                      \
      const int d = (int)((dec[(t - s) * words + (jstar >> 6)] >> (jstar & 63)) & 1u);       \
      jstar = ((jstar << 1) & (S - 1)) | d;                                                  \
    }                                                                                        \
    free(pm);                                                                                \
    free(nm);                                                                                \
    free(dec);                                                                               \
    return 0;                                                                                \
  }

DEFINE_WINDOW(window_f32, float, float, -INFINITY, add_f32, bm_f32)
DEFINE_WINDOW(window_f64, double, double, -INFINITY, add_f64, bm_f64)
DEFINE_WINDOW(window_i8, int64_t, int8_t, I64_NEG_INF, add_i64, bm_i8)

int vref_window_f64(const vref_code *code, const double *llr, int64_t s, int64_t e,
                    int32_t start_known, int32_t end_zero, int64_t emit_lo,
                    int64_t emit_hi, uint8_t *out, double *final_metric) {
  if (!code_ok(code) || !llr || s < 0 || e < s || emit_lo < s || emit_hi > e ||
      (emit_hi > emit_lo && !out))
    return -1;
  return window_f64(code, llr, s, e, start_known, end_zero, emit_lo, emit_hi, out,
                    final_metric);
}

/* Full frame: one window over every stage, all n bits emitted. */
#define DEFINE_FULL(NAME, WINDOW, T, LT)                                                     \
  int NAME(const vref_code *code, const LT *llr, int64_t n, int32_t terminated,            \
           uint8_t *out, T *final_metric) {                                                 \
    if (!code_ok(code) || n <= 0 || !llr || !out) return -1;                                \
    const int64_t N = n + (terminated ? code->k - 1 : 0);                                   \
    return WINDOW(code, llr, 0, N, 1, terminated != 0, 0, n, out, final_metric);            \
  }

DEFINE_FULL(vref_decode_full_f32, window_f32, float, float)
DEFINE_FULL(vref_decode_full_f64, window_f64, double, double)
DEFINE_FULL(vref_decode_full_i8, window_i8, int64_t, int8_t)

/* 16-bit modulo metrics (see vref.h).  wrap16 reduces an integer modulo 2^16
 * into [-2^15, 2^15); a is "greater" than b when the wrapped difference a - b
 * is positive.  The forward and backward procedures are those of the window
 * above (Algorithms 1 and 2, ties to the lower predecessor, argmax with the
 * lowest index on ties), with these two operations in place of + and >. */
static int16_t wrap16(int64_t x) {
  const int64_t r = x & 0xffff;
  return (int16_t)(r >= 0x8000 ? r - 0x10000 : r);
}
static int gt16(int16_t a, int16_t b) { return wrap16((int64_t)a - (int64_t)b) > 0; }

int vref_decode_full_i16mod(const vref_code *code, const int8_t *llr, int64_t n,
                            int32_t terminated, uint8_t *out, int16_t *final_metric) {
  if (!code_ok(code) || n <= 0 || !llr || !out) return -1;
  trellis tr;
  build_trellis(code, &tr);
  const int S = tr.S, kk = code->k, beta = code->beta;
  const int words = (S + 63) / 64;
  const int64_t N = n + (terminated ? kk - 1 : 0);
  int16_t pm[VREF_MAX_S], nm[VREF_MAX_S];
  uint64_t *dec = (uint64_t *)calloc((size_t)N * (size_t)words, sizeof(uint64_t));
  if (!dec) return -2;
  for (int j = 0; j < S; ++j) pm[j] = j == 0 ? 0 : wrap16(-(1 << 14));
  for (int64_t t = 0; t < N; ++t) {
    const int8_t *l = llr + t * beta;
    uint64_t *dt = dec + t * words;
    for (int j = 0; j < S; ++j) {
      const int16_t m0 = wrap16((int64_t)pm[tr.pred[j][0]] + bm_i8(l, beta, tr.aout[j][0]));
      const int16_t m1 = wrap16((int64_t)pm[tr.pred[j][1]] + bm_i8(l, beta, tr.aout[j][1]));
      const int d = gt16(m1, m0);
      nm[j] = d ? m1 : m0;
      if (d) dt[j >> 6] |= 1ull << (j & 63);
    }
    memcpy(pm, nm, sizeof(int16_t) * (size_t)S);
  }
  int jstar = 0;
  if (!terminated)
    for (int j = 1; j < S; ++j)
      if (gt16(pm[j], pm[jstar])) jstar = j;
  if (final_metric) *final_metric = pm[jstar];
  for (int64_t t = N - 1; t >= 0; --t) {
    if (t < n) out[t] = (uint8_t)(jstar >> (kk - 2));
    const int d = (int)((dec[t * words + (jstar >> 6)] >> (jstar & 63)) & 1u);
    jstar = ((jstar << 1) & (S - 1)) | d;
  }
  free(dec);
  return 0;
}

/* Sec. III: frames of L output bits, each decoded from its own window that
 * adds v1 stages of history on the left and v2 stages on the right, clipped
 * to the stream.  A window that starts at stage 0 knows the encoder state;
 * a window that ends at the last stage of a terminated stream knows it too. */
#define DEFINE_BLOCKED(NAME, WINDOW, LT)                                                     \
  int NAME(const vref_code *code, const LT *llr, int64_t n, int32_t terminated, int64_t L, \
           int64_t v1, int64_t v2, uint8_t *out, int32_t nthreads) {                        \
    if (!code_ok(code) || n <= 0 || !llr || !out || L <= 0 || v1 < 0 || v2 < 0) return -1;  \
    const int64_t N = n + (terminated ? code->k - 1 : 0);                                   \
    const int64_t nblocks = (n + L - 1) / L;                                                \
    int err = 0;                                                                            \
    if (nthreads < 1) nthreads = 1;                                                         \
    _Pragma("omp parallel for num_threads(nthreads) schedule(dynamic, 8) reduction(|:err)") \
    for (int64_t b = 0; b < nblocks; ++b) {                                                 \
      const int64_t cs = b * L;                                                             \
      const int64_t ce = (cs + L < n) ? cs + L : n;                                         \
      const int64_t s = (cs - v1 > 0) ? cs - v1 : 0;                                        \
      const int64_t e = (ce + v2 < N) ? ce + v2 : N;                                        \
      err |= WINDOW(code, llr, s, e, s == 0, terminated && e == N, cs, ce, out + cs, NULL); \
    }                                                                                       \
    return err ? -2 : 0;                                                                    \
  }

DEFINE_BLOCKED(vref_decode_blocked_f32, window_f32, float)
DEFINE_BLOCKED(vref_decode_blocked_f64, window_f64, double)
DEFINE_BLOCKED(vref_decode_blocked_i8, window_i8, int8_t)

/* SplitMix64 (see vref.h): the sequential generator adds the golden-ratio
 * increment to its state and returns the mixed state, so output i is the mix
 * of seed + (i + 1) * increment. */
uint64_t vref_splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Sec. IV-D, first parallel traceback, as vref.h states it.  The forward
 * procedure is DEFINE_WINDOW's (Algorithm 1 over [s, e)); after each stage
 * x_c - 1 at which an inner chain (x_c < e) starts, the metrics are kept
 * (the paper's second start-state solution keeps only their best state; the
 * whole vector is kept here and reduced when the chain starts).  Then every
 * subframe runs Algorithm 2 from its own start, emitting only its own bits. */
#define DEFINE_WINDOW_PT(NAME, T, LT, NEG_INF, ADD, BM)                                        \
  static int NAME(const vref_code *c, const LT *llr, int64_t s, int64_t e, int start_known,     \
                  int end_zero, int64_t cs, int64_t ce, int64_t f0, int64_t w, int start_rule,  \
                  uint64_t seed, int64_t block, uint8_t *out) {                                 \
    trellis tr;                                                                                \
    build_trellis(c, &tr);                                                                     \
    const int S = tr.S, kk = c->k, beta = c->beta;                                             \
    const int words = (S + 63) / 64;                                                           \
    const int64_t nst = e - s;                                                                 \
    const int64_t C = (ce - cs + f0 - 1) / f0;                                                 \
    int64_t *x = (int64_t *)malloc(sizeof(int64_t) * (size_t)C);                               \
    T *pm = (T *)malloc(sizeof(T) * (size_t)S);                                                \
    T *nm = (T *)malloc(sizeof(T) * (size_t)S);                                                \
    T *snap = (T *)malloc(sizeof(T) * (size_t)S * (size_t)C);                                  \
    uint64_t *dec = (uint64_t *)calloc((size_t)(nst > 0 ? nst : 1) * (size_t)words,            \
                                       sizeof(uint64_t));                                      \
    if (!x || !pm || !nm || !snap || !dec) {                                                   \
      free(x);                                                                                 \
      free(pm);                                                                                \
      free(nm);                                                                                \
      free(snap);                                                                              \
      free(dec);                                                                               \
      return -2;                                                                               \
    }                                                                                          \
    for (int64_t ch = 0; ch < C; ++ch) {                                                       \
      const int64_t b_end = (cs + (ch + 1) * f0 < ce) ? cs + (ch + 1) * f0 : ce;               \
      x[ch] = (ch == C - 1 || b_end + w >= e) ? e : b_end + w;                                 \
    }                                                                                          \
    for (int j = 0; j < S; ++j) pm[j] = start_known ? (j == 0 ? (T)0 : NEG_INF) : (T)0;       \
    for (int64_t t = s; t < e; ++t) {                                                          \
      const LT *l = llr + t * beta;                                                            \
      uint64_t *dt = dec + (t - s) * words;                                                    \
      for (int j = 0; j < S; ++j) {                                                            \
        const T m0 = ADD(pm[tr.pred[j][0]], BM(l, beta, tr.aout[j][0]));                       \
        const T m1 = ADD(pm[tr.pred[j][1]], BM(l, beta, tr.aout[j][1]));                       \
        const int d = m1 > m0;                                                                 \
        nm[j] = d ? m1 : m0;                                                                   \
        if (d) dt[j >> 6] |= 1ull << (j & 63);                                                 \
      }                                                                                        \
      T *tmp = pm;                                                                             \
      pm = nm;                                                                                 \
      nm = tmp;                                                                                \
      /* the metrics after stage t, for every inner chain that starts there */                \
      for (int64_t ch = 0; ch < C; ++ch)                                                       \
        if (x[ch] < e && x[ch] - 1 == t)                                                       \
          for (int j = 0; j < S; ++j) snap[ch * S + j] = pm[j];                                \
    }                                                                                          \
    for (int64_t ch = 0; ch < C; ++ch) {                                                       \
      const int64_t a_lo = cs + ch * f0;                                                       \
      const int64_t b_end = (a_lo + f0 < ce) ? a_lo + f0 : ce;                                 \
      int j = 0;                                                                               \
      if (x[ch] == e) {                                                                        \
        if (!end_zero)                                                                         \
          for (int i = 1; i < S; ++i)                                                          \
            if (pm[i] > pm[j]) j = i;                                                          \
      } else if (start_rule == VREF_PT_RANDOM) {                                               \
        j = (int)(vref_splitmix64(seed, ((uint64_t)block << 32) | (uint64_t)ch) >> (65 - kk)); \
      } else {                                                                                 \
        const T *mt = snap + ch * S;                                                           \
        for (int i = 1; i < S; ++i)                                                            \
          if (mt[i] > mt[j]) j = i;                                                            \
      }                                                                                        \
      for (int64_t t = x[ch] - 1; t >= a_lo; --t) {                                            \
        if (t < b_end) out[t - cs] = (uint8_t)(j >> (kk - 2));                                 \
        const int d = (int)((dec[(t - s) * words + (j >> 6)] >> (j & 63)) & 1u);               \
        j = ((j << 1) & (S - 1)) | d;                                                          \
      }                                                                                        \
    }                                                                                          \
    free(x);                                                                                   \
    free(pm);                                                                                  \
    free(nm);                                                                                  \
    free(snap);                                                                                \
    free(dec);                                                                                 \
    return 0;                                                                                  \
  }

DEFINE_WINDOW_PT(window_pt_f32, float, float, -INFINITY, add_f32, bm_f32)
DEFINE_WINDOW_PT(window_pt_i8, int64_t, int8_t, I64_NEG_INF, add_i64, bm_i8)

#define DEFINE_BLOCKED_PT(NAME, WINDOW, LT)                                                     \
  int NAME(const vref_code *code, const LT *llr, int64_t n, int32_t terminated, int64_t L,    \
           int64_t v1, int64_t v2, int64_t f0, int64_t w, int32_t start_rule, uint64_t seed,   \
           uint8_t *out, int32_t nthreads) {                                                   \
    if (!code_ok(code) || n <= 0 || !llr || !out || L <= 0 || v1 < 0 || v2 < 0 || f0 < 1 ||   \
        w < 0 || (start_rule != VREF_PT_STORED && start_rule != VREF_PT_RANDOM) ||             \
        (L + f0 - 1) / f0 > ((int64_t)1 << 32))                                                \
      return -1;                                                                               \
    const int64_t N = n + (terminated ? code->k - 1 : 0);                                      \
    const int64_t nblocks = (n + L - 1) / L;                                                   \
    int err = 0;                                                                               \
    if (nthreads < 1) nthreads = 1;                                                            \
    _Pragma("omp parallel for num_threads(nthreads) schedule(dynamic, 8) reduction(|:err)")    \
    for (int64_t b = 0; b < nblocks; ++b) {                                                    \
      const int64_t cs = b * L;                                                                \
      const int64_t ce = (cs + L < n) ? cs + L : n;                                            \
      const int64_t s = (cs - v1 > 0) ? cs - v1 : 0;                                           \
      const int64_t e = (ce + v2 < N) ? ce + v2 : N;                                           \
      err |= WINDOW(code, llr, s, e, s == 0, terminated && e == N, cs, ce, f0, w, start_rule,  \
                    seed, b, out + cs);                                                        \
    }                                                                                          \
    return err ? -2 : 0;                                                                       \
  }

DEFINE_BLOCKED_PT(vref_decode_blocked_pt_f32, window_pt_f32, float)
DEFINE_BLOCKED_PT(vref_decode_blocked_pt_i8, window_pt_i8, int8_t)

int vref_quantize_i8(const float *llr, int64_t count, float scale, int8_t *q) {
  if (count < 0 || (count > 0 && (!llr || !q))) return -1;
  for (int64_t i = 0; i < count; ++i) {
    const float x = nearbyintf(llr[i] * scale); /* default rounding: half to even */
    q[i] = (int8_t)(x > 127.0f ? 127 : (x < -127.0f ? -127 : (int)x));
  }
  return 0;
}

/* De-puncturing (Sec. IV-E): walk the output stream stage by stage and slot
 * by slot; a slot the pattern keeps takes the next received value, a
 * punctured slot gets a zero LLR (no information). */
#define DEFINE_DEPUNCTURE(NAME, T)                                                  \
  int NAME(const T *in, int64_t in_count, const uint8_t *mask, int32_t period,     \
           int32_t beta, int64_t stages, T *out) {                                 \
    if (period < 1 || beta < 1 || stages < 0 || !mask || (stages > 0 && !out))      \
      return -1;                                                                    \
    int64_t used = 0;                                                               \
    for (int64_t t = 0; t < stages; ++t) {                                          \
      for (int32_t b = 0; b < beta; ++b) {                                          \
        if (mask[(t % period) * beta + b]) {                                        \
          if (used >= in_count) return -1;                                          \
          out[t * beta + b] = in[used++];                                           \
        } else {                                                                    \
          out[t * beta + b] = (T)0;                                                 \
        }                                                                           \
      }                                                                             \
    }                                                                               \
    return used == in_count ? 0 : -1;                                               \
  }
DEFINE_DEPUNCTURE(vref_depuncture_f32, float)
DEFINE_DEPUNCTURE(vref_depuncture_i8, int8_t)

/* Exhaustive search (see vref.h).  x[] holds the k-1 prehistory inputs
 * followed by the window inputs, oldest first; the register of window stage
 * t' is built from x[t'] .. x[t'+k-1] with the newest input in bit k-1. */
int vref_bruteforce_window(const vref_code *code, const double *llr, int64_t s,
                           int64_t e, int32_t start_known, int32_t end_zero,
                           uint8_t *out, double *best_metric) {
  return vref_bruteforce_window_to(code, llr, s, e, start_known, end_zero ? 0 : -1, out,
                                   best_metric);
}

int vref_bruteforce_window_to(const vref_code *code, const double *llr, int64_t s,
                              int64_t e, int32_t start_known, int32_t end_state,
                              uint8_t *out, double *best_metric) {
  if (!code_ok(code) || !llr || !out || s < 0 || e <= s || end_state < -1 ||
      end_state >= (1 << (code->k - 1)))
    return -1;
  const int km1 = code->k - 1;
  const int64_t w = e - s;
  const int64_t nbits = km1 + w;
  if (nbits > 26) return -1;
  uint8_t x[26 + VREF_MAX_K];
  double best = -INFINITY;
  uint64_t bestkey = 0;
  int found = 0;
  for (uint64_t key = 0; key < (1ull << nbits); ++key) {
    /* bit p of key is x[p]: the latest input is the most significant bit */
    for (int64_t p = 0; p < nbits; ++p) x[p] = (uint8_t)((key >> p) & 1u);
    int ok = 1;
    if (start_known)
      for (int p = 0; p < km1; ++p) ok &= (x[p] == 0);
    if (end_state >= 0) {
      /* the state after the last stage: its last k-1 inputs, newest in the MSB */
      int st = 0;
      for (int m = 0; m < km1; ++m) st |= (int)x[nbits - 1 - m] << (km1 - 1 - m);
      ok &= (st == end_state);
    }
    if (!ok) continue;
    double metric = 0.0;
    for (int64_t tp = 0; tp < w; ++tp) {
      uint32_t reg = 0;
      for (int m = 0; m < code->k; ++m) reg |= (uint32_t)x[tp + km1 - m] << (code->k - 1 - m);
      metric = metric + bm_f64(llr + (s + tp) * code->beta, code->beta, register_output(code, reg));
    }
    if (!found || metric > best || (metric == best && key < bestkey)) {
      best = metric;
      bestkey = key;
      found = 1;
    }
  }
  for (int64_t tp = 0; tp < w; ++tp) out[tp] = (uint8_t)((bestkey >> (km1 + tp)) & 1u);
  if (best_metric) *best_metric = best;
  return 0;
}
