/*
 * vref.h -- plain CPU oracle for soft-decision Viterbi decoding of (beta,1,k)
 * convolutional codes, full-frame and blocked-with-overlap.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference that
 * the GPU decoder is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product decoder
 * never calls it and shares no code, header, table or helper with it.
 *
 * Source: Mohammadidoost & Hashemi, "High-Throughput and Memory-Efficient
 * Parallel Viterbi Decoder for Convolutional Codes on GPU" (arXiv 2011.09337).
 *   encoder ............ Sec. II-A, eq. (1)
 *   trellis / FSM ...... Sec. II-A (states are the k-1 previous inputs)
 *   branch metric ...... Sec. II-B, eq. (2)
 *   path metric, ACS ... Sec. II-B, eqs. (3)-(4), Algorithm 1 (forward)
 *   traceback .......... Sec. II-B, Algorithm 2 (backward)
 *   overlapping frames . Sec. III (frames of f bits, left overlap v1, right v2)
 *
 * Conventions (the paper leaves these open; these are the readings taken):
 *   - gen[b] is a k-bit generator; its bit k-1 taps the current input in_t
 *     and bit 0 taps in_{t-k+1} (eq. 1 multiplies in_t by g_{k-1}).
 *   - output bit b of a stage is produced by gen[b], in the order listed.
 *   - LLRs are time-major: llr[t*beta + b]; positive means "bit 0 likely".
 *   - a state holds the k-1 previous inputs with the newest in the MSB.
 *   - ACS ties go to the lower predecessor index; the final argmax picks the
 *     lowest state index on ties.
 *   - decoded bits are returned UNPACKED, one byte (0 or 1) per bit.
 *
 * Every function returns 0 on success and a negative value on invalid input.
 */
#ifndef VREF_H
#define VREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t k;        /* constraint length, 3..9            */
  int32_t beta;     /* coded bits per input bit, 2..4     */
  uint32_t gen[4];  /* generators, 0 < gen[b] < 2^k       */
} vref_code;

/* eq. (1): encode n bits; if terminated, k-1 zero tail inputs are appended.
 * coded receives N*beta bytes (0/1), N = n + (terminated ? k-1 : 0). */
int vref_encode(const vref_code *code, const uint8_t *bits, int64_t n,
                int32_t terminated, uint8_t *coded);

/* Full-frame maximum-likelihood decoding (Algorithms 1 and 2 over the whole
 * stream).  llr holds N*beta values.  out receives n bytes.  If
 * final_metric is not NULL it receives the path metric of the traced path. */
int vref_decode_full_f32(const vref_code *code, const float *llr, int64_t n,
                         int32_t terminated, uint8_t *out, float *final_metric);
int vref_decode_full_f64(const vref_code *code, const double *llr, int64_t n,
                         int32_t terminated, uint8_t *out, double *final_metric);
/* Integer LLRs (e.g. int8-quantised), exact int64 path metrics. */
int vref_decode_full_i8(const vref_code *code, const int8_t *llr, int64_t n,
                        int32_t terminated, uint8_t *out, int64_t *final_metric);
/* The same integer decode with 16-bit path metrics kept modulo 2^16, as a
 * fixed-width integer datapath would hold them (the paper does not discuss
 * metric overflow): every sum wraps, and two metrics are compared by the sign
 * of their wrapped difference.  States other than 0 start at -2^14 instead of
 * minus infinity.  Its decisions equal the exact ones while any two compared
 * metrics differ by less than 2^15; it exists to check that reading against
 * vref_decode_full_i8.  final_metric receives the traced path's metric modulo
 * 2^16 (as a signed 16-bit value). */
int vref_decode_full_i16mod(const vref_code *code, const int8_t *llr, int64_t n,
                            int32_t terminated, uint8_t *out, int16_t *final_metric);

/* Blocked decoding with overlap (Sec. III): the n output bits are split into
 * cores of L bits; block b covers trellis stages
 *   [max(0, bL - v1), min(N, min((b+1)L, n) + v2))
 * and emits only its core bits.  nthreads > 1 decodes blocks in parallel
 * (OpenMP); results do not depend on nthreads. */
int vref_decode_blocked_f32(const vref_code *code, const float *llr, int64_t n,
                            int32_t terminated, int64_t L, int64_t v1, int64_t v2,
                            uint8_t *out, int32_t nthreads);
int vref_decode_blocked_f64(const vref_code *code, const double *llr, int64_t n,
                            int32_t terminated, int64_t L, int64_t v1, int64_t v2,
                            uint8_t *out, int32_t nthreads);
int vref_decode_blocked_i8(const vref_code *code, const int8_t *llr, int64_t n,
                           int32_t terminated, int64_t L, int64_t v1, int64_t v2,
                           uint8_t *out, int32_t nthreads);

/* One window of the blocked decoder, exposed for tests: run the forward
 * procedure over stages [s, e) from either the known state 0 (start_known=1)
 * or an unknown state (all path metrics 0), start the traceback from state 0
 * (end_zero=1) or from the best state, and write bits for stages
 * [emit_lo, emit_hi) to out[t - emit_lo]. */
int vref_window_f64(const vref_code *code, const double *llr, int64_t s, int64_t e,
                    int32_t start_known, int32_t end_zero, int64_t emit_lo,
                    int64_t emit_hi, uint8_t *out, double *final_metric);

/* Saturating int8 quantiser: q = clamp(round_half_even(llr * scale), -127, 127). */
int vref_quantize_i8(const float *llr, int64_t count, float scale, int8_t *q);

/* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) used as a counter-based generator: output i of
 * the sequential generator seeded with `seed` (i = 0, 1, ...), that is
 * mix(seed + (i + 1) * 0x9E3779B97F4A7C15) with the published mix function. */
uint64_t vref_splitmix64(uint64_t seed, uint64_t i);

/* Start rules of the parallel traceback's inner chains (Sec. IV-D). */
enum { VREF_PT_STORED = 0, VREF_PT_RANDOM = 1 };

/* Blocked decoding with the first parallel traceback of Sec. IV-D, in the
 * paper's geometry.  Block geometry as vref_decode_blocked_*: block b has
 * stages [s, e) and core [cs, ce).  The core is cut into C = ceil((ce-cs)/f0)
 * subframes of f0 bits, subframe c = [a_c, b_c) = [cs + c*f0, min(cs +
 * (c+1)*f0, ce)).  Its traceback starts after stage x_c - 1, runs down to
 * its first bit and keeps only its own bits, where
 *   x_c = e                  for the last subframe (the block's own right
 *                            overlap above it),
 *   x_c = min(e, b_c + w)    for the others (w stages of overlap into the
 *                            right neighbour).
 * Start state: at x_c = e the block's own (state 0 at the end of a
 * terminated stream, else the best final state, lowest index on ties);
 * otherwise, with start_rule VREF_PT_STORED the state with the best metric
 * after stage x_c - 1 (lowest index on ties), with VREF_PT_RANDOM the state
 * given by the top k-1 bits of vref_splitmix64(seed, (b << 32) | c).
 * f0 >= L with w >= v2 gives vref_decode_blocked_*.  Requires f0 >= 1,
 * w >= 0 and at most 2^32 subframes per block. */
int vref_decode_blocked_pt_f32(const vref_code *code, const float *llr, int64_t n, int32_t terminated,
                               int64_t L, int64_t v1, int64_t v2, int64_t f0, int64_t w, int32_t start_rule,
                               uint64_t seed, uint8_t *out, int32_t nthreads);
int vref_decode_blocked_pt_i8(const vref_code *code, const int8_t *llr, int64_t n, int32_t terminated,
                              int64_t L, int64_t v1, int64_t v2, int64_t f0, int64_t w, int32_t start_rule,
                              uint64_t seed, uint8_t *out, int32_t nthreads);

/* De-puncturing (Sec. IV-E): expand a punctured stream into `stages` stages
 * of beta LLRs.  mask[p*beta + b] != 0 when output b of stage t with
 * t mod period = p was transmitted; transmitted values are taken from `in`
 * in stream order, punctured slots get 0.  Returns 0, or -1 if in_count is
 * not exactly the number of transmitted slots. */
int vref_depuncture_f32(const float *in, int64_t in_count, const uint8_t *mask, int32_t period, int32_t beta,
                        int64_t stages, float *out);
int vref_depuncture_i8(const int8_t *in, int64_t in_count, const uint8_t *mask, int32_t period, int32_t beta,
                       int64_t stages, int8_t *out);

/* Exhaustive search over every input sequence of a window, for small windows
 * only (prehistory + window inputs <= 24 bits).  The window covers stages
 * [s, e) of an LLR stream; the k-1 inputs before stage s are free unless
 * start_known (then 0); if end_zero the inputs of the last k-1 stages are 0.
 * Among the sequences with the largest metric (eq. 2 summed over the window,
 * in stage order, in double precision) it returns the one that is smallest
 * when read as an integer whose most significant bit is the latest input.
 * out receives the inputs of stages [s, e); best_metric the metric. */
int vref_bruteforce_window(const vref_code *code, const double *llr, int64_t s,
                           int64_t e, int32_t start_known, int32_t end_zero,
                           uint8_t *out, double *best_metric);
/* The same search with the state after the window's last stage fixed:
 * end_state in [0, 2^(k-1)) keeps only the sequences whose last k-1 inputs
 * form that state (newest input in the MSB); end_state = -1 leaves it free.
 * end_state = 0 is end_zero = 1 above. */
int vref_bruteforce_window_to(const vref_code *code, const double *llr, int64_t s,
                              int64_t e, int32_t start_known, int32_t end_state,
                              uint8_t *out, double *best_metric);

#ifdef __cplusplus
}
#endif
#endif
