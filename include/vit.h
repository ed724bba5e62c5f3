/*
 * vit.h -- C ABI of the MI355X (gfx950) soft-decision Viterbi decoder.
 *
 * The library decodes a (beta,1,k) convolutional code from a stream of soft
 * inputs (log-likelihood ratios), following Mohammadidoost & Hashemi,
 * "High-Throughput and Memory-Efficient Parallel Viterbi Decoder for
 * Convolutional Codes on GPU" (arXiv 2011.09337):
 *   - branch metric: Sec. II-B, eq. (2);
 *   - add-compare-select and survivor selection: Sec. II-B, eqs. (3)-(4),
 *     forward procedure of Algorithm 1;
 *   - traceback and decoding: Algorithm 2;
 *   - overlapping frames (f = L decoded bits per block, left overlap v1,
 *     right overlap v2): Sec. III; forward and backward in one kernel with
 *     survivors kept on chip: Sec. IV-A.
 *
 * Conventions shared by every entry point:
 *   - gen[b] is a k-bit generator; bit k-1 taps the current input in_t and
 *     bit 0 taps in_{t-k+1} (eq. 1).  Output bit b of a stage is produced by
 *     gen[b], b = 0..beta-1, and pairs with LLR slot b.
 *   - LLRs are time-major and interleaved: llr[t*beta + b].  A positive LLR
 *     means "coded bit 0 is more likely" (Sec. II-C).  For a terminated stream
 *     the k-1 tail stages follow the n information stages, so the stream holds
 *     N = n + k - 1 stages; an open stream holds N = n stages.
 *   - Decoded bits are packed LSB first: bit t goes to byte t >> 3, bit
 *     position t & 7.  out_bits must hold ceil(n/8) bytes; pad bits are 0.
 *   - Ties: an add-compare-select tie keeps the lower predecessor index; the
 *     traceback starts from the lowest-index state among those with the
 *     largest path metric (VIT_TIE_LOWER_PRED, the only rule).
 *   - Blocked geometry (Sec. III): block b decodes core bits
 *     [bL, min((b+1)L, n)) from trellis stages
 *     [max(0, bL - v1), min(N, min((b+1)L, n) + v2)).  A block that starts at
 *     stage 0 starts from state 0; any other block starts with every path
 *     metric 0.  A block that ends at stage N of a terminated stream traces
 *     back from state 0; any other block from the best state.
 *   - L = 0 selects full-frame decoding: one block holding every stage.
 *
 * Pointers to LLRs and to decoded bits are DEVICE memory owned by the caller;
 * the library allocates no device memory on the decode path (except one flag
 * word per device for the optional finiteness pre-pass, on its first use).
 *
 * Return values: VIT_OK (0) or a negative status.  Argument errors are found
 * on the host before any device work (and need no GPU).  vit_last_error()
 * returns a thread-local message describing the last failure.
 */
#ifndef VIT_H
#define VIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VIT_ABI_VERSION 3

enum {
  VIT_OK = 0,
  VIT_EINVAL = -1,        /* an argument is invalid                            */
  VIT_EUNSUPPORTED = -2,  /* valid, but outside what the GPU kernel supports   */
  VIT_ENOMEM = -3,        /* host allocation failed                            */
  VIT_EDEVICE = -4,       /* a HIP runtime call or kernel launch failed        */
  VIT_EBUSY = -5,
  VIT_ETIMEDOUT = -6      /* a serving request waited longer than max_wait_ms  */
};

enum { VIT_TIE_LOWER_PRED = 0 };
/* Soft-input types.  VIT_LLR_HARD: hard decisions, one byte per coded bit,
 * 0 for coded bit 0 and any other value for coded bit 1, decoded as integer
 * LLRs +1 / -1 (the hard-decision mode of Sec. I and II-C). */
enum { VIT_LLR_F32 = 0, VIT_LLR_I8 = 1, VIT_LLR_HARD = 2 };
/* Start rules of the parallel traceback's inner chains (vit_opts). */
enum { VIT_SUBFRAME_STORED = 0, VIT_SUBFRAME_RANDOM = 1 };

/* A (beta,1,k) code: 3 <= k <= 9, 2 <= beta <= 4, 0 < gen[b] < 2^k. */
typedef struct {
  int32_t k;
  int32_t beta;
  uint32_t gen[4];
} vit_code;

/* Options of vit_decode_ex.  Fill with vit_opts_default() and set size. */
typedef struct {
  uint32_t size;         /* sizeof(vit_opts)                                     */
  int32_t llr_type;      /* VIT_LLR_F32 (float), VIT_LLR_I8 (int8) or VIT_LLR_HARD */
  int32_t terminated;    /* 1: the stream carries k-1 tail stages (default 1)    */
  int32_t v1;            /* left overlap; -1 = floor(v/2) (default -1)           */
  int32_t check_finite;  /* 1: scan FP32 LLRs first and return VIT_EINVAL if any is
                          * NaN or infinite (the call then waits for the scan on
                          * `stream`); 0 (default): LLRs must be finite, unchecked */
  int32_t reserved;
  void *stream;          /* hipStream_t to launch on; NULL = default stream      */
  /* Parallel traceback (Sec. IV-D, the paper's first scheme).  0 (default):
   * each block is traced back once from its end.  f0 = subframe_bits > 0:
   * the block's core [cs, ce) is cut into C = ceil((ce - cs) / f0) subframes
   * of f0 bits, subframe c = [cs + c*f0, min(cs + (c+1)*f0, ce)), and each
   * is traced back by its own chain (one lane of the block's wave) that
   * emits only its own bits.  Chain c starts after stage x_c - 1 with
   *   x_c = e (the block end) for the last subframe and wherever
   *         end_c + w >= e, else x_c = end_c + w (end_c = cs + (c+1)*f0,
   *         w = subframe_overlap stages of inner overlap).
   * A chain with x_c = e starts from the block's own traceback state (state
   * 0 at the end of a terminated stream, else the best final state).  Any
   * other starts, with subframe_start = VIT_SUBFRAME_STORED, from the state
   * with the best path metric after stage x_c - 1 (lowest index on ties;
   * the forward pass keeps it), or with VIT_SUBFRAME_RANDOM from the state
   * given by the top k-1 bits of output i = (b << 32) | c of the SplitMix64
   * generator seeded with subframe_seed (b = block index; see
   * vref_splitmix64 in the oracle for the definition).  f0 >= L gives the
   * one-trace decode.  Requires at most 64 subframes per block, FP32 LLRs or
   * 32-bit integer metrics (VIT_EUNSUPPORTED otherwise). */
  int32_t subframe_bits;
  int32_t subframe_overlap; /* w >= 0, in stages (default 0)                   */
  int32_t subframe_start;   /* VIT_SUBFRAME_STORED (default) or _RANDOM        */
  /* Path metrics of the integer inputs (VIT_LLR_I8, VIT_LLR_HARD); both give
   * the decisions of exact integer arithmetic.  16: 16-bit metrics kept
   * modulo 2^16, two blocks per wave, compared by the sign of their wrapped
   * difference (eq. 3 in 16 bits; exact while compared metrics differ by less
   * than 2^15, which the spread bound (k-1)*2*128*beta + 2^14 guarantees);
   * blocks up to the LDS limit of two blocks' survivors per wave.  32: the
   * integers held exactly in fp32 metrics, one block per wave; blocks up to
   * 2^24 / (128 beta) stages.  0 (default): 32 where the blocks fit, else 16
   * (32 measured faster on gfx950 at every shape but K=7 r1/2 at L = 256).
   * Subframe traceback runs with 32 only.  Ignored for FP32 LLRs. */
  int32_t metric_bits;
  uint64_t subframe_seed;   /* seed of VIT_SUBFRAME_RANDOM (default 0)         */
} vit_opts;

/* Decode n information bits from FP32 LLRs with blocks of L core bits and
 * total overlap v (v1 = floor(v/2) on the left, v2 = v - v1 on the right), on
 * a terminated stream.  L must be 0 (full frame) or a positive multiple of 8.
 * Launches on the default stream and waits for completion.
 * Errors: VIT_EINVAL for a bad code, NULL pointer, n <= 0, L < 0, v < 0 or an
 * unknown tie rule; VIT_EUNSUPPORTED if L is not a multiple of 8 or one block's
 * survivor storage exceeds the device's per-workgroup LDS; VIT_EDEVICE if a
 * HIP call fails (including errors left by earlier work on the stream). */
int vit_decode(const vit_code *code, const float *llr, int64_t n, int32_t L, int32_t v,
               int32_t tie_rule, uint8_t *out_bits);

/* As vit_decode, with options, asynchronous on opts->stream: returns once the
 * work is queued; kernel faults surface at the caller's next synchronisation.
 * With llr_type = VIT_LLR_I8 the LLRs are int8 values (any range, -128
 * allowed) and the decoder computes exactly in integers: decisions are those
 * of exact arithmetic on the int8 values.  With VIT_LLR_HARD the input is one
 * byte per coded bit (0 / nonzero) decoded as the integer LLRs +1 / -1.
 * opts may be NULL (defaults). */
int vit_decode_ex(const vit_code *code, const void *llr, int64_t n, int32_t L, int32_t v,
                  int32_t tie_rule, uint8_t *out_bits, const vit_opts *opts);

/* int8 quantisation of soft inputs (the input stage of the int8 decode path;
 * the paper does not fix one): q[i] = clamp(round_half_even(llr[i] * scale),
 * -127, 127), the product rounded once to fp32.  -128 is never produced.
 * llr (count floats) and q (count bytes) are device memory; asynchronous on
 * `stream` (hipStream_t, NULL = default).  LLRs must be finite.
 * Errors: VIT_EINVAL for count < 0, NULL buffers, or a scale that is not
 * positive and finite; VIT_EDEVICE for launch failures. */
int vit_quantize_i8(const float *llr, int64_t count, float scale, int8_t *q, void *stream);

/* De-puncturing (Sec. IV-E): expand a punctured stream of soft inputs into
 * `stages` stages of beta values, with a zero LLR in every punctured slot, for
 * the decoders above.  mask (host, period*beta bytes, period*beta <= 64):
 * mask[p*beta + b] != 0 if output b of a stage t with t mod period = p is
 * transmitted.  received (device) holds the transmitted values in stream
 * order, exactly as many as the pattern keeps in `stages` stages; out
 * (device) receives stages*beta values.  llr_type VIT_LLR_F32 or VIT_LLR_I8.
 * Asynchronous on `stream`.  Errors: VIT_EINVAL for a bad pattern, count or
 * buffer; VIT_EDEVICE for launch failures. */
int vit_depuncture(const void *received, int64_t received_count, int32_t llr_type, const uint8_t *mask,
                   int32_t period, int32_t beta, int64_t stages, void *out, void *stream);

/* Default options: FP32, terminated, v1 = floor(v/2), default stream, one
 * traceback per block. */
vit_opts vit_opts_default(void);

/* Geometry of a blocked decode, computed on the host (no device needed). */
typedef struct {
  int64_t n_stages;        /* N                                              */
  int64_t n_blocks;        /* ceil(n / L)                                    */
  int64_t v1, v2;          /* overlaps actually used                         */
  int64_t stages_total;    /* sum over blocks of trellis stages processed    */
  int64_t max_block_stages;
  int64_t lds_bytes_per_block; /* survivor storage of one block (one wave)   */
} vit_geometry;

/* Fill *geo for the given decode arguments (same validation as vit_decode_ex,
 * with v1 < 0 meaning floor(v/2)). */
int vit_query_geometry(const vit_code *code, int64_t n, int32_t L, int32_t v, int32_t v1,
                       int32_t terminated, vit_geometry *geo);

/* ---------------------------------------------------------------- batches
 * Many independent frames (each its own stream, Sec. III applied per frame),
 * possibly of different codes and lengths, decoded by one graph launch: one
 * persistent kernel per code (in sequence, most work per bit first) walks the
 * frames' blocks in a cost-sorted work list (longest first), wave w of W
 * taking items w, w + W, w + 2W, ...
 * Results are identical, bit for bit, to decoding each frame alone with
 * vit_decode_ex and the same (L, v, v1). */

/* One frame of a batch. */
typedef struct {
  int32_t code_id;     /* index into the codes array of the call                   */
  int32_t terminated;  /* 1: k-1 tail stages follow the n information stages       */
  int64_t n;           /* information bits, > 0                                    */
  int64_t llr_off;     /* element offset of the frame's first LLR in the batch LLRs */
  int64_t out_off;     /* byte offset of the frame's first decoded byte            */
} vit_frame;

/* Block shape for one code of a batch. */
typedef struct {
  int32_t L;                /* core bits per block: a positive multiple of 8     */
  int32_t v;                /* total overlap, >= 0                               */
  int32_t v1;               /* left overlap, -1 = floor(v/2)                     */
  int32_t waves_per_block;  /* waves per workgroup, 1..4                         */
} vit_tuning;

/* A plan owns pinned host staging for work lists, a captured hipGraph that is
 * reused while the buffers and shapes stay the same, and the autotuner's
 * choices.  It never allocates device memory: the caller supplies the
 * workspace.  A plan is not thread-safe, and the batch entry points are to be
 * called from one thread at a time: two threads decoding with two plans at
 * once ended the process once (a host-side crash inside vit_decode_batch
 * whose cause is not known). */
typedef struct vit_plan vit_plan;

int vit_plan_create(vit_plan **plan);
void vit_plan_destroy(vit_plan *plan);

/* Path metrics of the plan's integer decodes, as vit_opts.metric_bits: 0
 * (default), 16 or 32.  VIT_EINVAL for other values. */
int vit_plan_set_metric_bits(vit_plan *plan, int32_t bits);

/* Device workspace bytes that vit_decode_batch needs for these frames.  With
 * tune = NULL the size covers every shape the autotuner may choose. */
int vit_batch_workspace_size(const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes,
                             const vit_tuning *tune, size_t *bytes);

/* Decode a batch.  codes: ncodes (1..8) codes; frames: host array; llr: device
 * buffer of llr_count elements of llr_type (VIT_LLR_F32, VIT_LLR_I8 or
 * VIT_LLR_HARD); out: device buffer of out_bytes
 * bytes (frames' output ranges must not overlap); tune: one vit_tuning per
 * code, or NULL for the plan's autotuned shapes (default L = 256, v = 5k for k <= 7 and 8(k-1) above,
 * 1 wave per workgroup when not tuned); workspace: device memory of at least
 * vit_batch_workspace_size bytes, 256-byte aligned, not used by concurrent
 * calls.  Asynchronous on `stream`; the host staging of the previous use of
 * a staging slot is waited for before it is rewritten.
 * Errors: VIT_EINVAL for bad codes, frames outside the buffers, bad tunings
 * or a small workspace; VIT_EUNSUPPORTED for shapes without a kernel (LDS);
 * VIT_EDEVICE for HIP failures. */
int vit_decode_batch(vit_plan *plan, const vit_code *codes, int32_t ncodes, const vit_frame *frames,
                     int32_t nframes, const void *llr, int64_t llr_count, int32_t llr_type, uint8_t *out,
                     int64_t out_bytes, const vit_tuning *tune, void *workspace, size_t workspace_bytes,
                     void *stream);

/* For callers that cannot allocate: code that must not call hipMalloc or
 * create graphs (work under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The same decode as vit_decode_batch,
 * bit for bit, without a plan or workspace: the work list (header and work
 * items) lives in a fixed device array inside the library of 256 +
 * VIT_STATIC_BATCH_MAX_ITEMS * 40 bytes (10.5 MB), one copy per GPU the
 * library runs on, held until the process ends; the host builds it in fixed
 * host arrays of the same capacity.  The call makes no hipMalloc, hipFree,
 * hipHostMalloc or graph call and no host heap allocation.
 * tune: one vit_tuning per code, or NULL for the default shapes (L = 256,
 * v = 5k for k <= 7 and 8(k-1) above, 1 wave per workgroup; no autotuning).
 * Limits, checked before any device work: at most
 * VIT_STATIC_BATCH_MAX_FRAMES frames, VIT_STATIC_BATCH_MAX_ITEMS blocks and
 * VIT_STATIC_BATCH_MAX_STAGES stages per block (L + v); beyond them the call
 * returns VIT_EUNSUPPORTED with a message naming the limit.
 * Ordering: the work list is copied on `stream` and the call waits for that
 * copy (and so for earlier work on `stream`) before it launches the kernels
 * asynchronously on `stream`.  Every call on one GPU rewrites that GPU's
 * array: calls on one GPU must be ordered (the same stream, or synchronised
 * streams); calls that overlap on one GPU race.  The host side is serialised
 * by a lock.  Errors as vit_decode_batch. */
#define VIT_STATIC_BATCH_MAX_ITEMS 262144
#define VIT_STATIC_BATCH_MAX_FRAMES 65536
#define VIT_STATIC_BATCH_MAX_STAGES 65536
int vit_decode_batch_static(const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes,
                            const void *llr, int64_t llr_count, int32_t llr_type, uint8_t *out, int64_t out_bytes,
                            const vit_tuning *tune, void *stream);

/* One autotuned shape as a plan keeps it: the code, the LLR type and the
 * frame-length bucket it applies to (bucket b: the mean length of the batch's
 * frames of that code lies in [2^b, 2^(b+1)); 0 below 2). */
typedef struct {
  vit_code code;
  int32_t llr_type;
  int32_t length_bucket;
  vit_tuning tuning;
} vit_tuning_entry;

/* The plan's autotuned shapes, so that a caller can keep them (in a file,
 * per GPU model) and hand them to another plan instead of tuning again.
 * get: copies up to `max` entries (entries may be NULL when max = 0);
 * *count receives how many the plan holds.  set: adds or replaces entries
 * with the same (code, llr_type, length_bucket); every entry is validated
 * (code, tuning, llr_type, bucket in [0, 40]) before any is taken, and the
 * first bad one is reported with VIT_EINVAL; VIT_ENOMEM if the plan cannot
 * store them (none is taken then). */
int vit_plan_get_tuning(const vit_plan *plan, vit_tuning_entry *entries, int32_t max, int32_t *count);
int vit_plan_set_tuning(vit_plan *plan, const vit_tuning_entry *entries, int32_t count);

/* Autotune: for each code, decode the batch's frames of that code once with
 * a reference shape whose overlap lies far beyond the trellis's convergence
 * depth (L = 512, v1 = v2 = 128; Sec. III: the right overlap decides how
 * close a block's decisions come to full-frame ML), then with every
 * candidate shape: L in {64, 128, 256, 512, 1024}, v in {5k, 6k, 7k, 8(k-1),
 * 10(k-1)} with v1 = floor(v/2), 1 or 2 waves per workgroup.  A candidate
 * whose decoded bits differ from the reference's in more than the plan's
 * tolerance (vit_plan_set_tune_tolerance; default 8e-4 of the code's bits)
 * is rejected; the fastest of the others (3 timed runs each) is kept in the
 * plan, keyed by (code, llr_type, frame-length bucket).  If none qualifies,
 * the reference shape is kept.  chosen (may be NULL) receives one vit_tuning
 * per code.  Same buffers and errors as vit_decode_batch (plus a host copy
 * of the output buffer per candidate); the output buffer holds the last
 * candidate's result afterwards. */
int vit_plan_autotune(vit_plan *plan, const vit_code *codes, int32_t ncodes, const vit_frame *frames,
                      int32_t nframes, const void *llr, int64_t llr_count, int32_t llr_type, uint8_t *out,
                      int64_t out_bytes, void *workspace, size_t workspace_bytes, void *stream,
                      vit_tuning *chosen);

/* The autotuner's accuracy bound: the largest fraction, in [0, 1], of a
 * code's decoded bits in which an accepted shape may differ from the
 * reference decode.  VIT_EINVAL outside [0, 1] (or NaN). */
int vit_plan_set_tune_tolerance(vit_plan *plan, double max_diff_fraction);

/* ---------------------------------------------------------------- serving
 * A request loop with continuous batching.  Requests are frames whose LLRs
 * sit in a caller-owned pinned host region; an engine thread owned by the
 * server admits queued frames while frame slots and device arena memory
 * allow, and runs iterations of at most max_items blocks (the independent
 * windows of Sec. III) taken from the admitted frames in arrival order.  A
 * long frame spreads over several iterations; frames that arrive while the
 * device is busy join the next one, and two iterations are in flight at
 * once.  Each iteration gathers its work list and its new frames' LLRs into
 * the device (on a stream of the server's own, so that it overlaps the
 * decode of the iteration before) and decodes its blocks with the batch
 * kernels on the configured stream, which write the decoded bytes straight
 * into the requests' places in the host region.  A frame's decoded bits are
 * identical to decoding it alone with vit_decode_ex and its code's
 * (L, v, v1); only the block is the unit of scheduling, and a block's path
 * metrics stay on chip.  Latency runs from the request's arrival time to the
 * moment the engine sees its last iteration finish (CLOCK_MONOTONIC). */
typedef struct vit_server vit_server;

typedef struct {
  uint32_t size;             /* sizeof(vit_server_config)                           */
  int32_t llr_type;          /* VIT_LLR_I8, VIT_LLR_F32 or VIT_LLR_HARD, every request */
  int32_t max_frames;        /* frames admitted to the device at once (slots), >= 1  */
  int32_t max_items;         /* blocks per iteration, >= 1                           */
  int32_t max_pending;       /* queued requests beyond which submit says VIT_EBUSY   */
  int32_t max_wait_ms;       /* a request still queued (not admitted) this long after
                                its arrival completes with VIT_ETIMEDOUT, undecoded;
                                checked in queue order; 0 = no limit                 */
  void *arena;               /* device, 256-aligned: admitted frames' LLRs           */
  size_t arena_bytes;        /* the memory budget that admission respects            */
  void *workspace;           /* device, 256-aligned, vit_server_workspace_size bytes */
  size_t workspace_bytes;
  void *host;                /* pinned host memory (hipHostMalloc) holding every
                                request's LLRs and decoded bytes                     */
  size_t host_bytes;
  void *stream;              /* hipStream_t the server works on (NULL = default)     */
  int32_t metric_bits;       /* integer inputs: as vit_opts.metric_bits (0 default)  */
  int32_t reserved;
} vit_server_config;

typedef struct {
  int32_t code_id;           /* index into the server's codes                        */
  int32_t terminated;        /* 1: k-1 tail stages follow the n information stages   */
  int64_t n;                 /* information bits, > 0                                */
  const void *llr;           /* inside the host region: N*beta LLRs of llr_type      */
  uint8_t *out;              /* inside the host region: ceil(n/8) bytes, written by
                                the device before the completion is reported         */
  uint64_t tag;              /* returned with the completion                         */
  int64_t arrival_ns;        /* CLOCK_MONOTONIC arrival time; <= 0 = time of submit  */
} vit_request;

typedef struct {
  uint64_t tag;
  int32_t status;            /* VIT_OK, VIT_ETIMEDOUT, or the device error that
                                stopped the server                                   */
  int32_t reserved;
  int64_t arrival_ns, done_ns;
} vit_completion;

typedef struct {
  int64_t submitted, completed, failed, bits_completed;
  int64_t iterations, items_launched;
  int64_t pending, frames_on_device, peak_frames_on_device, peak_arena_bytes;
  int64_t first_arrival_ns, last_done_ns;
  int64_t p50_ns, p99_ns, max_ns;   /* latency of completed frames */
  /* Where the time goes.  Device time per retired iteration, from events:
   * its ingest (work-list and LLR gather on the server's stream) and its
   * decode (batch kernels on the configured stream, from the moment that
   * stream starts it); summed, and the longest iteration from ingest start
   * to completion. */
  int64_t iter_ingest_ns, iter_decode_ns, iter_max_ns;
  /* Admission wait (admission time - arrival), summed and largest. */
  int64_t admit_wait_ns, admit_wait_max_ns;
  /* Hand-over lag of requests that carry an arrival time (the time they
   * reach vit_server_submit - arrival_ns: for vit_server_submit_paced, how
   * late the replay runs), summed over submit_lag_count requests, and the
   * largest. */
  int64_t submit_lag_ns, submit_lag_max_ns, submit_lag_count;
  /* Host time the engine thread spent scheduling and launching iterations. */
  int64_t engine_host_ns;
} vit_serve_stats;

/* Device workspace bytes for a configuration (two iterations' work lists). */
int vit_server_workspace_size(const vit_server_config *cfg, size_t *bytes);

/* Create a server for ncodes (1..8) codes with one block shape per code
 * (tune = NULL: L = 256, v = 5k for k <= 7 and 8(k-1) above, v1 = floor(v/2),
 * 1 wave per workgroup).
 * The arena, workspace and host region stay owned by the caller and must stay
 * valid until vit_server_destroy returns.  Errors: VIT_EINVAL for bad codes,
 * shapes, sizes or buffers (not device/pinned memory, misaligned, too small);
 * VIT_EUNSUPPORTED for shapes without a kernel; VIT_EDEVICE, VIT_ENOMEM. */
int vit_server_create(const vit_code *codes, int32_t ncodes, const vit_tuning *tune, const vit_server_config *cfg,
                      vit_server **server);

/* Queue requests in order.  *accepted receives how many were taken; on the
 * first one refused the call stops and returns VIT_EINVAL (bad request, or one
 * that can never fit the arena), VIT_EBUSY (queue full: retry later) or the
 * device error that stopped the server.  Thread-safe with poll and stats. */
int vit_server_submit(vit_server *server, const vit_request *reqs, int32_t count, int32_t *accepted);

/* Replay an arrival process: submit reqs in order, each no earlier than its
 * arrival_ns (CLOCK_MONOTONIC; requests with arrival_ns <= 0 go at once).
 * The calling thread sleeps or spins between arrivals and submits all
 * requests whose time has come in one batch; a full queue is retried.
 * Returns once every request is queued (*accepted = count) or on the first
 * refusal other than VIT_EBUSY, as vit_server_submit. */
int vit_server_submit_paced(vit_server *server, const vit_request *reqs, int32_t count, int32_t *accepted);

/* Move up to max completions (in completion order) into out; *count receives
 * how many.  A completion with status VIT_OK means its bytes are in place. */
int vit_server_poll(vit_server *server, vit_completion *out, int32_t max, int32_t *count);

/* Wait until every queued request has completed (timeout_ms < 0: no limit).
 * VIT_EBUSY on timeout. */
int vit_server_drain(vit_server *server, int64_t timeout_ms);

/* Counters and latency percentiles of the frames completed since creation or
 * the last reset (reset != 0 clears them after reading). */
int vit_server_stats(vit_server *server, vit_serve_stats *stats, int32_t reset);

/* Stop launching, wait for the iterations in flight, free the server.
 * Requests still queued are dropped without a completion. */
void vit_server_destroy(vit_server *server);

/* Thread-local description of the last error ("" if none). */
const char *vit_last_error(void);

/* VIT_ABI_VERSION of the built library. */
int vit_abi_version(void);

/* Test hook for the error paths (not part of the decode): the next `count`
 * host allocations at the library's allocation points fail as if memory were
 * exhausted (plan and server creation, the server's scheduler state, a batch's
 * output-range list, a statistics snapshot), and the call that made them
 * returns VIT_ENOMEM.  0 clears pending failures.  Process-wide; count < 0
 * returns VIT_EINVAL.  Independently of this hook, no C++ exception leaves any
 * entry point: a host allocation that fails inside the library returns
 * VIT_ENOMEM (inside the serving engine it fails the server with VIT_ENOMEM). */
int vit_debug_fail_allocations(int32_t count);

#ifdef __cplusplus
}
#endif
#endif
