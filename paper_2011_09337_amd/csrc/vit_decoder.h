// vit_decoder.h -- blocked soft-decision Viterbi decoder for gfx950 (MI355X):
// device templates, instantiated per constraint length in vit_kernels_k*.hip.
//
// One wave decodes one block (a frame of L core bits with v1 stages of history
// on the left and v2 on the right, Sec. III of the paper).  Forward procedure
// (eqs. 2-4) and traceback (Algorithm 2) run in the same kernel, with the
// survivor decisions kept in LDS for the block's lifetime (the point of the
// paper's unified kernel, Sec. IV-A).  Design, mapped to CDNA4 rather than
// following the paper's CUDA layout:
//
//  * State-per-slot layout.  Each of the S = 2^(k-1) states lives in one slot
//    (lane, register): 64 lanes x S/64 registers, or one state per lane for
//    k <= 7.  Instead of moving metrics to canonical positions each stage, the
//    state held by a slot rotates: after m stages slot j holds state
//    rotr^m(j) (k-1 bit rotation).  The two predecessors 2p, 2p+1 of a
//    butterfly then always sit in slots that differ in one bit q = m mod (k-1),
//    so each stage costs one pairwise exchange and no permutation.
//  * Slot bits 0..5 map to lanes through the xor patterns 1, 2, 7, 8, 16, 32:
//    the first four are single DPP patterns (quad_perm, row_half_mirror,
//    row_ror:8) fused into the add; 16 and 32 are in-place v_permlane16_swap /
//    v_permlane32_swap.  Slot bits 6.. are register bits (k = 8, 9).
//  * Sign-folded ACS.  A slot whose own predecessor is odd keeps its path
//    metric negated, so that "odd predecessor wins" is A > B in every lane and
//    the survivor metric is max or min (v_med3 against +-inf).  Since the
//    multiplier is +-1, fma(+-1, sigma, delta) rounds exactly like
//    sigma +- delta: every metric equals the oracle's, bit for bit.
//    Per state and stage: 2 fma, 1 compare, 1 med3, 1 add-with-carry that
//    shifts the decision bit into a per-lane word.
//  * Branch metrics (eq. 2): per tile of 64/2^beta stages the wave builds the
//    2^beta branch metrics of each stage (one per lane, summed left to right);
//    each stage every slot fetches its own one with ds_bpermute (LDS crossbar,
//    no VALU).  The complement identity (eq. 8) gives the partner branch as a
//    negation, folded into the fma.
//  * Decisions: 32 stages per dword per lane, stored to LDS.  Traceback runs
//    on the scalar unit: one v_readlane per stage; the lane to read moves by
//    replacing one bit of the slot index with the decision bit.
//  * The unrolled loop body covers lcm(k-1, tile, 32) stages; a block enters it
//    at an offset (Duff's device) chosen so that its last stage is the body's
//    last, which makes the final state of slot j equal to j.
#pragma once

#include "vit_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

namespace vit {
namespace dev {

// Largest d <= cap dividing n with n / d even (n is even, so d = 1 always fits).
constexpr int largest_even_split_divisor(int n, int cap) {
  int best = 1;
  for (int d = 1; d <= cap; ++d)
    if (n % d == 0 && (n / d) % 2 == 0) best = d;
  return best;
}

template <int K, int BETA>
struct Shape {
  static constexpr int P = K - 1;                      // bits of a state
  static constexpr int S = 1 << P;                     // states
  static constexpr int REGS = S > 64 ? S / 64 : 1;     // states per lane
  static constexpr int NCODE = 1 << BETA;              // output patterns
  // Unrolled body: a whole number of phase periods, at most 32 stages, so that
  // one body's decision bits fill one dword per state slot.
  static constexpr int BODY = P * (32 / P);
  // Stages per branch-metric tile: a divisor of the body that fits 64 lanes
  // and leaves an even number of tiles per body (the LLR loads run two tiles
  // ahead through two buffers whose roles alternate tile by tile).
  static constexpr int T = largest_even_split_divisor(BODY, 64 / NCODE);
};

// Physical lane xor pattern of slot bit q (q < 6).
__host__ __device__ constexpr int lane_vec(int q) {
  return q == 0 ? 1 : q == 1 ? 2 : q == 2 ? 7 : q == 3 ? 8 : q == 4 ? 16 : 32;
}

// Sign factor that register `reg` adds to the lane sign of phase q: bits q and
// q-1 of the slot index (reg << 6 | lane slot) decide the sign convention.
template <int P>
__host__ __device__ constexpr bool reg_neg(int q, int reg) {
  const int hi = reg << 6;
  return (((hi >> q) ^ (hi >> ((q + P - 1) % P))) & 1) != 0;
}

__device__ __forceinline__ int parity32(uint32_t x) { return __builtin_popcount(x) & 1; }

// ---------------------------------------------------------------- ACS kernels
// One ACS of one slot: o is the slot's stored metric (updated), x the
// partner branch metric, sign-adjusted for this slot (consumed), s = +-1,
// c = +inf (keep the max) or -inf (keep the min).  The compare mask of this
// stage is returned in `pend` and shifted into the decision word d by the NEXT
// stage's block (d = 2d + pend), which keeps every hazard distance >= 2
// instructions without s_nop:
//   * the DPP read of o comes 2 VALU ops after the previous stage's med3 wrote it;
//   * the VALU-written compare mask is read as a carry 2 VALU ops after.
// Instruction order: B = s*o - x; d += prev mask; A = s*o(partner) + x;
// mask = A > B; o = med3(A, B, c).
#define VIT_ACS_DPP(DPPSTR, SN, BTERM)                                                   \
  asm volatile("v_fma_f32 %[B], " SN "%[s], %[o], " BTERM "\n\t"                         \
               "v_addc_co_u32 %[d], vcc, %[d], %[d], %[pd]\n\t"                          \
               "v_fmac_f32_dpp %[x], %[o], " SN "%[s] " DPPSTR "\n\t"                    \
               "v_cmp_gt_f32 %[pd], %[x], %[B]\n\t"                                      \
               "v_med3_f32 %[o], %[x], %[B], %[c]"                                       \
               : [o] "+v"(o), [x] "+v"(x), [d] "+v"(d), [B] "=&v"(B), [pd] "+s"(pend)    \
               : [s] "v"(s), [c] "v"(c), [y] "v"(y)                                      \
               : "vcc")

// Slot bits 4 and 5 flip lane bits 4 and 5 (xor 16 / xor 32): the partner
// metric comes from v_permlane16_swap / v_permlane32_swap of o with itself,
// which exchanges the two halves of each row pair / of the wave in place (o is
// dead after B, and rewritten by med3).  Same hazard distances as the DPP form.
#define VIT_ACS_PERM(PERM, SN, BTERM)                                                    \
  asm volatile("v_fma_f32 %[B], " SN "%[s], %[o], " BTERM "\n\t"                         \
               "v_addc_co_u32 %[d], vcc, %[d], %[d], %[pd]\n\t"                          \
               PERM " %[o], %[o]\n\t"                                                    \
               "v_fma_f32 %[x], " SN "%[s], %[o], %[x]\n\t"                              \
               "v_cmp_gt_f32 %[pd], %[x], %[B]\n\t"                                      \
               "v_med3_f32 %[o], %[x], %[B], %[c]"                                       \
               : [o] "+v"(o), [x] "+v"(x), [d] "+v"(d), [B] "=&v"(B), [pd] "+s"(pend)    \
               : [s] "v"(s), [c] "v"(c), [y] "v"(y)                                      \
               : "vcc")

// Both predecessors in the same lane (slot bit q >= 6 is a register bit):
// registers a (own predecessor even) and b (odd).
#define VIT_ACS_PAIR(SA, SB, BTA, BTB)                                                   \
  asm volatile("v_fma_f32 %[Ba], " SA "%[s], %[oa], " BTA "\n\t"                         \
               "v_addc_co_u32 %[da], vcc, %[da], %[da], %[pa]\n\t"                       \
               "v_fma_f32 %[xa], " SA "%[s], %[ob], %[xa]\n\t"                           \
               "v_fma_f32 %[Bb], " SB "%[s], %[ob], " BTB "\n\t"                         \
               "v_addc_co_u32 %[db], vcc, %[db], %[db], %[pb]\n\t"                       \
               "v_fma_f32 %[xb], " SB "%[s], %[oa], %[xb]\n\t"                           \
               "v_cmp_gt_f32 %[pa], %[xa], %[Ba]\n\t"                                    \
               "v_med3_f32 %[oa], %[xa], %[Ba], %[ca]\n\t"                               \
               "v_cmp_gt_f32 %[pb], %[xb], %[Bb]\n\t"                                    \
               "v_med3_f32 %[ob], %[xb], %[Bb], %[cb]"                                   \
               : [oa] "+v"(oa), [ob] "+v"(ob), [xa] "+v"(xa), [xb] "+v"(xb),             \
                 [da] "+v"(da), [db] "+v"(db), [Ba] "=&v"(Ba), [Bb] "=&v"(Bb),           \
                 [pa] "+s"(pa), [pb] "+s"(pb)                                            \
               : [s] "v"(s), [ca] "v"(ca), [cb] "v"(cb), [ya] "v"(ya), [yb] "v"(yb)      \
               : "vcc")

// Shift the last pending decision mask into the word (end of a body).
__device__ __forceinline__ void flush_decision(uint32_t &d, uint64_t &pend) {
  asm volatile("s_nop 1\n\t"
               "v_addc_co_u32 %[d], vcc, %[d], %[d], %[pd]"
               : [d] "+v"(d)
               : [pd] "s"(pend)
               : "vcc");
  pend = 0;
}

#define VIT_DPP_Q0 "quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf"
#define VIT_DPP_Q1 "quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf"
#define VIT_DPP_Q2 "row_half_mirror row_mask:0xf bank_mask:0xf"
#define VIT_DPP_Q3 "row_ror:8 row_mask:0xf bank_mask:0xf"

template <int Q, bool NEG, bool STD>
__device__ __forceinline__ void acs_lane(float &o, float &x, uint32_t &d, uint64_t &pend, float s, float c,
                                         float y) {
  float B;
  if constexpr (Q < 4) {
#define VIT_DISPATCH_DPP(DPPSTR)                                                            \
  if constexpr (STD) {                                                                      \
    if constexpr (NEG) VIT_ACS_DPP(DPPSTR, "-", "-%[x]"); else VIT_ACS_DPP(DPPSTR, "", "-%[x]"); \
  } else {                                                                                  \
    if constexpr (NEG) VIT_ACS_DPP(DPPSTR, "-", "%[y]"); else VIT_ACS_DPP(DPPSTR, "", "%[y]");   \
  }
    if constexpr (Q == 0) { VIT_DISPATCH_DPP(VIT_DPP_Q0) }
    else if constexpr (Q == 1) { VIT_DISPATCH_DPP(VIT_DPP_Q1) }
    else if constexpr (Q == 2) { VIT_DISPATCH_DPP(VIT_DPP_Q2) }
    else { VIT_DISPATCH_DPP(VIT_DPP_Q3) }
#undef VIT_DISPATCH_DPP
  } else {
    if constexpr (Q == 4) {
      if constexpr (STD) {
        if constexpr (NEG) VIT_ACS_PERM("v_permlane16_swap_b32", "-", "-%[x]");
        else VIT_ACS_PERM("v_permlane16_swap_b32", "", "-%[x]");
      } else {
        if constexpr (NEG) VIT_ACS_PERM("v_permlane16_swap_b32", "-", "%[y]");
        else VIT_ACS_PERM("v_permlane16_swap_b32", "", "%[y]");
      }
    } else {
      if constexpr (STD) {
        if constexpr (NEG) VIT_ACS_PERM("v_permlane32_swap_b32", "-", "-%[x]");
        else VIT_ACS_PERM("v_permlane32_swap_b32", "", "-%[x]");
      } else {
        if constexpr (NEG) VIT_ACS_PERM("v_permlane32_swap_b32", "-", "%[y]");
        else VIT_ACS_PERM("v_permlane32_swap_b32", "", "%[y]");
      }
    }
  }
}

template <bool NA, bool NB, bool STD>
__device__ __forceinline__ void acs_pair(float &oa, float &ob, float &xa, float &xb, uint32_t &da,
                                         uint32_t &db, uint64_t &pa, uint64_t &pb, float s, float ca, float cb,
                                         float ya, float yb) {
  float Ba, Bb;
#define VIT_PAIR_SIGNS(BTA, BTB)                                             \
  if constexpr (NA && NB) VIT_ACS_PAIR("-", "-", BTA, BTB);                  \
  else if constexpr (NA) VIT_ACS_PAIR("-", "", BTA, BTB);                    \
  else if constexpr (NB) VIT_ACS_PAIR("", "-", BTA, BTB);                    \
  else VIT_ACS_PAIR("", "", BTA, BTB);
  if constexpr (STD) {
    VIT_PAIR_SIGNS("-%[xa]", "-%[xb]")
  } else {
    VIT_PAIR_SIGNS("%[ya]", "%[yb]")
  }
#undef VIT_PAIR_SIGNS
}

// ---------------------------------------------------------------- decoder
// Register rsel (uniform) of a per-lane register array, without branches.
template <int REGS>
__device__ __forceinline__ uint32_t select_reg(const uint32_t (&v)[REGS], uint32_t rsel) {
  typedef uint32_t vec_t __attribute__((ext_vector_type(REGS)));
  vec_t t;
#pragma unroll
  for (int i = 0; i < REGS; ++i) t[i] = v[i];
  return t[rsel & (REGS - 1)];
}

// IN: input kind, VIT_LLR_F32 (float LLRs), VIT_LLR_I8 (int8 LLRs) or
// VIT_LLR_HARD (hard-decision bytes), fixed per kernel instance.
template <int K, int BETA, bool STD, int IN>
struct Decoder {
  static constexpr bool I8 = IN != VIT_LLR_F32;       // one byte per value
  static constexpr bool HARD = IN == VIT_LLR_HARD;
  using Sh = Shape<K, BETA>;
  static constexpr int P = Sh::P, S = Sh::S, REGS = Sh::REGS, NCODE = Sh::NCODE, T = Sh::T,
                       BODY = Sh::BODY;
  static constexpr int NY = STD ? 1 : P;
  static constexpr int RY = STD ? 1 : REGS;

  // per-lane constants (depend only on the code)
  int addr_x[P][REGS];   // byte address of this slot's partner branch metric within a stage
  int addr_y[NY][RY];    // own branch metric (codes without both end taps)
  float sgn[P];          // sign convention product for register 0
  float cmed[P];         // +inf / -inf for lane-bit phases
  float bsign[BETA];     // signs of this lane's output pattern in the metric table
  int tl;                // stage of this lane's metric table entry within a tile
  int lane;
  int slot0;             // slot index of register 0 in this lane
  uint32_t own_mask[REGS];  // per body offset: bit q of this slot's index (traceback encoding)

  // per-block state
  float o[REGS];
  uint32_t dec[REGS];
  uint64_t pend[REGS];       // compare mask of the last stage, not yet in dec
  float xn[REGS], yn[REGS];  // branch metrics prefetched for the next step
  int table;
  int nxt[2][BETA];      // raw LLR words of the next two tiles (float bits or sign-extended int8);
                         // tile tau lives in buffer tau % 2
  const void *llr;
  int64_t stage_base, s, e;
  int tile_stage0;       // stage_base + this lane's table row
  int s_lo, s_hi;        // first and last stage of the block
  uint32_t *lds;
  int body;

  // Byte offset, within one stage of the metric table, of the branch metric a
  // slot needs at phase q: the partner branch (own = false) or its own
  // branch (own = true), negated (complemented pattern) if the slot keeps its
  // metric negated.  Slot = (reg << 6) | slot0 holds state rotr^q(slot) as
  // predecessor; the branch register is (input u << (k-1)) | predecessor with
  // u = the predecessor's low bit, and the partner predecessor differs in bit 0.
  __device__ __forceinline__ int metric_addr(const uint32_t *gen, int q, int reg, bool own) const {
    const int st = ((reg << 6) | slot0) & (S - 1);
    const int up = (st >> q) & 1;
    const uint32_t iown = (uint32_t)(((st >> q) | (st << (P - q))) & (S - 1));
    const uint32_t rown = ((uint32_t)up << (K - 1)) | iown;
    const uint32_t rb = own ? rown : (rown ^ 1u);
    int c = 0;
#pragma unroll
    for (int b = 0; b < BETA; ++b) c |= parity32(gen[b] & rb) << b;
    return (c ^ (up ? NCODE - 1 : 0)) << 2;
  }

  // Codes whose generators all tap both ends of the register: the partner
  // address above reduces to the complemented output pattern of the rotated
  // slot index, and bit b of that pattern is the parity of the slot index
  // with generator b's low P bits rotated left by q (uniform, so the rotation
  // is scalar work).
  __device__ __forceinline__ int partner_addr_std(const uint32_t *gen, int q, int reg) const {
    const uint32_t st = (uint32_t)(((reg << 6) | slot0) & (S - 1));
    int c = 0;
#pragma unroll
    for (int b = 0; b < BETA; ++b) c |= parity32(rotl_p(gen[b] & (uint32_t)(S - 1), q) & st) << b;
    return (c ^ (NCODE - 1)) << 2;
  }

  __device__ __forceinline__ void setup(const uint32_t *gen) {
    lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    slot0 = lane ^ (((lane >> 2) & 1) ? 3 : 0);  // inverse of the lane_vec map
    tl = lane >> BETA;
    const int pat = lane & (NCODE - 1);
#pragma unroll
    for (int b = 0; b < BETA; ++b) bsign[b] = ((pat >> b) & 1) ? -1.0f : 1.0f;
#pragma unroll
    for (int q = 0; q < P; ++q) {
#pragma unroll
      for (int reg = 0; reg < REGS; ++reg) {
        if constexpr (STD) {
          addr_x[q][reg] = partner_addr_std(gen, q, reg);
        } else {
          addr_x[q][reg] = metric_addr(gen, q, reg, false);
          addr_y[q][reg] = metric_addr(gen, q, reg, true);
        }
      }
      const int st0 = slot0 & (S - 1);
      const int bq = (st0 >> q) & 1, bqm = (st0 >> ((q + P - 1) % P)) & 1;
      sgn[q] = (bq ^ bqm) ? -1.0f : 1.0f;
      cmed[q] = bq ? -INFINITY : INFINITY;
    }
    // The survivor word of a slot stores, for body offset pos (bit BODY-1-pos),
    // its decision XOR bit (pos mod P) of the slot index: following the
    // survivor then flips that bit of the traceback's slot index instead of
    // replacing it.
    // Body offset pos = P*a + j sits at bit BODY-1-pos, so period a holds the
    // slot's P bits reversed (bit P-1-j = slot bit j) at bit BODY-P-P*a: one
    // reversed copy, repeated by a multiply (the copies do not overlap).
    constexpr uint32_t kRep = [] {
      uint32_t r = 0;
      for (int a = 0; a < BODY / P; ++a) r |= 1u << (BODY - P - P * a);
      return r;
    }();
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      const uint32_t st = (uint32_t)(((reg << 6) | slot0) & (S - 1));
      own_mask[reg] = (__builtin_bitreverse32(st) >> (32 - P)) * kRep;
    }
  }

  // LLRs of tile tau (stages stage_base + tau*T + 0..T-1, one per table row),
  // clamped into the block so every lane reads inside the stream, into buffer
  // BUF.  Offsets are 32-bit (the host guarantees N*beta*sizeof(LLR) < 2^32).
  template <int BUF>
  __device__ __forceinline__ void load_tile(int tau) {
    const int raw = tile_stage0 + tau * T;
    const int stc = __builtin_elementwise_max(__builtin_elementwise_min(raw, s_hi), s_lo);
    const uint32_t off = (uint32_t)stc * (uint32_t)(BETA * (I8 ? 1 : 4));
    const char *base = (const char *)llr;
    if constexpr (I8) {
      const int8_t *p = (const int8_t *)(base + off);
#pragma unroll
      for (int b = 0; b < BETA; ++b) nxt[BUF][b] = p[b];
    } else {
      const int *p = (const int *)(base + off);
#pragma unroll
      for (int b = 0; b < BETA; ++b) nxt[BUF][b] = p[b];
    }
  }
  // Same, with the buffer chosen at run time (block prologue only).
  __device__ __forceinline__ void load_tile_rt(int tau) {
    if (tau & 1) load_tile<1>(tau);
    else load_tile<0>(tau);
  }

  // eq. (2) for output pattern `pat` of this lane: sum in order b = 0..beta-1;
  // fma with a +-1 multiplier rounds exactly like the plain add.
  __device__ __forceinline__ float llr_value(int raw) const {
    if constexpr (I8) {
      if constexpr (HARD) return raw == 0 ? 1.0f : -1.0f;  // hard decision: coded bit 0 -> +1, 1 -> -1
      return (float)raw;                         // exact: |int8| <= 128
    } else {
      return __builtin_bit_cast(float, raw);
    }
  }

  template <int BUF>
  __device__ __forceinline__ void build_table() {
    float dl = llr_value(nxt[BUF][0]) * bsign[0];
#pragma unroll
    for (int b = 1; b < BETA; ++b) dl = __builtin_fmaf(bsign[b], llr_value(nxt[BUF][b]), dl);
    table = __builtin_bit_cast(int, dl);
  }
  __device__ __forceinline__ void build_table_rt(int tau) {
    if (tau & 1) build_table<1>();
    else build_table<0>();
  }

  // Hide the per-lane branch-metric addresses from loop-invariant code motion
  // so that each fetch keeps its tile offset in the instruction's offset field.
  __device__ __forceinline__ void refresh_addresses() {
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int reg = 0; reg < REGS; ++reg) {
        asm volatile("" : "+v"(addr_x[q][reg]));
        if constexpr (!STD) asm volatile("" : "+v"(addr_y[q][reg]));
      }
  }

  __device__ __forceinline__ float fetch(int addr, int tlc) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr + tlc * NCODE * 4, table));
  }

  // Branch metrics of the slots for the step at body offset G (tile table
  // already holding G's tile).
  template <int G>
  __device__ __forceinline__ void fetch_step(float (&x)[REGS], float (&y)[REGS]) const {
    constexpr int q = G % P;
    constexpr int tlc = G % T;
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      x[reg] = fetch(addr_x[q][reg], tlc);
      if constexpr (!STD) y[reg] = fetch(addr_y[q][reg], tlc);
      else y[reg] = 0.0f;
    }
  }

  // Same, for a runtime body offset (the entry step of a block); the
  // addresses are recomputed rather than indexed, to stay in registers.
  __device__ __forceinline__ void fetch_entry(const uint32_t *gen, int g, float (&x)[REGS],
                                              float (&y)[REGS]) const {
    const int q = g % P, tlc = g % T;
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      x[reg] = fetch(metric_addr(gen, q, reg, false), tlc);
      y[reg] = STD ? 0.0f : fetch(metric_addr(gen, q, reg, true), tlc);
    }
  }

  // One trellis stage at body offset G.  Software pipeline: the branch
  // metrics of this step were fetched by the previous step (xn, yn); this
  // step fetches the next step's before running its own ACS.  The LLRs of
  // tile t+2 are loaded when tile t starts (into the buffer tile t used);
  // tile t+1's metric table is built at the last step of tile t.  A body
  // holds an even number of tiles, so tile parity is (G / T) % 2.
  template <int G>
  __device__ __forceinline__ void step() {
    constexpr int q = G % P;
    constexpr int tlc = G % T;
    float x[REGS], y[REGS];
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      x[reg] = xn[reg];
      y[reg] = yn[reg];
    }
    constexpr int par = (G / T) % 2;
    if constexpr (tlc == 0) load_tile<par>(body * (BODY / T) + G / T + 2);
    if constexpr (tlc == T - 1) build_table<par ^ 1>();
    fetch_step<(G + 1) % BODY>(xn, yn);
    if constexpr (q < 6) {
#pragma unroll
      for (int reg = 0; reg < REGS; ++reg) step_lane<q>(reg, x[reg], y[reg]);
    } else {
      constexpr int bit = 1 << (q - 6);
#pragma unroll
      for (int ra = 0; ra < REGS; ++ra) {
        if ((ra & bit) == 0) step_pair<q>(ra, ra | bit, x[ra], x[ra | bit], y[ra], y[ra | bit]);
      }
    }
    if constexpr (G == BODY - 1) {
#pragma unroll
      for (int reg = 0; reg < REGS; ++reg) {
        flush_decision(dec[reg], pend[reg]);
        lds[(body * REGS + reg) * 64 + slot0] = dec[reg] ^ own_mask[reg];
      }
    }
  }

  // Wave-wide max of v, in every lane: a butterfly over lane xor 1, 2, 7, 8
  // (max fused with a DPP read: quad_perm, row_half_mirror, row_ror:8) and
  // xor 16, 32 (in-place v_permlane16/32_swap of a copy).  For the finite
  // metrics here it equals a chain of fmaxf without the compiler's NaN
  // quieting of every operand.  Each s_nop 1 covers the two wait states
  // between a VALU write and the next DPP or permlane read of that register.
  __device__ __forceinline__ static float wave_max(float v) {
    float t;
    asm volatile(
        "s_nop 1\n\t"
        "v_max_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_max_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_max_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_max_f32_dpp %0, %0, %0 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_mov_b32 %1, %0\n\t"
        "s_nop 1\n\t"
        "v_permlane16_swap_b32 %1, %1\n\t"
        "s_nop 1\n\t"
        "v_max_f32 %0, %0, %1\n\t"
        "v_mov_b32 %1, %0\n\t"
        "s_nop 1\n\t"
        "v_permlane32_swap_b32 %1, %1\n\t"
        "s_nop 1\n\t"
        "v_max_f32 %0, %0, %1"
        : "+v"(v), "=&v"(t));
    return v;
  }

  // Rotation of a P-bit slot or state index by r places (0 <= r < P).
  __device__ __forceinline__ static uint32_t rotr_p(uint32_t x, int r) {
    return ((x >> r) | (x << ((P - r) % P))) & (uint32_t)(S - 1);
  }
  __device__ __forceinline__ static uint32_t rotl_p(uint32_t x, int r) {
    return ((x << r) | (x >> ((P - r) % P))) & (uint32_t)(S - 1);
  }

  // Slot holding the best state after the step at body offset G (any G):
  // slot j then holds state rotr^(G+1)(j) with the sign convention of phase
  // G mod P; largest metric, lowest state index on ties.  Uniform.
  template <int G>
  __device__ __forceinline__ int best_slot_after() const {
    constexpr int qg = G % P, rot = (G + 1) % P;
    // The largest metric by max, then the slot holding it; this runs between
    // trellis steps, with their pending compare masks live in SGPRs.
    float best = -INFINITY;
    int labs[REGS];
    float sigs[REGS];
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      const int slot = ((reg << 6) | slot0) & (S - 1);
      labs[reg] = (int)rotr_p((uint32_t)slot, rot);
      sigs[reg] = ((slot >> qg) & 1) ? -o[reg] : o[reg];
    }
    if constexpr (S >= 64) {
      // Every lane holds distinct slots: the largest metric by a butterfly of
      // in-register lane exchanges (no LDS round trips), then, when a single
      // slot holds it (the usual case with real-valued LLRs), that slot
      // straight from the ballot.
      float m = sigs[0];
#pragma unroll
      for (int reg = 1; reg < REGS; ++reg) m = __builtin_fmaxf(m, sigs[reg]);
      best = wave_max(m);
      uint64_t hit[REGS];
      int nhit = 0;
#pragma unroll
      for (int reg = 0; reg < REGS; ++reg) {
        hit[reg] = __builtin_amdgcn_ballot_w64(sigs[reg] == best);
        nhit += __builtin_popcountll(hit[reg]);
      }
      if (nhit == 1) {
        int slot = 0;
#pragma unroll
        for (int reg = 0; reg < REGS; ++reg)
          if (hit[reg]) {
            const int l = __builtin_ctzll(hit[reg]);
            slot = (reg << 6) | (l ^ (((l >> 2) & 1) ? 3 : 0));
          }
        return slot & (S - 1);
      }
    } else {
#pragma unroll
      for (int reg = 0; reg < REGS; ++reg) best = __builtin_fmaxf(best, sigs[reg]);
      // (lane exchanges by ds_bpermute at lane ^ m; the compiler's shuffle
      // helper adds a width compare that does not compile here)
#pragma unroll
      for (int m = 1; m < 64; m <<= 1)
        best = __builtin_fmaxf(best, __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(
                                                                    (lane ^ m) << 2, __builtin_bit_cast(int, best))));
    }
    // ties (or fewer states than lanes): the lowest label holding the maximum
    int lab = 0x7fffffff;
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      const int cand = sigs[reg] == best ? labs[reg] : 0x7fffffff;
      lab = cand < lab ? cand : lab;
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      const int ol = __builtin_amdgcn_ds_bpermute((lane ^ m) << 2, lab);
      lab = ol < lab ? ol : lab;
    }
    return (int)rotl_p((uint32_t)__builtin_amdgcn_readfirstlane(lab), rot);
  }

  // Slot index of the best state at a body end, where slot j holds state j
  // with the sign convention of the body's last phase; lowest index on ties.
  // Uniform across the wave.  This is the snapshot after the body's last step
  // (BODY is a multiple of P, so the rotation there is the identity).
  __device__ __forceinline__ int best_state() const { return best_slot_after<BODY - 1>(); }

  // Traceback (Algorithm 2) through one group (body) of survivor words for
  // each of NCH independent chains, interleaved so that the scalar steps of
  // one chain fill the latency of the other's.  ulam[c] is chain c's slot
  // index (the current state).  Following the survivor at body offset pos
  // replaces bit q = pos mod P of the slot index with the decision bit; the
  // survivor words hold that bit XOR the slot's own bit q, so the step is
  // ulam ^= (word bit) << q.  The words are bit-reversed and, per phase
  // period p0..p0+P-1, shifted so that offset p0 + q sits at bit q: a step is
  // one v_readlane and two scalar operations.  After a period the slot index
  // holds that period's P decision bits; the group's decision word replaces
  // its first survivor word in LDS when wr[c] (every lane writes the same
  // word).
  template <int NCH>
  __device__ __forceinline__ void tb_groups(const int (&grp)[NCH], uint32_t (&ulam)[NCH],
                                            const bool (&wr)[NCH]) const {
    uint32_t dv[NCH][REGS];
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int rr = 0; rr < REGS; ++rr) dv[c][rr] = __builtin_bitreverse32(lds[(grp[c] * REGS + rr) * 64 + lane]);
    uint32_t acc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = 0;
#pragma unroll
    for (int p0 = BODY - P; p0 >= 0; p0 -= P) {
      uint32_t sh[NCH][REGS], src[NCH];
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
#pragma unroll
        for (int rr = 0; rr < REGS; ++rr) sh[c][rr] = dv[c][rr] >> (32 - BODY + p0);
        src[c] = sh[c][0];
      }
#pragma unroll
      for (int q = P - 1; q >= 0; --q) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          if constexpr (REGS > 1) {
            // the register holding slot ulam is given by bits >= 6 of the
            // slot index, which change only at q >= 6: select at q >= 5 only
            if (q >= 5) src[c] = select_reg<REGS>(sh[c], ulam[c] >> 6);
          }
          const uint32_t w = __builtin_amdgcn_readlane(src[c], (int)(ulam[c] & 63u));
          ulam[c] ^= w & (1u << q);
        }
      }
#pragma unroll
      for (int c = 0; c < NCH; ++c) acc[c] |= (ulam[c] & (uint32_t)(S - 1)) << p0;
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c)
      if (wr[c]) lds[(grp[c] * REGS) * 64] = acc[c];
  }

  template <int Q>
  __device__ __forceinline__ void step_lane(int reg, float x, float y) {
    // unrolled by the caller, so `reg` is a constant after inlining
#pragma unroll
    for (int r = 0; r < REGS; ++r) {
      if (r == reg) {
        if (reg_neg<P>(Q, r)) acs_lane<Q, true, STD>(o[r], x, dec[r], pend[r], sgn[Q], cmed[Q], y);
        else acs_lane<Q, false, STD>(o[r], x, dec[r], pend[r], sgn[Q], cmed[Q], y);
      }
    }
  }

  template <int Q>
  __device__ __forceinline__ void step_pair(int ra, int rb, float xa, float xb, float ya, float yb) {
#pragma unroll
    for (int r = 0; r < REGS; ++r) {
      if (r == ra) {
        const bool na = reg_neg<P>(Q, ra), nb = reg_neg<P>(Q, rb);
        const float cpos = INFINITY, cneg = -INFINITY;
        if (na && nb) acs_pair<true, true, STD>(o[ra], o[rb], xa, xb, dec[ra], dec[rb], pend[ra], pend[rb], sgn[Q], cpos, cneg, ya, yb);
        else if (na) acs_pair<true, false, STD>(o[ra], o[rb], xa, xb, dec[ra], dec[rb], pend[ra], pend[rb], sgn[Q], cpos, cneg, ya, yb);
        else if (nb) acs_pair<false, true, STD>(o[ra], o[rb], xa, xb, dec[ra], dec[rb], pend[ra], pend[rb], sgn[Q], cpos, cneg, ya, yb);
        else acs_pair<false, false, STD>(o[ra], o[rb], xa, xb, dec[ra], dec[rb], pend[ra], pend[rb], sgn[Q], cpos, cneg, ya, yb);
      }
    }
  }
};

// SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) as a counter-based generator: output i (i = 0,
// 1, ...) of the sequential generator seeded with `seed`, i.e. the published
// mix function applied to seed + (i + 1) * 0x9E3779B97F4A7C15.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Parallel traceback of Sec. IV-D (SUB instances): subframes of f0 core bits,
// w stages of inner overlap, inner chains started from the stored best state
// (VIT_SUBFRAME_STORED) or a random state (VIT_SUBFRAME_RANDOM, SplitMix64 of
// seed at counter (block << 32) | subframe).
struct SubframeArgs {
  int32_t f0, w, start;
  uint64_t seed;
  int64_t block;
};

// The first (partial) body of a block: step G runs only from the entry offset
// r on (uniform, scalar branches).  Later bodies run every step unguarded.
// SUB instances take, after step G, the best state an inner subframe chain
// starts from when its start stage is that step (sr = its body offset).
#define VIT_SNAP(NN)                                                 \
  if constexpr (SUB) {                                               \
    if ((NN) == sr) take_snapshot(D.template best_slot_after<(NN)>()); \
  }
#define VIT_G1(NN, M)                                        \
  if constexpr ((NN) < (M)) {                                \
    if ((NN) >= r) {                                         \
      D.template step<(NN)>();                               \
      VIT_SNAP(NN)                                           \
    }                                                        \
  }
#define VIT_U1(NN, M)                                        \
  if constexpr ((NN) < (M)) {                                \
    D.template step<(NN)>();                                 \
    VIT_SNAP(NN)                                             \
  }
#define VIT_X8(X, B, M)                                                                  \
  X(B + 0, M) X(B + 1, M) X(B + 2, M) X(B + 3, M) X(B + 4, M) X(B + 5, M) X(B + 6, M)   \
  X(B + 7, M)
#define VIT_X32(X, M) VIT_X8(X, 0, M) VIT_X8(X, 8, M) VIT_X8(X, 16, M) VIT_X8(X, 24, M)

// Decode one block (Sec. III): trellis stages [s, e) of a frame whose LLRs
// start (stage 0) at `llr` and whose decoded bits start (bit 0) at byte `out`;
// emit core bits [cs, ce).  start_known: the window starts at the frame's
// first stage (state 0); end_zero: it ends at the last stage of a terminated
// frame (trace back from state 0).  SUB instances run the parallel traceback
// of Sec. IV-D (sa: subframes of f0 bits, one lane per chain; the caller
// guarantees at most 64 subframes and ceil((ce - cs) / 4) spare words of LDS
// after the survivors); others trace each block once from its end.  Stages
// are frame-local; the caller guarantees (e - s) * beta * sizeof(LLR) <
// 2^31 and cs a multiple of 8.
template <bool SUB, int K, int BETA, bool STD, int IN>
__device__ __forceinline__ void decode_block(Decoder<K, BETA, STD, IN> &D, const void *llr, uint8_t *out,
                                             int64_t s, int64_t e, int64_t cs, int64_t ce, bool start_known,
                                             bool end_zero, const SubframeArgs &sa, const uint32_t *gen) {
  using Sh = Shape<K, BETA>;
  constexpr int P = Sh::P, S = Sh::S, REGS = Sh::REGS, BODY = Sh::BODY, T = Sh::T;
  (void)T;
  D.llr = llr;
  const int M = (int)(e - s);
  const int r = (BODY - M % BODY) % BODY;
  const int nbody = (M + r) / BODY;
  D.s = s;
  D.e = e;
  D.stage_base = s - r;
  D.tile_stage0 = (int)(s - r) + D.tl;
  D.s_lo = (int)s;
  D.s_hi = (int)e - 1;
  D.body = 0;

  // Subframe geometry (Sec. IV-D).  The core [cs, ce) splits into C
  // subframes of f0 bits; subframe c = [cs + c f0, min(cs + (c+1) f0, ce))
  // is traced from stage x_c - 1 down, x_c = e for the last one or where its
  // end plus w reaches e, else its end plus w.  The inner chains (x_c < e)
  // are c = 0 .. n_inner - 1; with the stored start rule the forward pass
  // keeps the best state after each stage x_c - 1 in lane c of snap_v.
  const int f0 = SUB ? sa.f0 : 1;
  const int C = SUB ? (int)((ce - cs + f0 - 1) / f0) : 1;
  int n_inner = 0;
  if constexpr (SUB) {
    // c < C - 1 and cs + (c + 1) f0 + w < e
    const int64_t room = e - 1 - sa.w - cs;  // (c + 1) f0 <= room
    n_inner = room >= f0 ? (int)(room / f0) : 0;
    if (n_inner > C - 1) n_inner = C - 1;
  }
  uint32_t snap_v = 0;
  int snap_c = 0;
  // body offset, in the current body, of the next snapshot (none: -1)
  int64_t snap_rel = (SUB && sa.start == VIT_SUBFRAME_STORED && n_inner > 0)
                         ? (cs + f0 + sa.w - 1) - D.stage_base : -1;
  int sr = -1;
  auto take_snapshot = [&](int slot) {
    snap_v = D.lane == snap_c ? (uint32_t)slot : snap_v;
    ++snap_c;
    if (snap_c < n_inner) {
      snap_rel += f0;
      sr += f0;
    } else {
      snap_rel = -1;
      sr = -1;
    }
  };
  (void)take_snapshot;

  // Initial metrics: state 0 known at the stream start, else all zero.  The
  // slot holding state rotr^r(slot) keeps it with sign convention of phase r-1.
  {
    const int qm1 = (r + P - 1) % P;
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      const int slot = ((reg << 6) | D.slot0) & (S - 1);
      const bool neg = (slot >> qm1) & 1;
      D.o[reg] = (start_known && slot != 0) ? (neg ? INFINITY : -INFINITY) : 0.0f;
      D.dec[reg] = 0u;
      D.pend[reg] = 0u;
    }
  }
  // Pipeline prologue for the entry step r: metric table of its tile tau0,
  // raw LLRs of tiles tau0+1 and tau0+2 (the step that starts a tile loads
  // the one two ahead; if the block enters mid-tile that step is skipped),
  // and the entry step's own branch metrics.
  {
    const int tau0 = r / T;
    D.load_tile_rt(tau0);
    D.build_table_rt(tau0);
    D.load_tile_rt(tau0 + 1);
    if (r % T != 0) D.load_tile_rt(tau0 + 2);
    D.body = 0;
    D.fetch_entry(gen, r, D.xn, D.yn);
  }
  D.body = 0;
  D.refresh_addresses();
  if constexpr (SUB) sr = snap_rel >= 0 && snap_rel < BODY ? (int)snap_rel : -1;
  VIT_X32(VIT_G1, BODY)
  for (D.body = 1; D.body < nbody; ++D.body) {
    D.refresh_addresses();
    if constexpr (SUB) {
      const int64_t rel = snap_rel - (int64_t)D.body * BODY;
      sr = snap_rel >= 0 && rel < BODY ? (int)rel : -1;
    }
    VIT_X32(VIT_U1, BODY)
  }

  // ---- traceback start: state 0 at a terminated end, else the best state.
  const int lam = end_zero ? 0 : D.best_state();

  if constexpr (SUB) {
    // ---- parallel traceback (Sec. IV-D): lane c runs subframe c's chain.
    // The chain holds the slot u of its state after stage t; at a stage of
    // body offset pos (q = pos mod P) the decoded bit of stage t is bit q of
    // u (the state's newest input, rotated into place) and following the
    // survivor flips bit q by the stored word bit (decision XOR own bit q).
    // Decoded bits go to one LDS byte each, after the survivors.
    uint8_t *dbytes = (uint8_t *)(D.lds + nbody * REGS * 64);
    const int c = D.lane;
    int len = 0, t = 0, b_end = 0, pos = 0, q = 0, bdy = 0;
    uint32_t u = 0;
    if (c < C) {
      const int a_lo = (int)cs + c * f0;
      b_end = a_lo + f0 < (int)ce ? a_lo + f0 : (int)ce;
      const bool inner = c < n_inner;
      const int x = inner ? b_end + sa.w : (int)e;
      const int rel = x - 1 - (int)D.stage_base;
      bdy = rel / BODY;
      pos = rel - bdy * BODY;
      q = pos % P;
      if (!inner) {
        u = (uint32_t)lam;  // the block end is a body end: slot j holds state j
      } else if (sa.start == VIT_SUBFRAME_RANDOM) {
        const uint64_t z = splitmix64_at(sa.seed, ((uint64_t)sa.block << 32) | (uint64_t)c);
        const uint32_t st = (uint32_t)(z >> (65 - K));
        u = D.rotl_p(st, (pos + 1) % P);
      } else {
        u = snap_v;
      }
      t = x - 1;
      len = x - a_lo;
    }
    int maxlen = len;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      const int o = __shfl_xor(maxlen, m);
      maxlen = o > maxlen ? o : maxlen;
    }
    maxlen = __builtin_amdgcn_readfirstlane(maxlen);
    for (int i = 0; i < maxlen; ++i) {
      if (i < len) {
        if (t < b_end) dbytes[t - (int)cs] = (uint8_t)((u >> q) & 1u);
        const uint32_t wd = D.lds[(bdy * REGS + (int)(u >> 6)) * 64 + (int)(u & 63u)];
        u ^= ((wd >> (BODY - 1 - pos)) & 1u) << q;
        --t;
        q = q == 0 ? P - 1 : q - 1;
        if (--pos < 0) {
          pos = BODY - 1;
          --bdy;
        }
      }
    }
    // ---- output: lane-parallel packing of the decoded bytes (the wave's
    // LDS writes are complete before its reads).
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t b_lo = cs >> 3, b_hi = (ce - 1) >> 3;
    for (int64_t B = b_lo + D.lane; B <= b_hi; B += 64) {
      const int base = (int)(8 * B - cs);
      const int nv = (int)(ce - 8 * B) < 8 ? (int)(ce - 8 * B) : 8;
      uint32_t byte = 0;
      for (int j = 0; j < nv; ++j) byte |= (uint32_t)(dbytes[base + j] & 1u) << j;
      out[B] = (uint8_t)byte;
    }
    return;
  }

  // ---- traceback on the scalar unit (Decoder::tb_groups).  The decision bit
  // at offset g is the input bit of offset g - (k-1) (the oldest input of the
  // state), so the decision stream, followed by the k-1 bits of the upper
  // chain's start slot, is the decoded sequence shifted by k-1: bit t of the
  // output is stream bit (t - stage_base) + k - 1.
  // The traceback is a short serial chain of scalar steps: raise the wave's
  // issue priority while it runs so that waves in their forward pass do not
  // stretch it (measured: about 8% faster overall).
  const int grp_lo = ((int)(cs - s) + r) / BODY;
  __builtin_amdgcn_s_setprio(1);
  const uint32_t lam_start = (uint32_t)lam;
  {
    uint32_t u1[1] = {(uint32_t)lam};
    const bool w1[1] = {true};
    for (int grp = nbody - 1; grp >= grp_lo; --grp) {
      const int g1[1] = {grp};
      D.template tb_groups<1>(g1, u1, w1);
    }
  }
  __builtin_amdgcn_s_setprio(0);

  // ---- output: lane-parallel assembly of the core bits [cs, ce) into bytes.
  {
    const int64_t b_lo = cs >> 3, b_hi = (ce - 1) >> 3;
    const uint32_t body_mask = BODY == 32 ? 0xffffffffu : ((1u << BODY) - 1u);
    for (int64_t B = b_lo + D.lane; B <= b_hi; B += 64) {
      const int gbit = (int)(8 * B - D.stage_base) + P;  // stream index of the byte's bit 0
      const int wa_i = gbit / BODY, sh = gbit - wa_i * BODY;
      auto word = [&](int i) -> uint64_t {
        if (i < nbody) return D.lds[(i * REGS) * 64] & body_mask;
        return i == nbody ? lam_start : 0u;
      };
      const uint64_t cat = word(wa_i) | (word(wa_i + 1) << BODY);
      uint32_t byte = (uint32_t)(cat >> sh) & 0xffu;
      const int64_t nvalid = ce - 8 * B;
      if (nvalid < 8) byte &= (1u << nvalid) - 1u;
      out[B] = (uint8_t)byte;
    }
  }
}

// For 5 <= k <= 7 the one-trace instances are held to 64 VGPRs (eight waves
// per SIMD): left to itself the scheduler trades occupancy for deeper
// prefetch of branch metrics in some instances; the few scalar spills this
// costs are in the block prologue.  (The subframe instances would spill
// vector registers under the same bound.)
template <int K, int BETA, bool STD, int IN, bool SUB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(!SUB && K >= 5 && K <= 7 ? 8 : 1, 8))) void vit_blocked_kernel(DecodeArgs a, int lds_words_per_wave) {
  using Dec = Decoder<K, BETA, STD, IN>;
  using Sh = Shape<K, BETA>;
  constexpr int P = Sh::P, S = Sh::S, REGS = Sh::REGS, BODY = Sh::BODY, T = Sh::T;
  static_assert(BODY <= 32, "unrolled body longer than one decision dword");
  extern __shared__ uint32_t vit_lds[];

  Dec D;
  D.setup(a.gen);
  // wave index and count are uniform across the wave: keep them scalar
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int wpb = (int)(blockDim.x >> 6);
  D.lds = vit_lds + (size_t)wid * lds_words_per_wave;

  // Blocks per wave, mapped so that neighbouring blocks (which share LLR
  // overlap) run on the same XCD: workgroups are dealt round-robin to the 8
  // XCDs, so XCD x gets a contiguous range of blocks.
  const int64_t nwaves = (int64_t)gridDim.x * wpb;
  int64_t first, stride, last;
  if ((gridDim.x & 7) == 0 && a.nblocks >= nwaves) {
    const int xcd = blockIdx.x & 7;
    const int64_t wx = (int64_t)(blockIdx.x >> 3) * wpb + wid;
    const int64_t per = (a.nblocks + 7) / 8;
    first = (int64_t)xcd * per + wx;
    last = (int64_t)(xcd + 1) * per;
    if (last > a.nblocks) last = a.nblocks;
    stride = nwaves / 8;
  } else {
    first = (int64_t)blockIdx.x * wpb + wid;
    last = a.nblocks;
    stride = nwaves;
  }

  for (int64_t blk = first; blk < last; blk += stride) {
    const int64_t cs = blk * a.L;
    const int64_t ce = (cs + a.L < a.n) ? cs + a.L : a.n;
    const int64_t s = (cs - a.v1 > 0) ? cs - a.v1 : 0;
    const int64_t e = (ce + a.v2 < a.N) ? ce + a.v2 : a.N;
    const SubframeArgs sa{a.sub_bits, a.sub_overlap, a.sub_start, a.sub_seed, blk};
    decode_block<SUB>(D, a.llr, a.out, s, e, cs, ce, s == 0, a.terminated && (e == a.N), sa, a.gen);
  }
}

// Batched decode: persistent waves walk the work list (one block of one frame
// per item, sorted by cost on the host, longest first) with a static stride:
// wave w takes items w, w + W, w + 2W, ... for W waves in the grid.  Each
// wave gets one item of every round of W, so with costs sorted the waves'
// totals differ by at most one block; no atomics are needed (a single
// device-wide counter serialises).  The item count and the offset of the
// code's run live in the workspace header.  For standard codes up to k = 7
// the register budget is held to 64 VGPRs (eight waves per SIMD, as the
// stream kernel).
template <int K, int BETA, bool STD, int IN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(STD && K <= 7 ? 8 : 1, 8))) void vit_batch_kernel(BatchArgs a, int lds_words_per_wave) {
  using Dec = Decoder<K, BETA, STD, IN>;
  extern __shared__ uint32_t vit_lds[];
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int wpb = (int)(blockDim.x >> 6);
  const int nitems = __builtin_amdgcn_readfirstlane(a.header[kMaxCodes + a.code_index]);
  // waves without an item leave before any setup (fixed grids larger than
  // the work list are cheap)
  if ((int)blockIdx.x * wpb + wid >= nitems) return;
  Dec D;
  D.setup(a.gen);
  D.lds = vit_lds + (size_t)wid * lds_words_per_wave;
  const WorkItem *items = a.items + a.header[2 * kMaxCodes + a.code_index];
  const int nwaves = (int)gridDim.x * wpb;
  for (int idx = (int)blockIdx.x * wpb + wid; idx < nitems; idx += nwaves) {
    const WorkItem it = items[idx];
    const char *base = (const char *)a.llr + it.llr_off;
    const SubframeArgs none{0, 0, 0, 0, 0};
    decode_block<false>(D, (const void *)base, a.out + it.out_off, it.s, it.e, it.cs, it.ce, (it.flags & 1) != 0,
                        (it.flags & 2) != 0, none, a.gen);
  }
}

#undef VIT_SNAP
#undef VIT_G1
#undef VIT_U1
#undef VIT_X8
#undef VIT_X32

}  // namespace dev

typedef void (*KernelFn)(DecodeArgs, int);
typedef void (*BatchKernelFn)(BatchArgs, int);

// Kernel instance for (K, beta, standard code, input kind, subframe traceback).
template <int K, bool SUB>
KernelFn pick_kernel_k(int beta, bool stdc, int in) {
  auto pick = [&](auto bt) -> KernelFn {
    constexpr int B = decltype(bt)::value;
    if (stdc) {
      if (in == VIT_LLR_HARD) return dev::vit_blocked_kernel<K, B, true, VIT_LLR_HARD, SUB>;
      return in == VIT_LLR_I8 ? dev::vit_blocked_kernel<K, B, true, VIT_LLR_I8, SUB>
                              : dev::vit_blocked_kernel<K, B, true, VIT_LLR_F32, SUB>;
    }
    if (in == VIT_LLR_HARD) return dev::vit_blocked_kernel<K, B, false, VIT_LLR_HARD, SUB>;
    return in == VIT_LLR_I8 ? dev::vit_blocked_kernel<K, B, false, VIT_LLR_I8, SUB>
                            : dev::vit_blocked_kernel<K, B, false, VIT_LLR_F32, SUB>;
  };
  switch (beta) {
    case 2: return pick(std::integral_constant<int, 2>{});
    case 3: return pick(std::integral_constant<int, 3>{});
    case 4: return pick(std::integral_constant<int, 4>{});
  }
  return nullptr;
}

template <int K>
BatchKernelFn pick_batch_kernel_k(int beta, bool stdc, int in) {
  auto pick = [&](auto bt) -> BatchKernelFn {
    constexpr int B = decltype(bt)::value;
    if (stdc) {
      if (in == VIT_LLR_HARD) return dev::vit_batch_kernel<K, B, true, VIT_LLR_HARD>;
      return in == VIT_LLR_I8 ? dev::vit_batch_kernel<K, B, true, VIT_LLR_I8> : dev::vit_batch_kernel<K, B, true, VIT_LLR_F32>;
    }
    if (in == VIT_LLR_HARD) return dev::vit_batch_kernel<K, B, false, VIT_LLR_HARD>;
    return in == VIT_LLR_I8 ? dev::vit_batch_kernel<K, B, false, VIT_LLR_I8> : dev::vit_batch_kernel<K, B, false, VIT_LLR_F32>;
  };
  switch (beta) {
    case 2: return pick(std::integral_constant<int, 2>{});
    case 3: return pick(std::integral_constant<int, 3>{});
    case 4: return pick(std::integral_constant<int, 4>{});
  }
  return nullptr;
}

KernelFn pick_kernel_k3(int beta, bool stdc, int in);
KernelFn pick_kernel_sub_k3(int beta, bool stdc, int in);
KernelFn pick_kernel_k4(int beta, bool stdc, int in);
KernelFn pick_kernel_sub_k4(int beta, bool stdc, int in);
KernelFn pick_kernel_k5(int beta, bool stdc, int in);
KernelFn pick_kernel_sub_k5(int beta, bool stdc, int in);
KernelFn pick_kernel_k6(int beta, bool stdc, int in);
KernelFn pick_kernel_sub_k6(int beta, bool stdc, int in);
KernelFn pick_kernel_k7(int beta, bool stdc, int in);
KernelFn pick_kernel_sub_k7(int beta, bool stdc, int in);
KernelFn pick_kernel_k8(int beta, bool stdc, int in);
KernelFn pick_kernel_sub_k8(int beta, bool stdc, int in);
KernelFn pick_kernel_k9(int beta, bool stdc, int in);
KernelFn pick_kernel_sub_k9(int beta, bool stdc, int in);
BatchKernelFn pick_batch_kernel_k3(int beta, bool stdc, int in);
BatchKernelFn pick_batch_kernel_k4(int beta, bool stdc, int in);
BatchKernelFn pick_batch_kernel_k5(int beta, bool stdc, int in);
BatchKernelFn pick_batch_kernel_k6(int beta, bool stdc, int in);
BatchKernelFn pick_batch_kernel_k7(int beta, bool stdc, int in);
BatchKernelFn pick_batch_kernel_k8(int beta, bool stdc, int in);
BatchKernelFn pick_batch_kernel_k9(int beta, bool stdc, int in);

}  // namespace vit
