// vit_decoder16.h -- integer decoder with 16-bit path metrics kept modulo
// 2^16, for int8 and hard-decision inputs on gfx950: device templates,
// instantiated per constraint length in vit_kernels16_k*.hip.
//
// The trellis layout is that of vit_decoder.h (rotating state slots: slot j
// holds state rotr^m(j) after m stages, so each stage pairs the two
// predecessors of a butterfly across slot bit q = m mod (k-1); slot bits 0..5
// are lane xors 1, 2, 7, 8, 16, 32, higher bits are registers).  What differs:
//
//  * Two blocks per wave.  Every metric register holds the metrics of one
//    slot for two blocks, the low 16 bits for one and the high 16 bits for
//    the other, so one exchange (DPP move or in-place v_permlane*_swap) and one
//    packed operation serve both.
//  * Modulo arithmetic (eq. 3 in 16 bits).  Sums wrap; a candidate beats
//    another when their wrapped difference is negative or positive, which is
//    the exact decision while every compared difference stays below 2^15 in
//    magnitude: the spread of a block's metrics is at most (k-1)*2*128*beta
//    (every state is reached from any state k-1 stages earlier), and states
//    unreachable from a known start begin 2^14 below state 0.  No
//    normalisation is ever needed.
//  * Tie rule by a bias.  In a slot whose own predecessor is odd (slot bit q
//    set), the partner (the even predecessor) must also win a tie.  The own
//    candidate of such a slot is formed with its branch metric less one, so
//    "partner wins" is the sign bit of own - partner in every slot, and the
//    survivor is own - min(own - partner, -e) for e = 0 or 1 (exact in both
//    cases).  The branch-metric table holds each pattern's metric twice,
//    plain and less one, so the bias costs no instruction.
//  * Per stage and register (two blocks x one slot): 2 packed adds, 1 packed
//    sub, 1 packed min, 1 packed sub, the exchange, and a shift + bit-field
//    insert that moves the two decision bits (bits 15 and 31 of the
//    difference) into the decision word.  The stored bit is "partner wins",
//    which is the decision XOR the slot's own bit q: following it flips bit q
//    of the traceback's slot index, as in vit_decoder.h.
//  * Survivor words hold 16 stages per block (low half / high half of a
//    dword), so an unrolled body is the largest even multiple of k-1 up to 16
//    stages.
//  * Blocks of different lengths share a wave: both end at the last stage of
//    the last body; the shorter one starts later and its half of the metric
//    registers is reset to its initial metrics at its first stage.
#pragma once

#include "vit_internal.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vit {
namespace dev16 {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_u(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as_w(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) { return as_w(as_u(a) + as_u(b)); }
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b) { return as_w(as_u(a) - as_u(b)); }
__device__ __forceinline__ uint32_t pk_min_i16(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t,
                            __builtin_elementwise_min(__builtin_bit_cast(i16x2, a), __builtin_bit_cast(i16x2, b)));
}

// Largest d <= cap dividing n with n / d even.
constexpr int even_split_divisor(int n, int cap) {
  int best = 1;
  for (int d = 1; d <= cap; ++d)
    if (n % d == 0 && (n / d) % 2 == 0) best = d;
  return best;
}
// Largest even multiple of p that is at most 16.
constexpr int body16(int p) {
  int b = p * (16 / p);
  return (b % 2 == 0) ? b : b - p;
}

template <int K, int BETA>
struct Shape16 {
  static constexpr int P = K - 1;
  static constexpr int S = 1 << P;
  static constexpr int REGS = S > 64 ? S / 64 : 1;
  static constexpr int NCODE = 1 << BETA;
  static constexpr int NENT = 2 * NCODE;  // table entries per stage: each pattern plain and less one
  static constexpr int BODY = body16(P);
  static constexpr int T = even_split_divisor(BODY, 64 / NENT);
};

__device__ __forceinline__ int parity32(uint32_t x) { return __builtin_popcount(x) & 1; }

// Partner metric across slot bit q (q < 6), both halves at once.
template <int Q>
__device__ __forceinline__ uint32_t exchange(uint32_t o) {
  if constexpr (Q == 0) return (uint32_t)__builtin_amdgcn_mov_dpp((int)o, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  else if constexpr (Q == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)o, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  else if constexpr (Q == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)o, 0x141, 0xF, 0xF, false);  // row_half_mirror
  else if constexpr (Q == 3) return (uint32_t)__builtin_amdgcn_mov_dpp((int)o, 0x128, 0xF, 0xF, false);  // row_ror:8
  else if constexpr (Q == 4) {
    // lane xor 16: v_permlane16_swap with both operands the same register
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %0" : "+v"(o));
    return o;
  } else {
    asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %0" : "+v"(o));
    return o;
  }
}

// IN: VIT_LLR_I8 (int8 LLRs) or VIT_LLR_HARD (hard-decision bytes).
template <int K, int BETA, int IN>
struct Decoder16 {
  using Sh = Shape16<K, BETA>;
  static constexpr int P = Sh::P, S = Sh::S, REGS = Sh::REGS, NCODE = Sh::NCODE, NENT = Sh::NENT, T = Sh::T,
                       BODY = Sh::BODY;
  static constexpr int QL = P < 6 ? P : 6;  // phases whose slot bit is a lane bit
  static constexpr uint32_t kUnreached = 0xC000u;  // -2^14: start metric of states other than 0

  // per-lane constants (depend only on the code)
  int addr_x[P][REGS];  // byte offset within a stage's table entries: partner branch, plain
  int addr_y[P][REGS];  // own branch, less e (e = own predecessor odd)
  uint32_t ce[QL];      // -e for the lane phases, both halves
  uint32_t ssign;       // byte b: +1 or -1 (int8), the sign of LLR b in this lane's table pattern
  int tbias;            // 0 or 1: this lane's table entry is "less one"
  uint32_t init_known[REGS];  // start metrics of a known start (state 0 at 0), both halves
  int tl;               // stage of this lane's table entry within a tile
  int lane;
  int slot0;

  // per-pair state
  uint32_t o[REGS];
  uint32_t dec[REGS];
  uint32_t xn[REGS], yn[REGS];
  int table;
  uint32_t nxt[2][2];   // [tile buffer][half]: byte b = LLR b of this lane's stage
  const uint8_t *llr[2];
  int tile_stage0[2];   // per half: stage of body offset 0 + this lane's table row
  int s_lo[2], s_hi[2];
  uint32_t *lds;
  int body;

  __device__ __forceinline__ int metric_addr(const uint32_t *gen, int q, int reg, bool own) const {
    const int st = ((reg << 6) | slot0) & (S - 1);
    const int up = (st >> q) & 1;
    const uint32_t iown = (uint32_t)(((st >> q) | (st << (P - q))) & (S - 1));
    const uint32_t rown = ((uint32_t)up << (K - 1)) | iown;
    const uint32_t rb = own ? rown : (rown ^ 1u);
    int c = 0;
#pragma unroll
    for (int b = 0; b < BETA; ++b) c |= parity32(gen[b] & rb) << b;
    const int bias = own ? up : 0;
    return (bias * NCODE + c) << 2;
  }

  __device__ __forceinline__ void setup(const uint32_t *gen) {
    lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    slot0 = lane ^ (((lane >> 2) & 1) ? 3 : 0);  // inverse of the lane xor map
    tl = lane / NENT;
    const int ent = lane % NENT;
    const int pat = ent % NCODE;
    tbias = (ent >= NCODE) ? 1 : 0;
    ssign = 0;
#pragma unroll
    for (int b = 0; b < BETA; ++b) ssign |= (((pat >> b) & 1) ? 0xFFu : 0x01u) << (8 * b);
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int reg = 0; reg < REGS; ++reg) {
        addr_x[q][reg] = metric_addr(gen, q, reg, false);
        addr_y[q][reg] = metric_addr(gen, q, reg, true);
      }
#pragma unroll
    for (int q = 0; q < QL; ++q) ce[q] = ((slot0 >> q) & 1) ? 0xFFFFFFFFu : 0u;
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      const int st = ((reg << 6) | slot0) & (S - 1);
      init_known[reg] = st == 0 ? 0u : (kUnreached | (kUnreached << 16));
    }
  }

  // LLR bytes of tile tau for both halves, the stage clamped into each
  // block's window (every lane reads inside its block).
  __device__ __forceinline__ uint32_t tile_word(int h, int tau) const {
    const int raw = tile_stage0[h] + tau * T;
    int stc;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(stc) : "v"(raw), "v"(s_lo[h]), "v"(s_hi[h]));
    const uint8_t *p = llr[h] + (uint32_t)stc * (uint32_t)BETA;
    uint32_t w = 0;
#pragma unroll
    for (int b = 0; b < BETA; ++b) w |= (uint32_t)p[b] << (8 * b);
    return w;
  }
  template <int BUF>
  __device__ __forceinline__ void load_tile(int tau) {
#pragma unroll
    for (int h = 0; h < 2; ++h) nxt[BUF][h] = tile_word(h, tau);
  }
  // Same, with the buffer chosen at run time (block prologue only): value
  // selects, so that the buffers stay in registers.
  __device__ __forceinline__ void load_tile_rt(int tau) {
    const bool odd = (tau & 1) != 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t w = tile_word(h, tau);
      nxt[0][h] = odd ? nxt[0][h] : w;
      nxt[1][h] = odd ? w : nxt[1][h];
    }
  }

  // Hard decisions: byte 0 (coded bit 0) -> +1, any other value -> -1.
  __device__ __forceinline__ static uint32_t hard_to_pm1(uint32_t w) {
    uint32_t t = w | ((w >> 4) & 0x0F0F0F0Fu);
    t |= (t >> 2) & 0x33333333u;
    t |= (t >> 1) & 0x55555555u;
    return 0x01010101u + (t & 0x01010101u) * 0xFEu;  // per byte: 0x01 or 0xFF
  }

  // eq. (2) for this lane's pattern in both halves, less the lane's table
  // bias: the dot product of the LLR bytes with the pattern's signs, exact
  // (|sum| <= 512), packed low half / high half.
  template <int BUF>
  __device__ __forceinline__ void build_table() {
    int d[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t w = nxt[BUF][h];
      if constexpr (IN == VIT_LLR_HARD) w = hard_to_pm1(w);
      d[h] = __builtin_amdgcn_sdot4((int)w, (int)ssign, -tbias, false);
    }
    table = (int)__builtin_amdgcn_perm((uint32_t)d[1], (uint32_t)d[0], 0x05040100u);
  }
  __device__ __forceinline__ void build_table_rt(int tau) {
    const bool odd = (tau & 1) != 0;
    const uint32_t keep0 = nxt[0][0], keep1 = nxt[0][1];
    nxt[0][0] = odd ? nxt[1][0] : keep0;
    nxt[0][1] = odd ? nxt[1][1] : keep1;
    build_table<0>();
    nxt[0][0] = keep0;
    nxt[0][1] = keep1;
  }

  __device__ __forceinline__ void refresh_addresses() {
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int reg = 0; reg < REGS; ++reg) {
        asm volatile("" : "+v"(addr_x[q][reg]));
        asm volatile("" : "+v"(addr_y[q][reg]));
      }
  }

  __device__ __forceinline__ uint32_t fetch(int addr, int tlc) const {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(addr + tlc * NENT * 4, table);
  }

  template <int G>
  __device__ __forceinline__ void fetch_step(uint32_t (&x)[REGS], uint32_t (&y)[REGS]) const {
    constexpr int q = G % P;
    constexpr int tlc = G % T;
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      x[reg] = fetch(addr_x[q][reg], tlc);
      y[reg] = fetch(addr_y[q][reg], tlc);
    }
  }

  __device__ __forceinline__ void fetch_entry(const uint32_t *gen, int g, uint32_t (&x)[REGS],
                                              uint32_t (&y)[REGS]) const {
    const int q = g % P, tlc = g % T;
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      x[reg] = fetch(metric_addr(gen, q, reg, false), tlc);
      y[reg] = fetch(metric_addr(gen, q, reg, true), tlc);
    }
  }

  // Shift the two decision bits (bits 15 and 31 of z) into the word: the
  // latest stage sits at bits 15 / 31.  Written out so that the compiler
  // keeps the two-instruction form.
  __device__ __forceinline__ static uint32_t push_decision(uint32_t d, uint32_t z) {
    asm("v_lshrrev_b32 %0, 1, %0\n\tv_bfi_b32 %0, %2, %1, %0" : "+v"(d) : "v"(z), "s"(0x80008000u));
    return d;
  }

  template <int Q>
  __device__ __forceinline__ void acs_lane(int reg, uint32_t x, uint32_t y) {
    const uint32_t B = pk_add(o[reg], y);       // own candidate (less e)
    const uint32_t p = exchange<Q>(o[reg]);     // partner metric
    const uint32_t A = pk_add(p, x);            // partner candidate
    const uint32_t z = pk_sub(B, A);            // sign: partner wins
    o[reg] = pk_sub(B, pk_min_i16(z, ce[Q]));   // the larger candidate, exactly
    dec[reg] = push_decision(dec[reg], z);
  }

  // Slot bit q >= 6: both predecessors in this lane, registers ra (own
  // predecessor even, e = 0) and rb (odd, e = 1).
  __device__ __forceinline__ void acs_pair(int ra, int rb, uint32_t xa, uint32_t xb, uint32_t ya, uint32_t yb) {
    const uint32_t oa = o[ra], ob = o[rb];
    const uint32_t Ba = pk_add(oa, ya), Aa = pk_add(ob, xa);
    const uint32_t Bb = pk_add(ob, yb), Ab = pk_add(oa, xb);
    const uint32_t za = pk_sub(Ba, Aa), zb = pk_sub(Bb, Ab);
    o[ra] = pk_sub(Ba, pk_min_i16(za, 0u));
    o[rb] = pk_sub(Bb, pk_min_i16(zb, 0xFFFFFFFFu));
    dec[ra] = push_decision(dec[ra], za);
    dec[rb] = push_decision(dec[rb], zb);
  }

  // One trellis stage at body offset G; same software pipeline as
  // vit_decoder.h (branch metrics one step ahead, LLRs two tiles ahead).
  template <int G>
  __device__ __forceinline__ void step() {
    constexpr int q = G % P;
    constexpr int tlc = G % T;
    uint32_t x[REGS], y[REGS];
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
      for (int reg = 0; reg < REGS; ++reg) acs_lane<q < 6 ? q : 0>(reg, x[reg], y[reg]);
    } else {
      constexpr int bit = 1 << (q - 6);
#pragma unroll
      for (int ra = 0; ra < REGS; ++ra)
        if ((ra & bit) == 0) acs_pair(ra, ra | bit, x[ra], x[ra | bit], y[ra], y[ra | bit]);
    }
    if constexpr (G == BODY - 1) {
#pragma unroll
      for (int reg = 0; reg < REGS; ++reg) lds[(body * REGS + reg) * 64 + slot0] = dec[reg];
    }
  }

  // Reset half h of the metrics to a block's start metrics.
  __device__ __forceinline__ void reinit(int h, bool known) {
    const uint32_t m = h ? 0xFFFF0000u : 0x0000FFFFu;
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      const uint32_t v = known ? init_known[reg] : 0u;
      o[reg] = (v & m) | (o[reg] & ~m);
    }
  }

  // Best state of half h at a body end (slot j holds state j): the largest
  // metric, lowest index on ties, compared through wrapped differences to
  // state 0's metric (lane 0, register 0).  Uniform across the wave.
  __device__ __forceinline__ int best_state(int h) const {
    const int sh = 16 * h;
    const int ref = (int)(short)(uint16_t)((uint32_t)__builtin_amdgcn_readfirstlane((int)o[0]) >> sh);
    int key = -1;
#pragma unroll
    for (int reg = 0; reg < REGS; ++reg) {
      const int label = ((reg << 6) | slot0) & (S - 1);
      const int m = (int)(short)(uint16_t)(o[reg] >> sh);
      const int d = (int)(short)(uint16_t)(uint32_t)(m - ref);  // wrapped difference, exact
      const int kk = ((d + 32768) << 8) | (255 - label);
      key = kk > key ? kk : key;
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      const int ok = __shfl_xor(key, m);
      key = ok > key ? ok : key;
    }
    return 255 - (__builtin_amdgcn_readfirstlane(key) & 255);
  }

  // Traceback (Algorithm 2) through one body of survivor words for NCH
  // chains (each a half of the pair), interleaved.  Chain c reads half
  // hh[c]; ulam[c] is its slot index.  Stage p0 + q of the body sits at bit
  // 16 - BODY + p0 + q of the half: per phase period the half is shifted so
  // that stage p0 + q is bit q, and a step is one v_readlane, one s_and and
  // one s_xor.  After a period the slot index holds that period's states'
  // inputs; the body's decoded bits replace the half of slot 0's word when
  // wr[c] (a chain never reads a body again once it has passed it, and the
  // other half belongs to the other chain).
  template <int NCH>
  __device__ __forceinline__ void tb_groups(const int (&grp)[NCH], const int (&hh)[NCH], uint32_t (&ulam)[NCH],
                                            const bool (&wr)[NCH]) const {
    uint32_t dv[NCH][REGS];
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int rr = 0; rr < REGS; ++rr) dv[c][rr] = lds[(grp[c] * REGS + rr) * 64 + lane] >> (16 * hh[c]);
    uint32_t acc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = 0;
#pragma unroll
    for (int p0 = BODY - P; p0 >= 0; p0 -= P) {
      uint32_t sh[NCH][REGS], src[NCH];
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
#pragma unroll
        for (int rr = 0; rr < REGS; ++rr) sh[c][rr] = dv[c][rr] >> (16 - BODY + p0);
        src[c] = sh[c][0];
      }
#pragma unroll
      for (int q = P - 1; q >= 0; --q) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          if constexpr (REGS > 1) {
            if (q >= 5) src[c] = select_reg16(sh[c], ulam[c] >> 6);
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
      if (wr[c]) ((uint16_t *)lds)[2 * (grp[c] * REGS * 64) + hh[c]] = (uint16_t)acc[c];
  }

  __device__ __forceinline__ static uint32_t select_reg16(const uint32_t (&v)[REGS], uint32_t rsel) {
    typedef uint32_t vec_t __attribute__((ext_vector_type(REGS)));
    vec_t t;
#pragma unroll
    for (int i = 0; i < REGS; ++i) t[i] = v[i];
    return t[rsel & (REGS - 1)];
  }
};

// One block of a pair.
struct Blk16 {
  const uint8_t *llr;  // the frame's stage 0
  uint8_t *out;       // the frame's decoded byte 0
  int64_t s, e, cs, ce;
  bool start_known, end_zero, emit;
};

#define VIT16_G(NN, M)                                        \
  if constexpr ((NN) < (M)) {                                 \
    if ((NN) >= rr) {                                         \
      if ((NN) == ry) D.reinit(hy, known_y);                  \
      D.template step<(NN)>();                                \
    }                                                         \
  }
#define VIT16_U(NN, M) \
  if constexpr ((NN) < (M)) D.template step<(NN)>();
#define VIT16_X8(X, B, M)                                                                \
  X(B + 0, M) X(B + 1, M) X(B + 2, M) X(B + 3, M) X(B + 4, M) X(B + 5, M) X(B + 6, M)   \
  X(B + 7, M)
#define VIT16_X16(X, M) VIT16_X8(X, 0, M) VIT16_X8(X, 8, M)

// Decode two blocks (Sec. III windows), one per half of the metric
// registers.  A block with emit = false is decoded but writes nothing.  The
// caller guarantees (e - s) * beta < 2^31 and cs a multiple of 8.
template <int K, int BETA, int IN>
__device__ __forceinline__ void decode_pair(Decoder16<K, BETA, IN> &D, const Blk16 (&b)[2], const uint32_t *gen) {
  using Sh = Shape16<K, BETA>;
  constexpr int P = Sh::P, S = Sh::S, REGS = Sh::REGS, BODY = Sh::BODY, T = Sh::T;
  const int M0 = (int)(b[0].e - b[0].s), M1 = (int)(b[1].e - b[1].s);
  const int M = M0 > M1 ? M0 : M1;
  const int r = (BODY - M % BODY) % BODY;
  const int nbody = (M + r) / BODY;
  // body offset of each block's first stage: both end at the last body's end
  const int g0 = r + M - M0, g1 = r + M - M1;
  int stage_base[2];
  stage_base[0] = (int)b[0].s - g0;
  stage_base[1] = (int)b[1].s - g1;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    D.llr[h] = b[h].llr;
    D.tile_stage0[h] = stage_base[h] + D.tl;
    D.s_lo[h] = (int)b[h].s;
    D.s_hi[h] = (int)b[h].e - 1;
  }
  // the later-starting half (if any) is reset at its first stage
  const int hy = g1 > g0 ? 1 : 0;
  const int gy = hy ? g1 : g0;
  const bool known_y = hy ? b[1].start_known : b[0].start_known;
  const int body_y = gy > r ? gy / BODY : -1;
  const int off_y = gy % BODY;
#pragma unroll
  for (int reg = 0; reg < REGS; ++reg) {
    const uint32_t i0 = b[0].start_known ? D.init_known[reg] : 0u;
    const uint32_t i1 = b[1].start_known ? D.init_known[reg] : 0u;
    D.o[reg] = (i0 & 0xFFFFu) | (i1 & 0xFFFF0000u);
    D.dec[reg] = 0u;
  }
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
  {
    const int rr = r;
    const int ry = body_y == 0 ? off_y : -1;
    VIT16_X16(VIT16_G, BODY)
  }
  for (D.body = 1; D.body < nbody; ++D.body) {
    D.refresh_addresses();
    if (D.body == body_y) {
      const int rr = 0;
      const int ry = off_y;
      VIT16_X16(VIT16_G, BODY)
    } else {
      VIT16_X16(VIT16_U, BODY)
    }
  }

  // traceback start per half: state 0 at a terminated end, else the best state
  uint32_t lam[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) lam[h] = b[h].end_zero ? 0u : (uint32_t)D.best_state(h);
  int grp_lo[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) grp_lo[h] = (int)(b[h].cs - stage_base[h]) / BODY;

  __builtin_amdgcn_s_setprio(1);
  {
    // both chains from the last body down, together while both run, then the
    // one with more bodies alone
    const int len0 = nbody - grp_lo[0], len1 = nbody - grp_lo[1];
    const int both = len0 < len1 ? len0 : len1;
    uint32_t u2[2] = {lam[0], lam[1]};
    const int h2[2] = {0, 1};
    const bool w2[2] = {true, true};
    for (int i = 0; i < both; ++i) {
      const int g2[2] = {nbody - 1 - i, nbody - 1 - i};
      D.template tb_groups<2>(g2, h2, u2, w2);
    }
    const int hl = len0 > len1 ? 0 : 1;
    const int lenl = hl ? len1 : len0;
    uint32_t u1[1] = {hl ? u2[1] : u2[0]};
    const int h1[1] = {hl};
    const bool w1[1] = {true};
    for (int i = both; i < lenl; ++i) {
      const int g1[1] = {nbody - 1 - i};
      D.template tb_groups<1>(g1, h1, u1, w1);
    }
  }
  __builtin_amdgcn_s_setprio(0);

  // output: lane-parallel assembly of each block's core bits into bytes
  constexpr uint32_t body_mask = (1u << BODY) - 1u;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (!b[h].emit) continue;
    const int64_t b_lo = b[h].cs >> 3, b_hi = (b[h].ce - 1) >> 3;
    for (int64_t B = b_lo + D.lane; B <= b_hi; B += 64) {
      const int gbit = (int)(8 * B - stage_base[h]) + P;  // stream index of the byte's bit 0
      const int wa_i = gbit / BODY, sh = gbit - wa_i * BODY;
      auto word = [&](int i) -> uint64_t {
        if (i < nbody) return (D.lds[(i * REGS) * 64] >> (16 * h)) & body_mask;
        return i == nbody ? lam[h] : 0u;
      };
      const uint64_t cat = word(wa_i) | (word(wa_i + 1) << BODY);
      uint32_t byte = (uint32_t)(cat >> sh) & 0xffu;
      const int64_t nvalid = b[h].ce - 8 * B;
      if (nvalid < 8) byte &= (1u << nvalid) - 1u;
      b[h].out[B] = (uint8_t)byte;
    }
  }
  (void)S;
}

// Stream kernel: wave w decodes blocks 2p and 2p+1 for its pairs p (a last
// odd block is decoded in both halves and emitted once), pairs dealt so that
// each XCD gets a contiguous range.
template <int K, int BETA, int IN>
__global__ __launch_bounds__(256) void vit_blocked16_kernel(DecodeArgs a, int lds_words_per_wave) {
  using Dec = Decoder16<K, BETA, IN>;
  extern __shared__ uint32_t vit_lds16[];
  Dec D;
  D.setup(a.gen);
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int wpb = (int)(blockDim.x >> 6);
  D.lds = vit_lds16 + (size_t)wid * lds_words_per_wave;
  const int64_t npairs = (a.nblocks + 1) / 2;
  const int64_t nwaves = (int64_t)gridDim.x * wpb;
  int64_t first, stride, last;
  if ((gridDim.x & 7) == 0 && npairs >= nwaves) {
    const int xcd = blockIdx.x & 7;
    const int64_t wx = (int64_t)(blockIdx.x >> 3) * wpb + wid;
    const int64_t per = (npairs + 7) / 8;
    first = (int64_t)xcd * per + wx;
    last = (int64_t)(xcd + 1) * per;
    if (last > npairs) last = npairs;
    stride = nwaves / 8;
  } else {
    first = (int64_t)blockIdx.x * wpb + wid;
    last = npairs;
    stride = nwaves;
  }
  for (int64_t p = first; p < last; p += stride) {
    Blk16 bb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int64_t blk = 2 * p + h;
      const bool emit = blk < a.nblocks;
      if (!emit) blk = 2 * p;
      const int64_t cs = blk * a.L;
      const int64_t ce = (cs + a.L < a.n) ? cs + a.L : a.n;
      const int64_t s = (cs - a.v1 > 0) ? cs - a.v1 : 0;
      const int64_t e = (ce + a.v2 < a.N) ? ce + a.v2 : a.N;
      bb[h] = Blk16{(const uint8_t *)a.llr, a.out, s, e, cs, ce, s == 0, a.terminated && (e == a.N), emit};
    }
    decode_pair(D, bb, a.gen);
  }
}

// Batch kernel: the code's work items (sorted by cost, longest first) in
// pairs 2i, 2i+1; wave w takes pairs w, w + W, ... (static stride).
template <int K, int BETA, int IN>
__global__ __launch_bounds__(256) void vit_batch16_kernel(BatchArgs a, int lds_words_per_wave) {
  using Dec = Decoder16<K, BETA, IN>;
  extern __shared__ uint32_t vit_lds16[];
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int wpb = (int)(blockDim.x >> 6);
  const int nitems = __builtin_amdgcn_readfirstlane(a.header[kMaxCodes + a.code_index]);
  const int npairs = (nitems + 1) / 2;
  // waves without a pair leave before any setup
  if ((int)blockIdx.x * wpb + wid >= npairs) return;
  Dec D;
  D.setup(a.gen);
  D.lds = vit_lds16 + (size_t)wid * lds_words_per_wave;
  const WorkItem *items = a.items + a.header[2 * kMaxCodes + a.code_index];
  const int nwaves = (int)gridDim.x * wpb;
  for (int p = (int)blockIdx.x * wpb + wid; p < npairs; p += nwaves) {
    Blk16 bb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int idx = 2 * p + h;
      const bool emit = idx < nitems;
      if (!emit) idx = 2 * p;
      const WorkItem it = items[idx];
      bb[h] = Blk16{(const uint8_t *)a.llr + it.llr_off, a.out + it.out_off, it.s, it.e, it.cs, it.ce,
                    (it.flags & 1) != 0, (it.flags & 2) != 0, emit};
    }
    decode_pair(D, bb, a.gen);
  }
}

#undef VIT16_G
#undef VIT16_U
#undef VIT16_X8
#undef VIT16_X16

}  // namespace dev16

typedef void (*KernelFn16)(DecodeArgs, int);
typedef void (*BatchKernelFn16)(BatchArgs, int);

// Kernel instances for (K, beta, input kind VIT_LLR_I8 / VIT_LLR_HARD).
template <int K>
void *pick_kernel16_k(int beta, int in, bool batch) {
  auto pick = [&](auto bt) -> void * {
    constexpr int B = decltype(bt)::value;
    if (batch)
      return in == VIT_LLR_HARD ? (void *)dev16::vit_batch16_kernel<K, B, VIT_LLR_HARD>
                                : (void *)dev16::vit_batch16_kernel<K, B, VIT_LLR_I8>;
    return in == VIT_LLR_HARD ? (void *)dev16::vit_blocked16_kernel<K, B, VIT_LLR_HARD>
                              : (void *)dev16::vit_blocked16_kernel<K, B, VIT_LLR_I8>;
  };
  switch (beta) {
    case 2: return pick(std::integral_constant<int, 2>{});
    case 3: return pick(std::integral_constant<int, 3>{});
    case 4: return pick(std::integral_constant<int, 4>{});
  }
  return nullptr;
}

void *pick_kernel16_k3(int beta, int in, bool batch);
void *pick_kernel16_k4(int beta, int in, bool batch);
void *pick_kernel16_k5(int beta, int in, bool batch);
void *pick_kernel16_k6(int beta, int in, bool batch);
void *pick_kernel16_k7(int beta, int in, bool batch);
void *pick_kernel16_k8(int beta, int in, bool batch);
void *pick_kernel16_k9(int beta, int in, bool batch);

}  // namespace vit
