// Issue cost of single VALU instruction forms on gfx950: every wave runs six
// independent chains of one instruction form, at eight waves per SIMD, and
// the kernel time gives cycles per wave64 instruction per SIMD.  Timing only:
// the values computed are meaningless; one store per thread keeps them live.
// Build and run (one MI355X):
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         tests/microbench/valu_issue_rates.hip -o /tmp/valu_issue_rates && /tmp/valu_issue_rates
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdint.h>

#define R6(X) X X X X X X
template <int V>
__global__ __launch_bounds__(256) void mb(float *out, int iters) {
  float a = threadIdx.x, b = 1.0f, c = 2.0f, d = 3.0f, e = 4.0f, f = 5.0f, s = 1.0f, t = 0.5f;
  uint32_t u0 = threadIdx.x, u1 = 1, u2 = 2, u3 = 3, u4 = 4, u5 = 5;
  uint64_t m = 0;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#define OP6(INS) asm volatile(INS(a) INS(b) INS(c) INS(d) INS(e) INS(f) : [a] "+v"(a), [b] "+v"(b), [c] "+v"(c), [d] "+v"(d), [e] "+v"(e), [f] "+v"(f) : [s] "v"(s), [t] "v"(t) : "vcc");
#define ADD(X) "v_add_f32 %[" #X "], %[" #X "], %[s]\n"
#define FMAC(X) "v_fmac_f32 %[" #X "], %[s], %[t]\n"
#define FMA3(X) "v_fma_f32 %[" #X "], %[s], %[" #X "], -%[t]\n"
#define MED3(X) "v_med3_f32 %[" #X "], %[" #X "], %[s], %[t]\n"
#define MAX(X) "v_max_f32 %[" #X "], %[" #X "], %[s]\n"
#define FMACDPP(X) "v_fmac_f32_dpp %[" #X "], %[s], %[t] quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n"
#define MOVDPP(X) "v_mov_b32_dpp %[" #X "], %[s] quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n"
#define CNDM(X) "v_cndmask_b32 %[" #X "], %[" #X "], %[s], vcc\n"
#define SUB(X) "v_sub_f32 %[" #X "], %[s], %[" #X "]\n"
      if constexpr (V == 0) OP6(ADD)
      if constexpr (V == 1) OP6(FMAC)
      if constexpr (V == 2) OP6(FMA3)
      if constexpr (V == 3) OP6(MED3)
      if constexpr (V == 4) OP6(MAX)
      if constexpr (V == 5) OP6(FMACDPP)
      if constexpr (V == 6) OP6(MOVDPP)
      if constexpr (V == 7) OP6(CNDM)
      if constexpr (V == 8) OP6(SUB)
      if constexpr (V == 9)  // compares to SGPR pairs (VOP3)
        asm volatile("v_cmp_gt_f32 %[m], %[a], %[s]\n v_cmp_gt_f32 %[m], %[b], %[s]\n v_cmp_gt_f32 %[m], %[c], %[s]\n v_cmp_gt_f32 %[m], %[d], %[s]\n v_cmp_gt_f32 %[m], %[e], %[s]\n v_cmp_gt_f32 %[m], %[f], %[s]\n"
                     : [m] "=s"(m) : [a] "v"(a), [b] "v"(b), [c] "v"(c), [d] "v"(d), [e] "v"(e), [f] "v"(f), [s] "v"(s));
      if constexpr (V == 10)  // compares to VCC (VOPC)
        asm volatile("v_cmp_gt_f32 vcc, %[a], %[s]\n v_cmp_gt_f32 vcc, %[b], %[s]\n v_cmp_gt_f32 vcc, %[c], %[s]\n v_cmp_gt_f32 vcc, %[d], %[s]\n v_cmp_gt_f32 vcc, %[e], %[s]\n v_cmp_gt_f32 vcc, %[f], %[s]\n"
                     :: [a] "v"(a), [b] "v"(b), [c] "v"(c), [d] "v"(d), [e] "v"(e), [f] "v"(f), [s] "v"(s) : "vcc");
      if constexpr (V == 11)  // add with carry from an SGPR pair (VOP3B)
        asm volatile("v_addc_co_u32 %[a], vcc, %[a], %[a], %[m]\n v_addc_co_u32 %[b], vcc, %[b], %[b], %[m]\n v_addc_co_u32 %[c], vcc, %[c], %[c], %[m]\n v_addc_co_u32 %[d], vcc, %[d], %[d], %[m]\n v_addc_co_u32 %[e], vcc, %[e], %[e], %[m]\n v_addc_co_u32 %[f], vcc, %[f], %[f], %[m]\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5) : [m] "s"(m) : "vcc");
      if constexpr (V == 12)  // add with carry from VCC (VOP2)
        asm volatile("v_addc_co_u32 %[a], vcc, %[a], %[a], vcc\n v_addc_co_u32 %[b], vcc, %[b], %[b], vcc\n v_addc_co_u32 %[c], vcc, %[c], %[c], vcc\n v_addc_co_u32 %[d], vcc, %[d], %[d], vcc\n v_addc_co_u32 %[e], vcc, %[e], %[e], vcc\n v_addc_co_u32 %[f], vcc, %[f], %[f], vcc\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5) :: "vcc");
      if constexpr (V == 13)  // integer add VOP2
        asm volatile("v_add_u32 %[a], %[a], %[b]\n v_add_u32 %[b], %[b], %[c]\n v_add_u32 %[c], %[c], %[d]\n v_add_u32 %[d], %[d], %[e]\n v_add_u32 %[e], %[e], %[f]\n v_add_u32 %[f], %[f], %[a]\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5));
      if constexpr (V == 14)  // packed int16 add
        asm volatile("v_pk_add_u16 %[a], %[a], %[b]\n v_pk_add_u16 %[b], %[b], %[c]\n v_pk_add_u16 %[c], %[c], %[d]\n v_pk_add_u16 %[d], %[d], %[e]\n v_pk_add_u16 %[e], %[e], %[f]\n v_pk_add_u16 %[f], %[f], %[a]\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5));
      if constexpr (V == 15)  // packed int16 max
        asm volatile("v_pk_max_i16 %[a], %[a], %[b]\n v_pk_max_i16 %[b], %[b], %[c]\n v_pk_max_i16 %[c], %[c], %[d]\n v_pk_max_i16 %[d], %[d], %[e]\n v_pk_max_i16 %[e], %[e], %[f]\n v_pk_max_i16 %[f], %[f], %[a]\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5));
      if constexpr (V == 16)  // permlane16 swap
        asm volatile("v_permlane16_swap_b32 %[a], %[a]\n v_permlane16_swap_b32 %[b], %[b]\n v_permlane16_swap_b32 %[c], %[c]\n v_permlane16_swap_b32 %[d], %[d]\n v_permlane16_swap_b32 %[e], %[e]\n v_permlane16_swap_b32 %[f], %[f]\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5));
      if constexpr (V == 17)
        asm volatile("v_alignbit_b32 %[a], %[a], %[b], 31\n v_alignbit_b32 %[b], %[b], %[c], 31\n v_alignbit_b32 %[c], %[c], %[d], 31\n v_alignbit_b32 %[d], %[d], %[e], 31\n v_alignbit_b32 %[e], %[e], %[f], 31\n v_alignbit_b32 %[f], %[f], %[a], 31\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5));
      if constexpr (V == 18)
        asm volatile("v_lshl_or_b32 %[a], %[a], 1, %[b]\n v_lshl_or_b32 %[b], %[b], 1, %[c]\n v_lshl_or_b32 %[c], %[c], 1, %[d]\n v_lshl_or_b32 %[d], %[d], 1, %[e]\n v_lshl_or_b32 %[e], %[e], 1, %[f]\n v_lshl_or_b32 %[f], %[f], 1, %[a]\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5));
      if constexpr (V == 19)
        asm volatile("v_lshrrev_b32 %[a], 1, %[a]\n v_lshrrev_b32 %[b], 1, %[b]\n v_lshrrev_b32 %[c], 1, %[c]\n v_lshrrev_b32 %[d], 1, %[d]\n v_lshrrev_b32 %[e], 1, %[e]\n v_lshrrev_b32 %[f], 1, %[f]\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5));
      if constexpr (V == 20)
        asm volatile("v_xor_b32 %[a], %[a], %[b]\n v_xor_b32 %[b], %[b], %[c]\n v_xor_b32 %[c], %[c], %[d]\n v_xor_b32 %[d], %[d], %[e]\n v_xor_b32 %[e], %[e], %[f]\n v_xor_b32 %[f], %[f], %[a]\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5));
      if constexpr (V == 21)
        asm volatile("v_bfi_b32 %[a], %[a], %[b], %[c]\n v_bfi_b32 %[b], %[b], %[c], %[d]\n v_bfi_b32 %[c], %[c], %[d], %[e]\n v_bfi_b32 %[d], %[d], %[e], %[f]\n v_bfi_b32 %[e], %[e], %[f], %[a]\n v_bfi_b32 %[f], %[f], %[a], %[b]\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5));
      if constexpr (V == 22)
        asm volatile("v_min_f32 %[a], %[a], %[s]\n v_min_f32 %[b], %[b], %[s]\n v_min_f32 %[c], %[c], %[s]\n v_min_f32 %[d], %[d], %[s]\n v_min_f32 %[e], %[e], %[s]\n v_min_f32 %[f], %[f], %[s]\n"
                     : [a] "+v"(a), [b] "+v"(b), [c] "+v"(c), [d] "+v"(d), [e] "+v"(e), [f] "+v"(f) : [s] "v"(s));
      if constexpr (V == 23)
        asm volatile("v_max3_f32 %[a], %[a], %[s], %[t]\n v_max3_f32 %[b], %[b], %[s], %[t]\n v_max3_f32 %[c], %[c], %[s], %[t]\n v_max3_f32 %[d], %[d], %[s], %[t]\n v_max3_f32 %[e], %[e], %[s], %[t]\n v_max3_f32 %[f], %[f], %[s], %[t]\n"
                     : [a] "+v"(a), [b] "+v"(b), [c] "+v"(c), [d] "+v"(d), [e] "+v"(e), [f] "+v"(f) : [s] "v"(s), [t] "v"(t));
      if constexpr (V == 24)
        asm volatile("v_mul_f32 %[a], %[a], %[s]\n v_mul_f32 %[b], %[b], %[s]\n v_mul_f32 %[c], %[c], %[s]\n v_mul_f32 %[d], %[d], %[s]\n v_mul_f32 %[e], %[e], %[s]\n v_mul_f32 %[f], %[f], %[s]\n"
                     : [a] "+v"(a), [b] "+v"(b), [c] "+v"(c), [d] "+v"(d), [e] "+v"(e), [f] "+v"(f) : [s] "v"(s));
      if constexpr (V == 25)
        asm volatile("v_cndmask_b32 %[a], %[a], %[b], %[m]\n v_cndmask_b32 %[b], %[b], %[c], %[m]\n v_cndmask_b32 %[c], %[c], %[d], %[m]\n v_cndmask_b32 %[d], %[d], %[e], %[m]\n v_cndmask_b32 %[e], %[e], %[f], %[m]\n v_cndmask_b32 %[f], %[f], %[a], %[m]\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5) : [m] "s"(m));
      if constexpr (V == 26) {  // lane reads into SGPRs (the traceback's step)
        uint32_t r0, r1, r2, r3, r4, r5;
        asm volatile("v_readlane_b32 %[r0], %[a], 5\n v_readlane_b32 %[r1], %[b], 9\n v_readlane_b32 %[r2], %[c], 17\n v_readlane_b32 %[r3], %[d], 33\n v_readlane_b32 %[r4], %[e], 40\n v_readlane_b32 %[r5], %[f], 63\n"
                     : [r0] "=s"(r0), [r1] "=s"(r1), [r2] "=s"(r2), [r3] "=s"(r3), [r4] "=s"(r4), [r5] "=s"(r5)
                     : [a] "v"(u0), [b] "v"(u1), [c] "v"(u2), [d] "v"(u3), [e] "v"(u4), [f] "v"(u5));
        m += r0 ^ r1 ^ r2 ^ r3 ^ r4 ^ r5;
      }
      if constexpr (V == 27)  // lane writes from an SGPR
        asm volatile("v_writelane_b32 %[a], %[m], 5\n v_writelane_b32 %[b], %[m], 9\n v_writelane_b32 %[c], %[m], 17\n v_writelane_b32 %[d], %[m], 33\n v_writelane_b32 %[e], %[m], 40\n v_writelane_b32 %[f], %[m], 63\n"
                     : [a] "+v"(u0), [b] "+v"(u1), [c] "+v"(u2), [d] "+v"(u3), [e] "+v"(u4), [f] "+v"(u5) : [m] "s"((uint32_t)m));
    }
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = a + b + c + d + e + f + (float)(u0 + u1 + u2 + u3 + u4 + u5) + (float)(m & 1);
}

typedef void (*K)(float *, int);
int main() {
  int ncu = 256;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0);
  const int blocks = ncu * 8, threads = 256;
  float *out;
  (void)hipMalloc(&out, sizeof(float) * blocks * threads);
  const int iters = 4000;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  K ks[] = {mb<0>, mb<1>, mb<2>, mb<3>, mb<4>, mb<5>, mb<6>, mb<7>, mb<8>, mb<9>, mb<10>, mb<11>, mb<12>, mb<13>, mb<14>, mb<15>, mb<16>, mb<17>, mb<18>, mb<19>, mb<20>, mb<21>, mb<22>, mb<23>, mb<24>, mb<25>, mb<26>, mb<27>};
  const char *names[] = {"v_add_f32", "v_fmac_f32", "v_fma_f32 (vop3,neg)", "v_med3_f32", "v_max_f32", "v_fmac_f32_dpp", "v_mov_b32_dpp", "v_cndmask_b32 vcc", "v_sub_f32", "v_cmp_gt_f32 ->sgpr", "v_cmp_gt_f32 ->vcc", "v_addc carry sgpr", "v_addc carry vcc", "v_add_u32", "v_pk_add_u16", "v_pk_max_i16", "v_permlane16_swap", "v_alignbit_b32", "v_lshl_or_b32", "v_lshrrev_b32", "v_xor_b32", "v_bfi_b32", "v_min_f32", "v_max3_f32", "v_mul_f32", "v_cndmask sgpr", "v_readlane_b32", "v_writelane_b32"};
  for (int v = 0; v < 28; ++v) {
    for (int rep = 0; rep < 2; ++rep) {
      (void)hipEventRecord(e0);
      hipLaunchKernelGGL(ks[v], dim3(blocks), dim3(threads), 0, 0, out, iters);
      (void)hipEventRecord(e1);
      (void)hipEventSynchronize(e1);
      float ms;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double instr = (double)blocks * threads / 64 * iters * 4 * 6;
      const double cyc = ms * 1e-3 * 2.4e9;
      if (rep) printf("%-24s %7.3f ms  %.2f cycles per wave64 instruction per SIMD\n", names[v], ms, (ncu * 4) * cyc / instr);
    }
  }
  (void)hipFree(out);
  return 0;
}
