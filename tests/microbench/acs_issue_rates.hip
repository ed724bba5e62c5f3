// Issue cost of add-compare-select instruction sequences on gfx950 (the
// decoder's sign-folded ACS and variants), one chain per wave at eight waves
// per SIMD.  Timing only.  Build and run (one MI355X):
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         tests/microbench/acs_issue_rates.hip -o /tmp/acs_issue_rates && /tmp/acs_issue_rates
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdint.h>

#define STAGE_FULL(DPP)                                                             \
  asm volatile(                                                                     \
      "v_fma_f32 %[A], %[s], %[o], -%[y]\n"                                         \
      "v_addc_co_u32 %[d], vcc, %[d], %[d], %[pd]\n"                                \
      "v_fmac_f32_dpp %[y], %[o], %[s] " DPP " row_mask:0xf bank_mask:0xf\n"       \
      "v_cmp_gt_f32 %[pd], %[y], %[A]\n"                                            \
      "v_med3_f32 %[o], %[y], %[A], %[c]\n"                                         \
      : [o] "+v"(o), [A] "=&v"(A), [y] "+v"(y), [d] "+v"(d), [pd] "+s"(pd)         \
      : [s] "v"(sg), [c] "v"(cm) : "vcc");

template <int V>
__global__ __launch_bounds__(256) void mb(float *out, int iters, float y0) {
  float o = threadIdx.x * 0.5f, sg = 1.0f, cm = 1e30f, A, T, y = y0;
  uint32_t d = 0;
  uint64_t pd = 0;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if constexpr (V == 0) { STAGE_FULL("quad_perm:[1,0,3,2]") }
      if constexpr (V == 1) {  // no DPP on the fmac
        asm volatile("v_fma_f32 %[A], %[s], %[o], -%[y]\n v_addc_co_u32 %[d], vcc, %[d], %[d], %[pd]\n v_fmac_f32 %[y], %[o], %[s]\n v_cmp_gt_f32 %[pd], %[y], %[A]\n v_med3_f32 %[o], %[y], %[A], %[c]\n"
            : [o] "+v"(o), [A] "=&v"(A), [y] "+v"(y), [d] "+v"(d), [pd] "+s"(pd) : [s] "v"(sg), [c] "v"(cm) : "vcc");
      }
      if constexpr (V == 2) {  // no compare / addc (select only)
        asm volatile("v_fma_f32 %[A], %[s], %[o], -%[y]\n v_fmac_f32_dpp %[y], %[o], %[s] quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n v_med3_f32 %[o], %[y], %[A], %[c]\n"
            : [o] "+v"(o), [A] "=&v"(A), [y] "+v"(y) : [s] "v"(sg), [c] "v"(cm));
      }
      if constexpr (V == 3) {  // compare to VCC-free VGPR instead of SGPR: v_sub + bit accumulate
        asm volatile("v_fma_f32 %[A], %[s], %[o], -%[y]\n v_fmac_f32_dpp %[y], %[o], %[s] quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n v_sub_f32 %[t], %[A], %[y]\n v_med3_f32 %[o], %[y], %[A], %[c]\n v_lshrrev_b32 %[t], 31, %[t]\n v_lshl_or_b32 %[d], %[d], 1, %[t]\n"
            : [o] "+v"(o), [A] "=&v"(A), [y] "+v"(y), [d] "+v"(d), [t] "=&v"(A) : [s] "v"(sg), [c] "v"(cm));
      }
      if constexpr (V == 4) {  // row_half_mirror DPP
        STAGE_FULL("row_half_mirror")
      }
      if constexpr (V == 5) {  // permlane16 swap exchange
        asm volatile("v_fma_f32 %[A], %[s], %[o], -%[y]\n v_addc_co_u32 %[d], vcc, %[d], %[d], %[pd]\n v_permlane16_swap_b32 %[o], %[o]\n v_fma_f32 %[y], %[s], %[o], %[y]\n v_cmp_gt_f32 %[pd], %[y], %[A]\n v_med3_f32 %[o], %[y], %[A], %[c]\n"
            : [o] "+v"(o), [A] "=&v"(A), [y] "+v"(y), [d] "+v"(d), [pd] "+s"(pd) : [s] "v"(sg), [c] "v"(cm) : "vcc");
      }
      if constexpr (V == 7) {  // new: sub + alignbit decision
        asm volatile("v_fma_f32 %[A], %[s], %[o], -%[y]\n v_fmac_f32_dpp %[y], %[o], %[s] quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n v_sub_f32 %[t], %[y], %[A]\n v_med3_f32 %[o], %[y], %[A], %[c]\n v_alignbit_b32 %[d], %[d], %[t], 31\n"
            : [o] "+v"(o), [A] "=&v"(A), [y] "+v"(y), [d] "+v"(d), [t] "=&v"(T) : [s] "v"(sg), [c] "v"(cm));
      }
      if constexpr (V == 6) {  // 5 independent plain adds (issue-rate reference)
        asm volatile("v_add_f32 %[A], %[A], %[s]\n v_add_f32 %[y], %[y], %[s]\n v_add_f32 %[o], %[o], %[s]\n v_add_f32 %[c2], %[c2], %[s]\n v_add_f32 %[e], %[e], %[s]\n"
            : [o] "+v"(o), [A] "+v"(A), [y] "+v"(y), [c2] "+v"(cm), [e] "+v"(sg) : [s] "v"(sg));
      }
    }
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = o + y + (float)d + (float)(pd & 1);
}

int main() {
  int ncu = 256;
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0);
  const int blocks = ncu * 8, threads = 256;  // 32 waves per CU = 8 per SIMD
  float *out;
  hipMalloc(&out, sizeof(float) * blocks * threads);
  const int iters = 4000;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  const char *names[] = {"full(quad_perm)", "no-dpp", "no-cmp/addc", "sub+shift bits", "full(half_mirror)", "permlane16", "5 plain adds", "sub+alignbit"};
  const int ninstr[] = {5, 5, 3, 6, 5, 6, 5, 5};
  for (int v = 0; v < 8; ++v) {
    for (int rep = 0; rep < 2; ++rep) {
      hipEventRecord(e0);
      switch (v) {
        case 0: mb<0><<<blocks, threads>>>(out, iters, 1.0f); break;
        case 1: mb<1><<<blocks, threads>>>(out, iters, 1.0f); break;
        case 2: mb<2><<<blocks, threads>>>(out, iters, 1.0f); break;
        case 3: mb<3><<<blocks, threads>>>(out, iters, 1.0f); break;
        case 4: mb<4><<<blocks, threads>>>(out, iters, 1.0f); break;
        case 5: mb<5><<<blocks, threads>>>(out, iters, 1.0f); break;
        case 6: mb<6><<<blocks, threads>>>(out, iters, 1.0f); break;
        case 7: mb<7><<<blocks, threads>>>(out, iters, 1.0f); break;
      }
      hipEventRecord(e1);
      hipEventSynchronize(e1);
      float ms;
      hipEventElapsedTime(&ms, e0, e1);
      const double waves = (double)blocks * threads / 64;
      const double instr = waves * iters * 6 * ninstr[v];
      const double cyc = ms * 1e-3 * 2.4e9;
      // per SIMD: instructions issued per cycle (1/4 = full wave64 rate on a 16-lane SIMD)
      if (rep) printf("%-20s %8.3f ms  %.3f wave-instr/cycle/SIMD  (%.2f cycles per instr)\n", names[v], ms,
                      instr / (ncu * 4) / cyc, (ncu * 4) * cyc / instr);
    }
  }
  hipFree(out);
  return 0;
}
