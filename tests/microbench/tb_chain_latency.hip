// Latency of one traceback-like dependent step on gfx950: a chain that hops
// over 64 words, the next index read out of the current word.
//   V0: the word sits in a VGPR, one per lane; a step is v_readlane with the
//       lane index from an SGPR, then a scalar AND and XOR (the decoder's
//       traceback step; `zero` is 0 at run time so the XOR stays).
//   V1: the 64 words sit in global memory (256 B per wave); a step is a
//       scalar load at the current byte offset, a wait, and a scalar AND.
//   V2: as V1 with two more scalar ALU operations per step (a bit extract
//       and an XOR, as a decision bit would need).
// Each wave runs its own chain; the table is a random cycle over the 64
// entries, so every index stays inside the wave's 64 words.  Reported per
// step: shader-clock cycles (s_memtime) and nanoseconds (s_memrealtime at
// 100 MHz), averaged over waves, at 1 wave per SIMD and at 8 waves per SIMD
// (every wave chaining), plus the kernel time.  Timing only.
// Build and run (one MI355X):
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         tests/microbench/tb_chain_latency.hip -o /tmp/tb_chain_latency && /tmp/tb_chain_latency
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                 \
      exit(1);                                                                \
    }                                                                         \
  } while (0)

template <int V>
__global__ __launch_bounds__(256) void chain(const uint32_t *tbl, uint64_t *out, int steps, uint32_t zero) {
  const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + threadIdx.x / 64));
  const uint32_t *reg = tbl + (size_t)wave * 64;
  uint32_t idx = 0;
  const uint32_t w = reg[threadIdx.x & 63];  // V0: lane index of the next word
  __builtin_amdgcn_s_waitcnt(0);
  const uint64_t t0 = __builtin_amdgcn_s_memtime();
  const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
  if constexpr (V == 0) {
    for (int i = 0; i < steps; i += 8) {
#pragma unroll
      for (int j = 0; j < 8; ++j) idx = ((uint32_t)__builtin_amdgcn_readlane((int)w, (int)idx) & 63u) ^ zero;
    }
  } else {
    const uint64_t base = (uint64_t)(uintptr_t)reg;
    uint32_t off = 0, acc = 0;
    for (int i = 0; i < steps; i += 8) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if constexpr (V == 1)
          asm volatile("s_load_dword %0, %1, %0\n\t"
                       "s_waitcnt lgkmcnt(0)\n\t"
                       "s_and_b32 %0, %0, 0xfc"
                       : "+s"(off)
                       : "s"(base)
                       : "scc");
        else
          asm volatile("s_load_dword %0, %2, %0\n\t"
                       "s_waitcnt lgkmcnt(0)\n\t"
                       "s_bfe_u32 %1, %0, 0x10002\n\t"
                       "s_xor_b32 %1, %1, %0\n\t"
                       "s_and_b32 %0, %0, 0xfc"
                       : "+s"(off), "+s"(acc)
                       : "s"(base)
                       : "scc");
      }
    }
    idx = off + (acc & 0u);
  }
  const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
  const uint64_t t1 = __builtin_amdgcn_s_memtime();
  if ((threadIdx.x & 63) == 0) {
    out[(size_t)wave * 3 + 0] = t1 - t0;
    out[(size_t)wave * 3 + 1] = r1 - r0;
    out[(size_t)wave * 3 + 2] = idx;
  }
}

int main() {
  int dev = 0, ncu = 0;
  CHECK(hipGetDevice(&dev));
  CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int steps = 4096;
  const int max_blocks = ncu * 8;  // 8 workgroups of 4 waves per CU = 8 waves per SIMD
  const int max_waves = max_blocks * 4;
  // a random single cycle over 0..63 per wave (Sattolo's shuffle)
  std::vector<uint32_t> cyc(64);
  std::vector<uint32_t> h_lane((size_t)max_waves * 64), h_byte((size_t)max_waves * 64);
  srand(1);
  for (int wv = 0; wv < max_waves; ++wv) {
    for (int i = 0; i < 64; ++i) cyc[i] = i;
    for (int i = 63; i > 0; --i) {
      const int j = rand() % i;
      const uint32_t t = cyc[i];
      cyc[i] = cyc[j];
      cyc[j] = t;
    }
    for (int i = 0; i < 64; ++i) {
      if (cyc[i] > 63) return 1;
      h_lane[(size_t)wv * 64 + i] = cyc[i];
      h_byte[(size_t)wv * 64 + i] = cyc[i] * 4u;
    }
  }
  uint32_t *d_lane = nullptr, *d_byte = nullptr;
  uint64_t *d_out = nullptr;
  CHECK(hipMalloc(&d_lane, h_lane.size() * 4));
  CHECK(hipMalloc(&d_byte, h_byte.size() * 4));
  CHECK(hipMalloc(&d_out, (size_t)max_waves * 3 * 8));
  CHECK(hipMemcpy(d_lane, h_lane.data(), h_lane.size() * 4, hipMemcpyHostToDevice));
  CHECK(hipMemcpy(d_byte, h_byte.data(), h_byte.size() * 4, hipMemcpyHostToDevice));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const char *names[3] = {"v_readlane + s_and + s_xor", "s_load + s_and", "s_load + 3 SALU"};
  printf("| Step | Waves per SIMD | Cycles per step (s_memtime) | ns per step | Kernel ms |\n|---|---|---|---|---|\n");
  for (int v = 0; v < 3; ++v) {
    for (int wps : {1, 8}) {
      const int blocks = ncu * wps;
      const int waves = blocks * 4;
      const uint32_t *tbl = v == 0 ? d_lane : d_byte;
      for (int rep = 0; rep < 2; ++rep) {
        CHECK(hipEventRecord(e0, 0));
        if (v == 0) hipLaunchKernelGGL(chain<0>, dim3(blocks), dim3(256), 0, 0, tbl, d_out, steps, 0u);
        if (v == 1) hipLaunchKernelGGL(chain<1>, dim3(blocks), dim3(256), 0, 0, tbl, d_out, steps, 0u);
        if (v == 2) hipLaunchKernelGGL(chain<2>, dim3(blocks), dim3(256), 0, 0, tbl, d_out, steps, 0u);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
      }
      float ms = 0;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      std::vector<uint64_t> h((size_t)waves * 3);
      CHECK(hipMemcpy(h.data(), d_out, h.size() * 8, hipMemcpyDeviceToHost));
      double cyc_sum = 0, rt_sum = 0;
      for (int wv = 0; wv < waves; ++wv) {
        cyc_sum += (double)h[(size_t)wv * 3];
        rt_sum += (double)h[(size_t)wv * 3 + 1];
      }
      printf("| %s | %d | %.1f | %.1f | %.3f |\n", names[v], wps, cyc_sum / waves / steps,
             rt_sum / waves / steps * 10.0, ms);
    }
  }
  CHECK(hipFree(d_lane));
  CHECK(hipFree(d_byte));
  CHECK(hipFree(d_out));
  return 0;
}
