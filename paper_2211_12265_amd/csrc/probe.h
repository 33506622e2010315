// Issue-rate probe of gfx950's vector ALU for the integer instructions the
// kernels are built from, used to establish the peak that the benchmark's
// roofline fraction divides by.  Every lane runs eight independent
// dependency chains of one instruction (written as inline assembly, so that
// the count is exact: 128 instructions per loop trip and lane, 16 unrolled
// rounds of 8 chains); the loop's own counter lives in scalar registers.  No
// memory is touched until the final vector store of one word per lane.
#pragma once
#include "common.h"

namespace dil {

constexpr int PROBE_INSTR_PER_ITER = 128;
constexpr int PROBE_WG = 256;

// KIND: 0 v_xor_b32, 1 v_add_u32, 2 v_bitop3_b32, 3 v_alignbit_b32,
//       4 v_mul_lo_u32, 5 v_mad_u64_u32 (64-bit accumulate)
template <int KIND>
__global__ void __launch_bounds__(PROBE_WG) alu_probe_k(uint32_t *out, uint32_t iters) {
  const uint32_t b = threadIdx.x * 2654435761u + 1u, c = threadIdx.x ^ 0x9E3779B9u;
  uint32_t a[8];
  uint64_t m[8];
#pragma unroll
  for (int j = 0; j < 8; j++) {
    a[j] = threadIdx.x + 0x1234567u * (uint32_t)j;
    m[j] = a[j];
  }
  for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
    for (int u = 0; u < 16; u++)
#pragma unroll
      for (int j = 0; j < 8; j++) {
        if constexpr (KIND == 0) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
        else if constexpr (KIND == 1) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
        else if constexpr (KIND == 2)
          asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[j]) : "v"(b), "v"(c));
        else if constexpr (KIND == 3) asm volatile("v_alignbit_b32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
        else if constexpr (KIND == 4) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
        else asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(m[j]) : "v"(a[j]), "v"(b) : "vcc");
      }
  }
  uint32_t x = 0;
#pragma unroll
  for (int j = 0; j < 8; j++) x ^= a[j] ^ (uint32_t)m[j] ^ (uint32_t)(m[j] >> 32);
  out[(size_t)blockIdx.x * PROBE_WG + threadIdx.x] = x;
}

}  // namespace dil
