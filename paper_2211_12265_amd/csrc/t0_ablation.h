// NTT(t0) of the signing procedure in four forms, for the optimisation
// ablation of Sec. 5 ("speedup breakdown"): t0 is unpacked from the secret
// key (13-bit fields, coefficient 2^(d-1) - v, reading 12 of the encodings)
// and transformed to the NTT domain.  The forms add the paper's three
// optimisations one at a time:
//   variant 3  basic: an unpacking kernel stores t0 in global memory, a second
//              kernel loads it and runs the NTT (unpadded LDS transpose);
//   variant 2  one fused kernel with the same memory access pattern (t0
//              written to global memory and read back inside the kernel);
//   variant 1  unpacking merged into the NTT: the coefficients go from the
//              staged key bytes straight into registers (unpadded transpose);
//   variant 0  as 1 with the padded, bank-conflict-free transpose -- the code
//              path of sg_secret_k, which the Sign setup runs.
// Every form writes NTT(t0) reduced to [0, q) in natural slot order
// (t0_hat[task][i][j] = slot j of polynomial i), the same words for all four.
#pragma once
#include "kernels.h"

namespace dil {

// full reduction of an NTT output (|x| < 9q) to [0, q)
__device__ __forceinline__ int32_t reduce_q(int32_t x) {
  const int32_t r = x % Q;
  return r + ((r >> 31) & Q);
}

// Unpack chunk c (coefficients 8c .. 8c + 7 of the task's K t0 polynomials,
// 13 bytes of the encoding) from the sk row in global memory to t0 in global
// memory, one lane per chunk.
template <int LV>
__device__ __forceinline__ void t0_unpack_chunk(const uint8_t *skrow, int32_t *t0row, int c) {
  const int i = c >> 5, c8 = c & 31;
  const uint8_t *src = skrow + P<LV>::OFF_T0 + i * P<LV>::T0B + 13 * c8;
  uint64_t lo = 0, hi = 0;
#pragma unroll
  for (int b = 0; b < 8; b++) lo |= (uint64_t)src[b] << (8 * b);
#pragma unroll
  for (int b = 0; b < 5; b++) hi |= (uint64_t)src[8 + b] << (8 * b);
  int32_t *dst = t0row + i * N + 8 * c8;
#pragma unroll
  for (int j = 0; j < 8; j++) {
    const int p = 13 * j;
    uint64_t v;
    if (p + 13 <= 64) v = lo >> p;
    else if (p >= 64) v = hi >> (p - 64);
    else v = (lo >> p) | (hi << (64 - p));
    dst[j] = (1 << (D - 1)) - (int32_t)(v & 0x1FFFu);
  }
}

// variant 3, first kernel: one lane per 8-coefficient chunk
template <int LV>
__global__ void __launch_bounds__(256) t0_unpack_k(const uint8_t *sk, int32_t *t0_hat, uint32_t count) {
  constexpr int K = Lv<LV>::K;
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (uint64_t)count * K * 32) return;
  const uint64_t task = c / (K * 32);
  t0_unpack_chunk<LV>(sk + task * P<LV>::SK, t0_hat + task * K * N, (int)(c % (K * 32)));
}

// variants 3 (second kernel, FUSED = false) and 2 (FUSED = true): NTT of t0
// loaded from global memory, in place; one wavefront per task, one 16-lane
// group per polynomial, unpadded transpose.  Each group loads its whole
// polynomial before it stores anything, so the transform can run in place.
template <int LV, bool FUSED>
__global__ void __launch_bounds__(64) t0_ntt_gmem_k(const uint8_t *sk, int32_t *t0_hat, uint32_t count) {
  constexpr int K = Lv<LV>::K;
  __shared__ int32_t tr[4 * NTT_LDS_GROUP];
  const uint32_t task = blockIdx.x;
  if (task >= count) return;
  const int lane = threadIdx.x, g = lane >> 4, t = lane & 15;
  int32_t *row = t0_hat + (size_t)task * K * N;
  if constexpr (FUSED) {
    for (int c = lane; c < K * 32; c += 64) t0_unpack_chunk<LV>(sk + (size_t)task * P<LV>::SK, row, c);
    // the chunks written by other lanes must be visible to this lane's loads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  const Tw ftw = ntt_lane_tw(t);
  for (int i = g; i < K; i += 4) {
    int32_t x[16];
    load_strided(x, row + i * N, t);
    ntt16<Tw, false>(x, ftw, tr + g * NTT_LDS_GROUP, t);
#pragma unroll
    for (int r = 0; r < 16; r++) x[r] = reduce_q(x[r]);
    store_slots(x, row + i * N, t);
  }
}

// variants 1 (PAD = false) and 0 (PAD = true): the t0 bytes of the key are
// staged in LDS with coalesced loads, each lane unpacks its strided
// coefficients into registers and the NTT starts from them.
template <int LV, bool PAD>
__global__ void __launch_bounds__(64) t0_ntt_reg_k(const uint8_t *sk, int32_t *t0_hat, uint32_t count) {
  constexpr int K = Lv<LV>::K, TW = P<LV>::T0B / 4;  // 104 words per packed t0 polynomial
  static_assert(P<LV>::OFF_T0 % 4 == 0 && P<LV>::T0B % 4 == 0, "t0 rows are word-aligned in the sk row");
  __shared__ int32_t tr[4 * NTT_LDS_GROUP];
  __shared__ uint32_t buf[K * TW + 2];
  const uint32_t task = blockIdx.x;
  if (task >= count) return;
  const int lane = threadIdx.x, g = lane >> 4, t = lane & 15;
  g2l_words<K * TW>((const uint32_t *)(sk + (size_t)task * P<LV>::SK + P<LV>::OFF_T0), buf, lane);
  if (lane < 2) buf[K * TW + lane] = 0;
  wave_sync();
  const Tw ftw = ntt_lane_tw(t);
  int32_t *row = t0_hat + (size_t)task * K * N;
  for (int i = g; i < K; i += 4) {
    uint32_t v[16];
    int32_t x[16];
    unpack_strided<13>(buf + i * TW, v, t);
#pragma unroll
    for (int r = 0; r < 16; r++) x[r] = (1 << (D - 1)) - (int32_t)v[r];
    ntt16<Tw, PAD>(x, ftw, tr + g * NTT_LDS_GROUP, t);
#pragma unroll
    for (int r = 0; r < 16; r++) x[r] = reduce_q(x[r]);
    store_slots(x, row + i * N, t);
  }
}

}  // namespace dil
