// Optimisation ablation of the NTT primitive c = INTT(NTT(a) o b) (Sec. 2.2,
// Sec. 3.2, Sec. 4.2): the forms the production kernel ntt_mul_k<true> was
// reached from, each computing the same butterflies with the same twiddles in
// the same order within every coefficient, so all of them return identical
// words.  They exist to be timed and counted, not to be used:
//
//   ntt_mul_k<false>     one LDS transpose per transform, unpadded (bank conflicts);
//   ntt_mul_perlevel_k   one LDS round trip and wave barrier per butterfly level,
//                        no levels merged in registers;
//   ntt_fwd_k, ntt_pointwise_k, ntt_inv_k
//                        unfused: forward NTT, pointwise product and inverse NTT
//                        as three launches that pass the polynomials through HBM.
#pragma once
#include "kernels.h"

namespace dil {

// Forward NTT in LDS, natural coefficient order in, slot order out: level by
// level, lane t of a 16-lane group does butterflies t, t + 16, ..., t + 112.
__device__ __forceinline__ void ntt_levels_lds(int32_t *p, int t) {
  for (int len = 128, k0 = 1; len >= 1; len >>= 1, k0 <<= 1) {
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const int b = t + 16 * i, grp = b / len, j = grp * 2 * len + (b & (len - 1));
      int32_t x = p[j], y = p[j + len];
      ct_bfly(x, y, kZT.z[k0 + grp]);
      p[j] = x;
      p[j + len] = y;
    }
    wave_sync();
  }
}

// Inverse NTT in LDS, slot order in (|x| < q), natural order out in (-q, q);
// the last level folds in 1/256 and the Montgomery factor of the pointwise product.
__device__ __forceinline__ void intt_levels_lds(int32_t *p, int t) {
  for (int len = 1, k0 = 128; len <= 64; len <<= 1, k0 >>= 1) {
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const int b = t + 16 * i, grp = b / len, j = grp * 2 * len + (b & (len - 1));
      int32_t x = p[j], y = p[j + len];
      gs_bfly(x, y, kZT.zi[k0 + grp]);
      p[j] = x;
      p[j + len] = y;
    }
    wave_sync();
  }
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const int j = t + 16 * i;
    const int32_t x = p[j], y = p[j + 128];
    p[j] = mont_mul(x + y, SCALE_M);
    p[j + 128] = mont_mul(x - y, zinv_scaled_m(1));
  }
  wave_sync();
}

__global__ void __launch_bounds__(256) ntt_mul_perlevel_k(const int32_t *a, const int32_t *b, int32_t *c,
                                                          uint64_t count) {
  __shared__ int32_t buf[16 * N];
  const int g = threadIdx.x >> 4, t = threadIdx.x & 15;
  int32_t *p = buf + g * N;
  for (uint64_t q = (uint64_t)blockIdx.x * 16 + g; q < count; q += (uint64_t)gridDim.x * 16) {
#pragma unroll
    for (int i = 0; i < 16; i++) p[t + 16 * i] = a[q * N + t + 16 * i];
    wave_sync();
    ntt_levels_lds(p, t);
#pragma unroll
    for (int i = 0; i < 16; i++) p[t + 16 * i] = mont_mul(p[t + 16 * i], b[q * N + t + 16 * i]);
    wave_sync();
    intt_levels_lds(p, t);
#pragma unroll
    for (int i = 0; i < 16; i++) c[q * N + t + 16 * i] = canon(p[t + 16 * i]);
    wave_sync();
  }
}

// unfused step 1: ahat (slot order, |x| < 9q) = NTT(a), written to out
__global__ void __launch_bounds__(256) ntt_fwd_k(const int32_t *a, int32_t *out, uint64_t count) {
  __shared__ int32_t trl[16 * NTT_LDS_GROUP];
  const int g = threadIdx.x >> 4, t = threadIdx.x & 15;
  int32_t *tr = trl + g * NTT_LDS_GROUP;
  const Tw ftw = ntt_lane_tw(t);
  for (uint64_t q = (uint64_t)blockIdx.x * 16 + g; q < count; q += (uint64_t)gridDim.x * 16) {
    int32_t x[16];
    load_strided(x, a + q * N, t);
    ntt16(x, ftw, tr, t);
    store_slots(x, out + q * N, t);
  }
}

// unfused step 2: c = c o b (one Montgomery product per word), four words per lane
__global__ void __launch_bounds__(256) ntt_pointwise_k(int32_t *c, const int32_t *b, uint64_t words4) {
  int4 *c4 = (int4 *)c;
  const int4 *b4 = (const int4 *)b;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words4;
       i += (uint64_t)gridDim.x * blockDim.x) {
    int4 x = c4[i];
    const int4 y = b4[i];
    x.x = mont_mul(x.x, y.x);
    x.y = mont_mul(x.y, y.y);
    x.z = mont_mul(x.z, y.z);
    x.w = mont_mul(x.w, y.w);
    c4[i] = x;
  }
}

// unfused step 3: c = canonical INTT(c), in place (each group reads its whole
// polynomial before the transpose's barrier and writes it after)
__global__ void __launch_bounds__(256) ntt_inv_k(int32_t *c, uint64_t count) {
  __shared__ int32_t trl[16 * NTT_LDS_GROUP];
  const int g = threadIdx.x >> 4, t = threadIdx.x & 15;
  int32_t *tr = trl + g * NTT_LDS_GROUP;
  const Tw itw = intt_lane_tw(t);
  for (uint64_t q = (uint64_t)blockIdx.x * 16 + g; q < count; q += (uint64_t)gridDim.x * 16) {
    int32_t x[16];
    load_slots(x, c + q * N, t);
    intt16(x, itw, tr, t);
#pragma unroll
    for (int r = 0; r < 16; r++) x[r] = canon(x[r]);
    store_strided(x, c + q * N, t);
  }
}

}  // namespace dil
