// 256-point negacyclic NTT / INTT over Z_q (Sec. 2.2, Sec. 3.2) for gfx950.
//
// One polynomial per group of 16 lanes, 16 coefficients per lane in VGPRs.
// Each transform runs four butterfly levels inside each lane, one 16x16
// transpose through LDS, and four more in-lane levels -- a single exchange per
// transform instead of one per level (the paper's warp-per-poly version
// exchanges through shared memory before level 4 and level 7).
//
// Layouts (t = lane within the group, r = register 0..15):
//   "strided"  x[r] holds coefficient  t + 16 r   (NTT input, INTT output)
//   "slots"    x[r] holds NTT slot    16 t + r    (NTT output, INTT input)
// Slot j holds the polynomial evaluated at psi^(2 brv8(j) + 1), psi = 1753.
// Loading or storing a strided polynomial is coalesced: for each r the 16
// lanes touch 64 contiguous bytes.
//
// Arithmetic: signed Montgomery with R = 2^32 (three VALU ops per product on
// gfx950).  Forward twiddles are psi^brv8(k) in Montgomery form, so the
// forward transform is exact; pointwise products carry one 2^-32 which the
// INTT's last level removes together with 1/256.
// Bounds: forward input |x| < q gives output |x| < 9q; INTT input |x| < q
// gives output in (-q, q).
//
// LDS transpose: element i of a group's 272-word region lives at i + i/16
// (one pad word per 16).  With groups 272 words apart the write (strided) and
// read (slots) patterns are both free of bank conflicts for 32 banks per
// half-wave and for 64 banks per wave.
#pragma once
#include "common.h"

namespace dil {

struct ZTab {
  int32_t z[256], zi[256];
  constexpr ZTab() : z(), zi() {
    for (int k = 0; k < 256; k++) {
      z[k] = k ? zeta_m(k) : 0;
      zi[k] = k ? zinv_m(k) : 0;
    }
  }
};
__constant__ constexpr ZTab kZT = ZTab();

constexpr int NTT_LDS_GROUP = 272;  // int32 words per 16-lane group

// PAD = false drops the pad word (the bank-conflicted layout, kept for the
// optimisation ablation of the NTT primitive)
template <bool PAD = true>
__device__ __forceinline__ int lds_idx(int i) { return PAD ? i + (i >> 4) : i; }

// An NTT-domain vector kept in LDS for pointwise products: polynomial j, lane
// t, register r (slot 16 t + r) lives at j * HAT_POLY + 17 t + r.  With one pad
// word per 16 slots, the 64 lanes of a wave hit 64 distinct banks both when
// each 16-lane group writes its own polynomial and when all groups read the
// same polynomial (then equal addresses broadcast).
constexpr int HAT_POLY = 272;
__device__ __forceinline__ int hat_idx(int j, int t, int r) { return j * HAT_POLY + 17 * t + r; }

// per-lane twiddles for the four lane-dependent levels (15 values), held in VGPRs
struct Tw {
  int32_t w[15];
  __device__ __forceinline__ int32_t operator()(int k) const { return w[k]; }
};

__device__ __forceinline__ Tw ntt_lane_tw(int t) {
  Tw tw;
  tw.w[0] = kZT.z[16 + t];
#pragma unroll
  for (int a = 0; a < 2; a++) tw.w[1 + a] = kZT.z[32 + 2 * t + a];
#pragma unroll
  for (int a = 0; a < 4; a++) tw.w[3 + a] = kZT.z[64 + 4 * t + a];
#pragma unroll
  for (int a = 0; a < 8; a++) tw.w[7 + a] = kZT.z[128 + 8 * t + a];
  return tw;
}
__device__ __forceinline__ Tw intt_lane_tw(int t) {
  Tw tw;
#pragma unroll
  for (int a = 0; a < 8; a++) tw.w[a] = kZT.zi[128 + 8 * t + a];
#pragma unroll
  for (int a = 0; a < 4; a++) tw.w[8 + a] = kZT.zi[64 + 4 * t + a];
#pragma unroll
  for (int a = 0; a < 2; a++) tw.w[12 + a] = kZT.zi[32 + 2 * t + a];
  tw.w[14] = kZT.zi[16 + t];
  return tw;
}

__device__ __forceinline__ void ct_bfly(int32_t &a, int32_t &b, int32_t z) {
  int32_t t = mont_mul(b, z);
  b = a - t;
  a = a + t;
}
__device__ __forceinline__ void gs_bfly(int32_t &a, int32_t &b, int32_t zi) {
  int32_t t = a;
  a = t + b;
  b = mont_mul(t - b, zi);
}

// strided -> slots within a group (lds points at the group's 272-word region)
template <bool PAD = true>
__device__ __forceinline__ void transpose_s2c(int32_t x[16], int32_t *lds, int t) {
#pragma unroll
  for (int r = 0; r < 16; r++) lds[lds_idx<PAD>(t + 16 * r)] = x[r];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int r = 0; r < 16; r++) x[r] = lds[lds_idx<PAD>(16 * t + r)];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <bool PAD = true>
__device__ __forceinline__ void transpose_c2s(int32_t x[16], int32_t *lds, int t) {
#pragma unroll
  for (int r = 0; r < 16; r++) lds[lds_idx<PAD>(16 * t + r)] = x[r];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int r = 0; r < 16; r++) x[r] = lds[lds_idx<PAD>(t + 16 * r)];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward NTT: strided input -> slots output.
template <class TW, bool PAD = true>
__device__ __forceinline__ void ntt16(int32_t x[16], const TW &tw, int32_t *lds, int t) {
  // levels with distance 128, 64, 32, 16: register distance 8, 4, 2, 1, compile-time twiddles
#pragma unroll
  for (int r = 0; r < 8; r++) ct_bfly(x[r], x[r + 8], zeta_m(1));
#pragma unroll
  for (int r = 0; r < 16; r++)
    if ((r & 4) == 0) ct_bfly(x[r], x[r + 4], zeta_m(2 + r / 8));
#pragma unroll
  for (int r = 0; r < 16; r++)
    if ((r & 2) == 0) ct_bfly(x[r], x[r + 2], zeta_m(4 + r / 4));
#pragma unroll
  for (int r = 0; r < 16; r += 2) ct_bfly(x[r], x[r + 1], zeta_m(8 + r / 2));
  transpose_s2c<PAD>(x, lds, t);
  // distance 8, 4, 2, 1 inside the lane's 16 consecutive slots, lane-dependent twiddles
#pragma unroll
  for (int r = 0; r < 8; r++) ct_bfly(x[r], x[r + 8], tw(0));
#pragma unroll
  for (int r = 0; r < 16; r++)
    if ((r & 4) == 0) ct_bfly(x[r], x[r + 4], tw(1 + r / 8));
#pragma unroll
  for (int r = 0; r < 16; r++)
    if ((r & 2) == 0) ct_bfly(x[r], x[r + 2], tw(3 + r / 4));
#pragma unroll
  for (int r = 0; r < 16; r += 2) ct_bfly(x[r], x[r + 1], tw(7 + r / 2));
}

// Inverse NTT: slots input (|x| < q) -> strided output in (-q, q); removes the
// 2^-32 of one Montgomery product and divides by 256.
template <class TW, bool PAD = true>
__device__ __forceinline__ void intt16(int32_t x[16], const TW &tw, int32_t *lds, int t) {
#pragma unroll
  for (int r = 0; r < 16; r += 2) gs_bfly(x[r], x[r + 1], tw(r / 2));
#pragma unroll
  for (int r = 0; r < 16; r++)
    if ((r & 2) == 0) gs_bfly(x[r], x[r + 2], tw(8 + r / 4));
#pragma unroll
  for (int r = 0; r < 16; r++)
    if ((r & 4) == 0) gs_bfly(x[r], x[r + 4], tw(12 + r / 8));
#pragma unroll
  for (int r = 0; r < 8; r++) gs_bfly(x[r], x[r + 8], tw(14));
  transpose_c2s<PAD>(x, lds, t);
#pragma unroll
  for (int r = 0; r < 16; r += 2) gs_bfly(x[r], x[r + 1], zinv_m(8 + r / 2));
#pragma unroll
  for (int r = 0; r < 16; r++)
    if ((r & 2) == 0) gs_bfly(x[r], x[r + 2], zinv_m(4 + r / 4));
#pragma unroll
  for (int r = 0; r < 16; r++)
    if ((r & 4) == 0) gs_bfly(x[r], x[r + 4], zinv_m(2 + r / 8));
#pragma unroll
  for (int r = 0; r < 8; r++) {
    int32_t a = x[r], b = x[r + 8];
    x[r] = mont_mul(a + b, SCALE_M);
    x[r + 8] = mont_mul(a - b, zinv_scaled_m(1));
  }
}

// ---- strided load/store of a polynomial in global memory ----
__device__ __forceinline__ void load_strided(int32_t x[16], const int32_t *p, int t) {
#pragma unroll
  for (int r = 0; r < 16; r++) x[r] = p[t + 16 * r];
}
__device__ __forceinline__ void store_strided(const int32_t x[16], int32_t *p, int t) {
#pragma unroll
  for (int r = 0; r < 16; r++) p[t + 16 * r] = x[r];
}
// slots layout: lane t owns 16 consecutive words -> four 16-byte accesses
__device__ __forceinline__ void load_slots(int32_t x[16], const int32_t *p, int t) {
  const int4 *q = (const int4 *)(p + 16 * t);
#pragma unroll
  for (int v = 0; v < 4; v++) {
    int4 u = q[v];
    x[4 * v] = u.x; x[4 * v + 1] = u.y; x[4 * v + 2] = u.z; x[4 * v + 3] = u.w;
  }
}
__device__ __forceinline__ void store_slots(const int32_t x[16], int32_t *p, int t) {
  int4 *q = (int4 *)(p + 16 * t);
#pragma unroll
  for (int v = 0; v < 4; v++) q[v] = make_int4(x[4 * v], x[4 * v + 1], x[4 * v + 2], x[4 * v + 3]);
}

}  // namespace dil
