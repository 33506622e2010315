// Coefficient-wise operations (Sec. 2.3 "Bits Extraction and Hints"), norm
// checks (Alg. 2 rejection conditions) and packing helpers for gfx950.
// Every function works on canonical coefficients in [0, q) unless noted.
#pragma once
#include "common.h"

namespace dil {

// Decompose(r, 2 gamma2) for canonical r: r0 = r mod+- alpha, r1 = (r - r0)/alpha,
// with the special case r - r0 = q - 1 mapped to (0, r0 - 1).  r1 is
// ceil((r - gamma2) / alpha) = floor((r + gamma2 - 1) / alpha); the special case
// is exactly r1 == (q-1)/alpha.
template <int LV>
__device__ __forceinline__ void decompose(int32_t r, int32_t &r1, int32_t &r0) {
  constexpr uint32_t G2 = Lv<LV>::GAMMA2, ALPHA = 2 * G2, M = (Q - 1) / ALPHA;
  uint32_t a1 = ((uint32_t)r + G2 - 1) / ALPHA;
  int32_t a0 = r - (int32_t)(a1 * ALPHA);
  if (a1 == M) {
    a1 = 0;
    a0 -= 1;
  }
  r1 = (int32_t)a1;
  r0 = a0;
}
template <int LV>
__device__ __forceinline__ int32_t highbits(int32_t r) {
  int32_t r1, r0;
  decompose<LV>(r, r1, r0);
  return r1;
}
template <int LV>
__device__ __forceinline__ int32_t use_hint(int32_t h, int32_t r) {
  constexpr int32_t M = (Q - 1) / (2 * Lv<LV>::GAMMA2);
  int32_t r1, r0;
  decompose<LV>(r, r1, r0);
  if (!h) return r1;
  if (r0 > 0) return r1 + 1 == M ? 0 : r1 + 1;
  return r1 == 0 ? M - 1 : r1 - 1;
}
// Power2Round with d = 13: r0 = r mod+- 2^13, r1 = (r - r0) / 2^13
__device__ __forceinline__ void power2round(int32_t r, int32_t &r1, int32_t &r0) {
  r1 = (r + (1 << (D - 1)) - 1) >> D;
  r0 = r - (r1 << D);
}
// ||x||_inf >= B for canonical x (B < q/2): centred value c has |c| >= B iff B <= x <= q - B
__device__ __forceinline__ bool norm_ge(int32_t x, int32_t B) {
  return (uint32_t)(x - B) <= (uint32_t)(Q - 2 * B);
}
// centred representative of a canonical value
__device__ __forceinline__ int32_t centred(int32_t x) { return x > (Q - 1) / 2 ? x - Q : x; }

// ---- wave-level helpers (one task per wavefront) ----
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- byte movement between global memory and LDS ----
// Copy NB bytes from global (any alignment) into LDS words (4-aligned,
// zero-padded to a whole word) with one wavefront.  Only aligned global words
// that contain a requested byte are read, and every lane issues all of its
// loads before its first LDS store: one memory round trip for the whole copy.
template <int NB>
__device__ __forceinline__ void g2l_bytes(const uint8_t *g, uint32_t *lw, int lane) {
  constexpr int NWD = (NB + 3) / 4, PER = (NWD + 63) / 64;
  const uintptr_t base = (uintptr_t)g;
  const int mis = (int)(base & 3);
  const uint32_t *gw = (const uint32_t *)(base - mis);
  const uintptr_t last_word = (base + NB - 1) >> 2;  // aligned word index of the last valid byte
  uint32_t lo[PER], hi[PER];
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const int i = lane + 64 * q;
    const bool in = i < NWD;
    lo[q] = in ? gw[i] : 0u;
    hi[q] = in && mis && (((uintptr_t)(gw + i + 1)) >> 2) <= last_word ? gw[i + 1] : 0u;
  }
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const int i = lane + 64 * q;
    if (i < NWD) {
      uint32_t v = mis ? __builtin_amdgcn_alignbit(hi[q], lo[q], 8 * mis) : lo[q];
      const int rem = NB - 4 * i;
      if (rem < 4) v &= (1u << (8 * rem)) - 1u;
      lw[i] = v;
    }
  }
}
// Copy NW aligned 32-bit words from global into LDS with one wavefront, all
// loads issued before the first store.
template <int NW>
__device__ __forceinline__ void g2l_words(const uint32_t *g, uint32_t *l, int lane) {
  constexpr int PER = (NW + 63) / 64;
  uint32_t v[PER];
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const int i = lane + 64 * q;
    v[q] = i < NW ? g[i] : 0u;
  }
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const int i = lane + 64 * q;
    if (i < NW) l[i] = v[q];
  }
}
// Copy nbytes of LDS (starting at a 4-aligned LDS byte address) to global (any alignment).
__device__ __forceinline__ void l2g_bytes(const uint32_t *lw, int nbytes, uint8_t *g, int lane, int nlanes) {
  const uint8_t *lb = (const uint8_t *)lw;
  uintptr_t base = (uintptr_t)g;
  int head = (int)((4 - (base & 3)) & 3);
  if (head > nbytes) head = nbytes;
  if (lane < head) g[lane] = lb[lane];
  int body = (nbytes - head) >> 2;
  uint32_t *gw = (uint32_t *)(g + head);
  for (int i = lane; i < body; i += nlanes) {
    int o = head + 4 * i;
    uint32_t v = (uint32_t)lb[o] | ((uint32_t)lb[o + 1] << 8) | ((uint32_t)lb[o + 2] << 16) | ((uint32_t)lb[o + 3] << 24);
    gw[i] = v;
  }
  int done = head + 4 * body;
  if (lane < nbytes - done) g[done + lane] = lb[done + lane];
}

// b-bit field number c of a little-endian bit stream held in 32-bit words
template <int B>
__device__ __forceinline__ uint32_t field(const uint32_t *w, int c) {
  int p = c * B;
  int i = p >> 5, s = p & 31;
  uint32_t v = __builtin_amdgcn_alignbit(w[i + 1], w[i], s);
  return v & ((1u << B) - 1u);
}
// unpack the strided coefficients of the lane (t + 16 r) from packed words in LDS
template <int B>
__device__ __forceinline__ void unpack_strided(const uint32_t *w, uint32_t v[16], int t) {
#pragma unroll
  for (int r = 0; r < 16; r++) v[r] = field<B>(w, t + 16 * r);
}

// Pack 16 consecutive B-bit values (the lane's coefficients 16t..16t+15) into
// the LDS byte stream at bit offset 16*B*t.  The lane's bits occupy exactly the
// 2B bytes starting at byte 2B*t, so lanes never share a byte.
template <int B>
__device__ __forceinline__ void pack16_to_lds(const uint32_t v[16], uint8_t *dst, int t) {
  uint32_t words[(16 * B + 31) / 32];
#pragma unroll
  for (int i = 0; i < (16 * B + 31) / 32; i++) words[i] = 0;
#pragma unroll
  for (int j = 0; j < 16; j++) {
    int p = j * B;  // compile-time after unrolling
    int i = p >> 5, s = p & 31;
    words[i] |= v[j] << s;
    if (s + B > 32) words[i + 1] |= v[j] >> (32 - s);
  }
  uint8_t *d = dst + 2 * B * t;
  if constexpr ((2 * B) % 4 == 0) {
    uint32_t *dw = (uint32_t *)d;
#pragma unroll
    for (int i = 0; i < (2 * B) / 4; i++) dw[i] = words[i];
  } else {
    // 2B is a multiple of 2: write halfwords
    uint16_t *dh = (uint16_t *)d;
#pragma unroll
    for (int i = 0; i < B; i++) dh[i] = (uint16_t)(words[i >> 1] >> (16 * (i & 1)));
  }
}

}  // namespace dil
