// SHAKE128/256 sponges over byte sources, and the per-lane samplers
// (Sec. 2.3 "Sampling"; Alg. 1 ExpandA/ExpandS, Alg. 2 ExpandMask/SampleInBall).
// Each lane runs its own sponge (see keccak.h).
#pragma once
#include "keccak.h"
#include "poly.h"

namespace dil {

constexpr int RATE128 = 168, RATE256 = 136;

// Absorb a message of `len` bytes into a zeroed state and apply SHAKE padding
// (suffix 1111 then 10*1).  `word(pos)` must return the little-endian 8-byte
// word of message bytes [pos, pos + 8), with bytes at or beyond `len` zero.
// On return the first output block is in s[0 .. RATE/4).
template <int RATE, class W>
__device__ __forceinline__ void shake_absorb(uint32_t s[50], uint64_t len, W word) {
  keccak_zero(s);
  uint64_t nblk = len / RATE + 1;
  for (uint64_t b = 0; b < nblk; b++) {
#pragma unroll
    for (int w = 0; w < RATE / 8; w++) {
      uint64_t pos = b * RATE + 8 * w;
      uint64_t v = pos < len ? word(pos) : 0;
      if (pos <= len && len < pos + 8) v ^= (uint64_t)0x1F << (8 * (len - pos));
      if (w == RATE / 8 - 1 && b == nblk - 1) v ^= (uint64_t)0x80 << 56;
      s[2 * w] ^= (uint32_t)v;
      s[2 * w + 1] ^= (uint32_t)(v >> 32);
    }
    keccak_f(s);
  }
}

// word source for one contiguous byte string (any alignment)
struct SrcBytes {
  const uint8_t *p;
  uint64_t len;
  __device__ __forceinline__ uint64_t operator()(uint64_t pos) const {
    uint64_t n = len - pos;
    return load_le_bytes(p + pos, n >= 8 ? 8 : (int)n);
  }
};
// ---- single-block absorption of the short fixed-size sampler seeds ----
// seed = 32-byte rho (word source) || two nonce bytes, SHAKE128
template <class W>
__device__ __forceinline__ void absorb_seed34(uint32_t s[50], W rho_word, uint32_t nonce16) {
  keccak_zero(s);
#pragma unroll
  for (int w = 0; w < 4; w++) {
    uint64_t v = rho_word(8 * w);
    s[2 * w] = (uint32_t)v;
    s[2 * w + 1] = (uint32_t)(v >> 32);
  }
  s[8] = nonce16 | (0x1Fu << 16);
  s[2 * (RATE128 / 8 - 1) + 1] ^= 0x80u << 24;
  keccak_f(s);
}
// seed = 64-byte rho' (8-byte aligned) || LE16 nonce, SHAKE256
__device__ __forceinline__ void absorb_seed66(uint32_t s[50], const uint8_t *rhop, uint32_t nonce16) {
  keccak_zero(s);
  const uint64_t *rp = (const uint64_t *)rhop;
#pragma unroll
  for (int w = 0; w < 8; w++) {
    uint64_t v = rp[w];
    s[2 * w] = (uint32_t)v;
    s[2 * w + 1] = (uint32_t)(v >> 32);
  }
  s[16] = (nonce16 & 0xFFFFu) | (0x1Fu << 16);
  s[2 * (RATE256 / 8 - 1) + 1] ^= 0x80u << 24;
  keccak_f(s);
}

// ExpandMask: y_i coefficients from the lane's SHAKE256 stream (absorbed and
// permuted once).  B-bit little-endian values v, coefficient gamma1 - v.
// Stores the 256 coefficients to out (natural order) four at a time.
template <int B, int32_t GAMMA1>
__device__ __forceinline__ void expand_mask_squeeze(uint32_t s[50], int32_t *out) {
  constexpr int HPB = RATE256 / 4;              // 34 halves per block
  constexpr int NBLK = (N * B / 8 + RATE256 - 1) / RATE256;  // 5
  uint32_t carry = 0;                           // last half of the previous block
  int32_t quad[4];
#pragma unroll
  for (int blk = 0; blk < NBLK; blk++) {
    if (blk > 0) keccak_f(s);
#pragma unroll
    for (int c = 0; c < N; c++) {
      // coefficient c is emitted in the block holding its last bit
      const int p0 = c * B, p1 = c * B + B - 1;
      const int end_blk = (p1 / 32) / HPB;
      if (end_blk == blk) {
        const int h0 = p0 / 32 - blk * HPB, h1 = p1 / 32 - blk * HPB, sh = p0 & 31;
        uint32_t lo = h0 < 0 ? carry : s[h0 < 0 ? 0 : h0];
        uint32_t hi = s[h1];
        uint32_t v = (h0 == h1) ? (lo >> sh) : __builtin_amdgcn_alignbit(hi, lo, sh);
        v &= (1u << B) - 1u;
        quad[c & 3] = GAMMA1 - (int32_t)v;
        if ((c & 3) == 3) ((int4 *)out)[c >> 2] = make_int4(quad[0], quad[1], quad[2], quad[3]);
      }
    }
    carry = s[HPB - 1];
  }
}

// ExpandS rejection sampling: nibbles (low then high) of the SHAKE256 stream;
// eta = 2 keeps v < 15 -> 2 - (v mod 5); eta = 4 keeps v < 9 -> 4 - v.
template <int ETA>
__device__ __forceinline__ void expand_s_squeeze(uint32_t s[50], int32_t *out) {
  int ctr = 0;
  for (;;) {
#pragma unroll
    for (int byte = 0; byte < RATE256; byte++) {
      uint32_t bv = (s[byte >> 2] >> (8 * (byte & 3))) & 0xFFu;
#pragma unroll
      for (int hlf = 0; hlf < 2; hlf++) {
        uint32_t v = hlf ? (bv >> 4) : (bv & 15u);
        bool ok;
        int32_t coef;
        if constexpr (ETA == 2) {
          ok = v < 15u;
          coef = 2 - (int32_t)(v - 5u * ((v * 13u) >> 6));  // v mod 5 for v < 15
        } else {
          ok = v < 9u;
          coef = 4 - (int32_t)v;
        }
        if (ok && ctr < N) out[ctr] = coef;
        ctr += ok;
      }
    }
    if (ctr >= N) break;
    keccak_f(s);
  }
}

}  // namespace dil
