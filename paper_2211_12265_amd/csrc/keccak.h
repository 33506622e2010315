// Keccak-f[1600] and SHAKE128/256 sponges for gfx950, one sponge per lane.
//
// The paper's hash design (Sec. 3.3) spreads one state over 25 threads of a
// warp and exchanges lanes with shuffles every round.  On gfx950 a cross-lane
// exchange costs an LDS-crossbar operation per 32-bit half, while every step
// of the permutation is plain per-lane ALU work; the batched path always has
// thousands of independent sponges (k*l ExpandA streams and l ExpandMask
// streams per task, one hash chain per task), so each lane keeps a whole
// 1600-bit state in 50 VGPRs and the wavefront exchanges nothing.  The round
// uses gfx950's three-input bit operation (v_bitop3_b32) for the five-way
// column parities, the theta update and chi, and v_alignbit_b32 for the
// 64-bit rotations on 32-bit halves.
//
// State layout: s[2*i] / s[2*i+1] = low / high 32 bits of lane i = x + 5y,
// bytes little-endian within a lane (FIPS 202).
#pragma once
#include "common.h"

namespace dil {

// ---- constants derived from FIPS 202 at compile time ----
constexpr int kc_rc_bit(int t) {
  if (t % 255 == 0) return 1;
  unsigned R = 1;
  for (int i = 1; i <= t % 255; i++) {
    R <<= 1;
    unsigned r8 = (R >> 8) & 1;
    R ^= r8 | (r8 << 4) | (r8 << 5) | (r8 << 6);
    R &= 0xFF;
  }
  return R & 1;
}
constexpr uint64_t kc_rc(int ir) {
  uint64_t rc = 0;
  for (int j = 0; j <= 6; j++)
    if (kc_rc_bit(j + 7 * ir)) rc |= (uint64_t)1 << ((1 << j) - 1);
  return rc;
}
constexpr int kc_rho(int lane) {  // rotation offset of lane x + 5y
  int x = 1, y = 0;
  for (int t = 0; t < 24; t++) {
    if (x + 5 * y == lane) return ((t + 1) * (t + 2) / 2) % 64;
    int nx = y, ny = (2 * x + 3 * y) % 5;
    x = nx;
    y = ny;
  }
  return 0;
}
// pi: lane (x, y) moves to (y, 2x + 3y)
constexpr int kc_pi_dst(int lane) {
  int x = lane % 5, y = lane / 5;
  return y + 5 * ((2 * x + 3 * y) % 5);
}

struct KRC {
  uint32_t lo[24], hi[24];
  constexpr KRC() : lo(), hi() {
    for (int i = 0; i < 24; i++) {
      lo[i] = (uint32_t)kc_rc(i);
      hi[i] = (uint32_t)(kc_rc(i) >> 32);
    }
  }
};
__constant__ constexpr KRC kKRC = KRC();

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);  // a ^ b ^ c
}
__device__ __forceinline__ uint32_t chi3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xD2);  // a ^ (~b & c)
}
// 64-bit rotate-left of (lo, hi) by compile-time n
template <int n>
__device__ __forceinline__ void rotl64(uint32_t lo, uint32_t hi, uint32_t &olo, uint32_t &ohi) {
  if constexpr (n == 0) {
    olo = lo; ohi = hi;
  } else if constexpr (n == 32) {
    olo = hi; ohi = lo;
  } else if constexpr (n < 32) {
    ohi = __builtin_amdgcn_alignbit(hi, lo, 32 - n);
    olo = __builtin_amdgcn_alignbit(lo, hi, 32 - n);
  } else {
    ohi = __builtin_amdgcn_alignbit(lo, hi, 64 - n);
    olo = __builtin_amdgcn_alignbit(hi, lo, 64 - n);
  }
}

template <int lane>
__device__ __forceinline__ void kc_rhopi_one(const uint32_t *a, const uint32_t *c, const uint32_t *r, uint32_t *b) {
  constexpr int x = lane % 5;
  constexpr int xm = (x + 4) % 5;
  // theta folded in: a ^ C[x-1] ^ rotl1(C[x+1])
  uint32_t lo = xor3(a[2 * lane], c[2 * xm], r[2 * x]);
  uint32_t hi = xor3(a[2 * lane + 1], c[2 * xm + 1], r[2 * x + 1]);
  constexpr int dst = kc_pi_dst(lane);
  rotl64<kc_rho(lane)>(lo, hi, b[2 * dst], b[2 * dst + 1]);
}

template <int... L>
__device__ __forceinline__ void kc_rhopi_all(const uint32_t *a, const uint32_t *c, const uint32_t *r, uint32_t *b,
                                             std::integer_sequence<int, L...>) {
  (kc_rhopi_one<L>(a, c, r, b), ...);
}

__device__ __forceinline__ void keccak_round(uint32_t s[50], int ir) {
  uint32_t c[10], r[10], b[50];
#pragma unroll
  for (int x = 0; x < 5; x++) {
#pragma unroll
    for (int h = 0; h < 2; h++)
      c[2 * x + h] = xor3(xor3(s[2 * x + h], s[2 * (x + 5) + h], s[2 * (x + 10) + h]), s[2 * (x + 15) + h],
                          s[2 * (x + 20) + h]);
  }
#pragma unroll
  for (int x = 0; x < 5; x++) {
    int xp = (x + 1) % 5;
    // rotl by 1
    r[2 * x + 1] = __builtin_amdgcn_alignbit(c[2 * xp + 1], c[2 * xp], 31);
    r[2 * x] = __builtin_amdgcn_alignbit(c[2 * xp], c[2 * xp + 1], 31);
  }
  kc_rhopi_all(s, c, r, b, std::make_integer_sequence<int, 25>{});
#pragma unroll
  for (int y = 0; y < 5; y++)
#pragma unroll
    for (int x = 0; x < 5; x++)
#pragma unroll
      for (int h = 0; h < 2; h++)
        s[2 * (x + 5 * y) + h] =
            chi3(b[2 * (x + 5 * y) + h], b[2 * ((x + 1) % 5 + 5 * y) + h], b[2 * ((x + 2) % 5 + 5 * y) + h]);
  s[0] ^= kKRC.lo[ir];
  s[1] ^= kKRC.hi[ir];
}

__device__ __forceinline__ void keccak_f(uint32_t s[50]) {
#pragma unroll 1
  for (int ir = 0; ir < 24; ir++) keccak_round(s, ir);
}

__device__ __forceinline__ void keccak_zero(uint32_t s[50]) {
#pragma unroll
  for (int i = 0; i < 50; i++) s[i] = 0;
}

// ---- byte-stream helpers ----
// Little-endian load of n (1..8) bytes at p that may be unaligned.  Only the
// aligned 8-byte words that hold at least one of the requested bytes are read,
// so the access never leaves the page of a valid byte.
__device__ __forceinline__ uint64_t load_le_bytes(const uint8_t *p, int n) {
  uintptr_t a = (uintptr_t)p;
  int off = (int)(a & 7);
  const uint64_t *w = (const uint64_t *)(a - off);
  uint64_t v = w[0] >> (8 * off);
  if (off + n > 8) v |= w[1] << (64 - 8 * off);
  if (n < 8) v &= (((uint64_t)1) << (8 * n)) - 1;
  return v;
}

}  // namespace dil
