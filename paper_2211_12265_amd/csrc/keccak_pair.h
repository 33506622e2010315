// Keccak-f[1600] and SHAKE256 with one state on two adjacent lanes, for the
// hash chains that have too few independent sponges to keep a wavefront's
// lanes busy: the challenge hash of a Sign candidate (one per slot, after the
// slots' w) and Verify's final hash (one per task).  The paper spreads a state
// over a warp's threads for the same reason (Sec. 3.3); on gfx950 the split
// that pays is the smallest one.
//
// Lane 2p holds the low 32 bits of each of the 25 64-bit state words, lane
// 2p + 1 the high 32 bits ("half" 0 and 1).  A 64-bit rotation by n then needs
// the partner's half of the same word, taken with one DPP lane swap
// (quad_perm [1, 0, 3, 2]) and merged with one v_alignbit_b32, the same
// instruction for both halves:
//   n < 32:  alignbit(mine, partner's, 32 - n);  n > 32:  alignbit(partner's, mine, 64 - n).
// A round is 120 VALU instructions per lane (five column parities, theta with
// rho and pi, chi, iota) against 180 for a whole state in one lane, so the
// sequential chain of permutations is 1.5x shorter.  Both lanes of a pair must
// be active together; different pairs may diverge.
#pragma once
#include "sponge.h"

namespace dil {

__device__ __forceinline__ uint32_t pair_swap(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);
}

template <int n>
__device__ __forceinline__ uint32_t rotl_pair(uint32_t mine, uint32_t other) {
  if constexpr (n == 0) return mine;
  else if constexpr (n == 32) return other;
  else if constexpr (n < 32) return __builtin_amdgcn_alignbit(mine, other, 32 - n);
  else return __builtin_amdgcn_alignbit(other, mine, 64 - n);
}

template <int lane>
__device__ __forceinline__ void kp_rhopi_one(const uint32_t *a, const uint32_t *c, const uint32_t *r, uint32_t *b) {
  constexpr int x = lane % 5;
  constexpr int n = kc_rho(lane);
  const uint32_t e = xor3(a[lane], c[(x + 4) % 5], r[x]);  // theta
  if constexpr (n == 0) b[kc_pi_dst(lane)] = e;
  else b[kc_pi_dst(lane)] = rotl_pair<n>(e, pair_swap(e));
}

template <int... L>
__device__ __forceinline__ void kp_rhopi_all(const uint32_t *a, const uint32_t *c, const uint32_t *r, uint32_t *b,
                                             std::integer_sequence<int, L...>) {
  (kp_rhopi_one<L>(a, c, r, b), ...);
}

// a[i] = this lane's half of state word i = x + 5y
__device__ __forceinline__ void keccak_f_pair(uint32_t a[25], int half) {
  const uint32_t hmask = 0u - (uint32_t)half;  // selects the round constant's high word on odd lanes
#pragma unroll 1
  for (int ir = 0; ir < 24; ir++) {
    uint32_t c[5], r[5], b[25];
#pragma unroll
    for (int x = 0; x < 5; x++) c[x] = xor3(xor3(a[x], a[x + 5], a[x + 10]), a[x + 15], a[x + 20]);
#pragma unroll
    for (int x = 0; x < 5; x++) {
      const uint32_t cx = c[(x + 1) % 5];
      r[x] = rotl_pair<1>(cx, pair_swap(cx));
    }
    kp_rhopi_all(a, c, r, b, std::make_integer_sequence<int, 25>{});
#pragma unroll
    for (int y = 0; y < 5; y++)
#pragma unroll
      for (int x = 0; x < 5; x++)
        a[x + 5 * y] = chi3(b[x + 5 * y], b[(x + 1) % 5 + 5 * y], b[(x + 2) % 5 + 5 * y]);
    const uint32_t lo = kKRC.lo[ir], hi = kKRC.hi[ir];  // uniform loads
    a[0] ^= lo ^ ((lo ^ hi) & hmask);
  }
}

// SHAKE256 absorption of a LEN-byte message (LEN a multiple of 8) into a
// zeroed pair state with the SHAKE padding; word32(pos) returns this lane's
// half of the message's 8-byte word at byte pos.  On return the first output
// block is in the pairs' a[0 .. 17).
template <int LEN, class W>
__device__ __forceinline__ void shake256_absorb_pair(uint32_t a[25], int half, W word32) {
  static_assert(LEN % 8 == 0, "whole 8-byte words");
  constexpr int RATE = 136, NBLK = LEN / RATE + 1;
#pragma unroll
  for (int i = 0; i < 25; i++) a[i] = 0;
  for (int blk = 0; blk < NBLK; blk++) {
#pragma unroll
    for (int w = 0; w < RATE / 8; w++) {
      const int pos = blk * RATE + 8 * w;
      uint32_t v = pos < LEN ? word32(pos) : 0u;
      if (pos == LEN && !half) v ^= 0x1Fu;                         // suffix 1111 + first pad bit
      if (w == RATE / 8 - 1 && blk == NBLK - 1 && half) v ^= 0x80u << 24;  // last pad bit
      a[w] ^= v;
    }
    keccak_f_pair(a, half);
  }
}

// tr || M absorption, one SHAKE256 block at a time: PRE leading words of tr
// (8 in the first block, 0 after), then message words from message byte m0 on.
// A block's message part is fetched as the aligned dwords that cover it (NW + 1
// for NW message words), with addresses clamped to M's last dword (no dword
// outside [M's first, M's last] is read; none at all when M is empty).
template <int NW>
__device__ __forceinline__ void tr_msg_fetch(uint32_t D[NW + 1], const uint32_t *base, int64_t last, uint32_t sh,
                                             int64_t m0) {
  const int64_t d0 = (int64_t)((sh + (uint64_t)m0) >> 2);
  // dwords from d0 on, clamped to the last one (a 32-bit offset from d0)
  const int64_t span = last - d0;
  const int dl = span < 0 ? 0 : span > NW ? NW : (int)span;
  const uint32_t *b0 = base + (last >= 0 ? (d0 > last ? last : d0) : 0);
#pragma unroll
  for (int i = 0; i < NW + 1; i++) D[i] = last >= 0 ? b0[i < dl ? i : dl] : 0u;
}
// The fetched dwords are funnel-shifted by the byte misalignment sh, bytes past
// the end of M masked, the padding added arithmetically, the lane's half of
// each 8-byte word absorbed into the pair state and the block permuted.  Both
// lanes of a pair build the whole block (their loads hit the same addresses).
// All indices are compile-time so the words stay in registers.
template <int PRE>
__device__ __forceinline__ void tr_msg_mix(uint32_t a[25], int half, const uint32_t tr[8],
                                           const uint32_t D[RATE256 / 4 - PRE + 1], uint32_t sh, int64_t m0,
                                           uint64_t mlen, bool final_block) {
  constexpr int WPB = RATE256 / 4;  // 34 words per block
  // message bytes left at the block's first message word, clamped to a small
  // range that keeps every per-word test below exact
  const int64_t r64 = (int64_t)mlen - m0;
  const int r0 = r64 < 0 ? -4 : r64 > 4 * WPB ? 4 * WPB + 4 : (int)r64;
#pragma unroll
  for (int j = 0; j < WPB; j++) {
    uint32_t v;
    if (j < PRE) {
      v = tr[j];
    } else {
      const int k = j - PRE;
      v = __builtin_amdgcn_alignbit(D[k + 1], D[k], 8 * sh);
      const int rem = r0 - 4 * k;  // message bytes left from this word on
      v = rem <= 0 ? 0u : rem < 4 ? v & ((1u << (8 * rem)) - 1u) : v;
      if (rem >= 0 && rem < 4) v ^= 0x1Fu << (8 * rem);   // SHAKE suffix right after M
    }
    if (j == WPB - 1 && final_block) v ^= 0x80u << 24;    // final bit of the 10*1 padding
    a[j >> 1] ^= (j & 1) == half ? v : 0u;
  }
  keccak_f_pair(a, half);
}

// SHAKE256 absorption of tr || M, for mu = H(tr || M): tr is 32 bytes given as
// eight little-endian words, M is mlen bytes at any alignment.  Lanes hash
// messages of different lengths, so nothing per word depends on a branch.
// Block b >= 1 carries message bytes from 136 b - 32 on, a multiple of 4, so
// one funnel shift serves every block; the next block's dwords are requested
// before the current block is permuted, so their latency overlaps it.  On
// return the first output block is in the pairs' a[0 .. 17).
__device__ __forceinline__ void absorb_tr_msg(uint32_t a[25], int half, const uint32_t tr[8], const uint8_t *msg,
                                              uint64_t mlen) {
  constexpr int WPB = RATE256 / 4;
#pragma unroll
  for (int i = 0; i < 25; i++) a[i] = 0;
  const uint32_t sh = (uint32_t)((uintptr_t)msg & 3u);
  const uint32_t *base = (const uint32_t *)(msg - sh);
  const int64_t last = mlen ? (int64_t)((sh + mlen - 1) >> 2) : -1;  // last dword holding message bytes
  const uint64_t nblk = (32 + mlen) / RATE256 + 1;
  uint32_t D0[WPB - 8 + 1], Dn[WPB + 1];
  tr_msg_fetch<WPB - 8>(D0, base, last, sh, 0);
  if (nblk > 1) tr_msg_fetch<WPB>(Dn, base, last, sh, RATE256 - 32);
  tr_msg_mix<8>(a, half, tr, D0, sh, 0, mlen, nblk == 1);
  for (uint64_t b = 1; b < nblk; b++) {
    uint32_t Dc[WPB + 1];
#pragma unroll
    for (int i = 0; i < WPB + 1; i++) Dc[i] = Dn[i];
    if (b + 1 < nblk) tr_msg_fetch<WPB>(Dn, base, last, sh, (int64_t)(b + 1) * RATE256 - 32);
    tr_msg_mix<0>(a, half, tr, Dc, sh, (int64_t)b * RATE256 - 32, mlen, b == nblk - 1);
  }
}

// SampleInBall (Sec. 2.3) on a pair whose state holds the first SHAKE256
// block of ctilde: the block is staged in bw (34 words, both halves), the
// dense challenge built in c (256 bytes, 4-byte aligned) by the even lane;
// both lanes follow the same byte sequence, and permute together when a
// further block is needed.
template <int TAU>
__device__ __forceinline__ void sample_in_ball_pair(uint32_t a[25], int half, int8_t *c, uint32_t *bw) {
#pragma unroll
  for (int w = 0; w < 17; w++) bw[2 * w + half] = a[w];
  uint32_t *cw = (uint32_t *)c;
#pragma unroll
  for (int w = 0; w < N / 8; w++) cw[2 * w + half] = 0;
  wave_sync();
  const uint8_t *bytes = (const uint8_t *)bw;
  uint64_t signs = (uint64_t)bw[0] | ((uint64_t)bw[1] << 32);
  int pos = 8;
  for (int i = N - TAU; i < N; i++) {
    int b;
    for (;;) {
      if (pos == RATE256) {
        keccak_f_pair(a, half);
#pragma unroll
        for (int w = 0; w < 17; w++) bw[2 * w + half] = a[w];
        wave_sync();
        pos = 0;
      }
      b = bytes[pos++];
      if (b <= i) break;
    }
    if (!half) {
      c[i] = c[b];
      c[b] = (int8_t)(1 - 2 * (int)(signs & 1));
    }
    signs >>= 1;
  }
}

// ctilde = H(mu || w1) and c = SampleInBall(ctilde) on a lane pair; mu and w1
// rows 8-byte aligned.  ctilde_out: 8 words (both halves written).
template <int LV>
__device__ __forceinline__ void dev_challenge_pair(const uint8_t *mu, const uint8_t *w1, int half, uint32_t *ctilde_out,
                                                   int8_t *c, uint32_t *bw) {
  uint32_t a[25];
  shake256_absorb_pair<P<LV>::MUW1>(a, half, [&](int pos) {
    return pos < 64 ? *(const uint32_t *)(mu + pos + 4 * half) : *(const uint32_t *)(w1 + (pos - 64) + 4 * half);
  });
  uint32_t ct[4];
#pragma unroll
  for (int w = 0; w < 4; w++) {
    ct[w] = a[w];
    ctilde_out[2 * w + half] = a[w];
  }
  // SHAKE256(ctilde): 32 message bytes, then the padding
#pragma unroll
  for (int i = 0; i < 25; i++) a[i] = i < 4 ? ct[i] : 0u;
  if (!half) a[4] ^= 0x1Fu;
  else a[16] ^= 0x80u << 24;
  keccak_f_pair(a, half);
  sample_in_ball_pair<Lv<LV>::TAU>(a, half, c, bw);
}

}  // namespace dil
