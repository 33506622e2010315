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
#include "msg_words.h"
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

// One SHAKE256 block of X = prefix || M on a pair (msg_words.h builds the
// words): the first PRE words come from the prefix, the rest from the fetched
// message dwords D; each lane absorbs its half of every 8-byte word.  All
// indices are compile-time so the words stay in registers.
template <int PB, int PRE>
__device__ __forceinline__ void mw_mix(uint32_t a[25], int half, const uint32_t *pre, const uint32_t *D, uint32_t fs,
                                       int r0, bool final_block) {
#pragma unroll
  for (int j = 0; j < MW_WPB; j++) {
    const uint32_t v = mw_word<PRE, PB % 4>(j, pre, D, fs, r0, final_block);
    a[j >> 1] ^= (j & 1) == half ? v : 0u;
  }
  keccak_f_pair(a, half);
}

// SHAKE256 absorption of X = prefix || M for a message representative: the
// prefix is tr (PB = 32, mu = H(tr || M)) or tr || 0x00 || 0x00 (PB = 66,
// ML-DSA's mu with an empty context), given as PB / 4 little-endian words; M
// is mlen bytes at any alignment.  Lanes hash messages of different lengths,
// so nothing per word depends on a branch.  Both lanes of a pair build the
// whole block (their loads hit the same addresses); the next block's dwords
// are requested before the current block is permuted, so their latency
// overlaps it.  On return the first output block is in the pairs' a[0 .. 17).
template <int PB>
__device__ __forceinline__ void absorb_prefix_msg(uint32_t a[25], int half, const uint32_t pre[PB / 4],
                                                  const uint8_t *msg, uint64_t mlen) {
  using Plan = MwPlan<PB>;
  constexpr int PW = Plan::PW, DL = Plan::DL;
#pragma unroll
  for (int i = 0; i < 25; i++) a[i] = 0;
  const Plan pl(msg, mlen);
  uint32_t D0[MW_WPB - PW + 1], Dn[MW_WPB + 1];
  mw_fetch<MW_WPB - PW, DL>(D0, pl.base, pl.last, pl.sh, Plan::m0(0));
  if (pl.nblk > 1) mw_fetch<MW_WPB, DL>(Dn, pl.base, pl.last, pl.sh, Plan::m0(1));
  mw_mix<PB, PW>(a, half, pre, D0, pl.fs, pl.r0(0), pl.nblk == 1);
  for (uint64_t b = 1; b < pl.nblk; b++) {
    uint32_t Dc[MW_WPB + 1];
#pragma unroll
    for (int i = 0; i < MW_WPB + 1; i++) Dc[i] = Dn[i];
    if (b + 1 < pl.nblk) mw_fetch<MW_WPB, DL>(Dn, pl.base, pl.last, pl.sh, Plan::m0(b + 1));
    mw_mix<PB, 0>(a, half, pre, Dc, pl.fs, pl.r0(b), b == pl.nblk - 1);
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
// rows 8-byte aligned.  ctilde is CT bytes (32 in round 3; lambda / 4 =
// 32 / 48 / 64 for ML-DSA, whose SampleInBall absorbs all of it);
// ctilde_out: CT / 4 words (both halves written).
template <int LV>
__device__ __forceinline__ void dev_challenge_pair(const uint8_t *mu, const uint8_t *w1, int half, uint32_t *ctilde_out,
                                                   int8_t *c, uint32_t *bw) {
  constexpr int CW = P<LV>::CT / 8;  // 8-byte words of ctilde
  uint32_t a[25];
  shake256_absorb_pair<P<LV>::MUW1>(a, half, [&](int pos) {
    return pos < 64 ? *(const uint32_t *)(mu + pos + 4 * half) : *(const uint32_t *)(w1 + (pos - 64) + 4 * half);
  });
  uint32_t ct[CW];
#pragma unroll
  for (int w = 0; w < CW; w++) {
    ct[w] = a[w];
    ctilde_out[2 * w + half] = a[w];
  }
  // SHAKE256(ctilde): CT message bytes, then the padding
#pragma unroll
  for (int i = 0; i < 25; i++) a[i] = i < CW ? ct[i] : 0u;
  if (!half) a[CW] ^= 0x1Fu;
  else a[16] ^= 0x80u << 24;
  keccak_f_pair(a, half);
  sample_in_ball_pair<Lv<LV>::TAU>(a, half, c, bw);
}

}  // namespace dil
