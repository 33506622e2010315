// The SHAKE256 input blocks of a message representative, X = prefix || M,
// built word by word from the message bytes in memory: mu = H(tr || M) in
// round 3 (Alg. 2 and 3), mu = H(tr || 0x00 || 0x00 || M) in ML-DSA's pure
// form with an empty context and mu = H(tr || M') of a formatted message in
// its internal form (FIPS 204, which the paper does not cover).
//
// The prefix is PB bytes: PB / 4 whole words given by the caller (tr), and
// DL = PB % 4 zero bytes in the word where M begins (PB = 32 or 64: DL = 0;
// PB = 66: DL = 2).  M has any length and any byte alignment.  Each 136-byte block
// is 34 little-endian words; its message words are fetched as the aligned
// dwords that cover them and funnel-shifted by one constant amount, bytes
// past the end of M are masked, and the SHAKE suffix and padding are added
// arithmetically, so lanes hashing messages of different lengths follow one
// instruction stream.  No dword outside the aligned hull of M (the dwords
// holding its first and last bytes) is read, and none at all when M is
// empty.
//
// Written without device intrinsics (the funnel shift aside, which has a
// portable form) so that a host test can build every block for all
// alignments and lengths under AddressSanitizer and compare it with the
// definition.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "batch_sched.h"  // DIL_HD

namespace dil {

constexpr int MW_RATE = 136;          // SHAKE256 rate in bytes
constexpr int MW_WPB = MW_RATE / 4;   // 34 words per block

// bytes [s, s + 4) of the 8-byte little-endian value hi:lo, s in 0..3 bytes
DIL_HD uint32_t mw_funnel(uint32_t hi, uint32_t lo, uint32_t s) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_alignbit(hi, lo, 8 * s);
#else
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> (8 * s));
#endif
}

// Fetch the NW + 1 dwords from which a block's NW message words are built:
// the words start at message byte m0 (m0 = -DL for the first block, where the
// word also holds the prefix's last DL bytes).  D[i] is the dword i after the
// one holding byte m0; dwords outside [first, last] of M are clamped to it
// (their bytes are masked later), and the dword before M that the first
// block's word would touch is never read (D[0] = 0 then).  base is M's
// address rounded down to 4 bytes, sh = M's misalignment, last = index of the
// dword holding M's last byte (-1: M empty).
template <int NW, int DL>
DIL_HD void mw_fetch(uint32_t D[NW + 1], const uint32_t *base, int64_t last, uint32_t sh, int64_t m0) {
  const int64_t d0 = ((int64_t)sh + m0) >> 2;  // floor: -1 only when the word starts in the prefix before M
  const bool before = DL != 0 && d0 < 0;
  const int64_t f = before ? 0 : d0;           // first dword fetched
  const int64_t span = last - f;
  const int dl = span < 0 ? 0 : span > NW ? NW : (int)span;
  const uint32_t *b0 = base + (last >= 0 ? (f > last ? last : f) : 0);
  uint32_t E[NW + 1];
#pragma unroll
  for (int i = 0; i < NW + 1; i++) E[i] = last >= 0 ? b0[i < dl ? i : dl] : 0u;
  if constexpr (DL != 0) {
#pragma unroll
    for (int i = NW; i >= 0; i--) D[i] = before ? (i ? E[i - 1] : 0u) : E[i];
  } else {
#pragma unroll
    for (int i = 0; i < NW + 1; i++) D[i] = E[i];
  }
}

// Word j (0..33) of a block whose first PRE words are prefix words (PRE = PB / 4
// in the first block, 0 after) and whose message words start at message byte
// m0.  fs = (sh + m0) & 3, the same for every block; r0 = message bytes left
// at m0, clamped to {-4} u [0, 4 * 34 + 4] so that every per-word test stays
// exact.  final_block adds the last padding bit.
template <int PRE, int DL>
DIL_HD uint32_t mw_word(int j, const uint32_t *pre, const uint32_t *D, uint32_t fs, int r0, bool final_block) {
  uint32_t v;
  if (j < PRE) {
    v = pre[j];
  } else {
    const int k = j - PRE;
    v = mw_funnel(D[k + 1], D[k], fs);
    const int rem = r0 - 4 * k;  // message bytes left from this word on
    v = rem <= 0 ? 0u : rem < 4 ? v & ((1u << (8 * rem)) - 1u) : v;
    if (DL != 0 && PRE != 0 && k == 0) v &= ~((1u << (8 * DL)) - 1u);  // the prefix's zero bytes
    if (rem >= 0 && rem < 4) v ^= 0x1Fu << (8 * rem);                    // SHAKE suffix right after M
  }
  if (j == MW_WPB - 1 && final_block) v ^= 0x80u << 24;  // final bit of the 10*1 padding
  return v;
}

// Geometry of X = prefix(PB) || M: blocks, and the message byte at which
// block b's message words start.
template <int PB>
struct MwPlan {
  static constexpr int PW = PB / 4, DL = PB % 4;
  static_assert(DL == 0 || DL == 2, "prefix ends on a word or half-word boundary");
  static_assert(PB + 8 <= MW_RATE, "the prefix fits the first block with a message word to spare");
  uint32_t sh, fs;
  const uint32_t *base;
  int64_t last;
  uint64_t nblk, mlen;
  DIL_HD MwPlan(const uint8_t *msg, uint64_t len) {
    sh = (uint32_t)((uintptr_t)msg & 3u);
    fs = (sh - (uint32_t)DL) & 3u;
    base = (const uint32_t *)(msg - sh);
    last = len ? (int64_t)((sh + len - 1) >> 2) : -1;
    nblk = (PB + len) / MW_RATE + 1;
    mlen = len;
  }
  DIL_HD static int64_t m0(uint64_t b) { return b == 0 ? -(int64_t)DL : (int64_t)b * MW_RATE - PB; }
  DIL_HD int r0(uint64_t b) const {
    const int64_t r = (int64_t)mlen - m0(b);
    return r < 0 ? -4 : r > 4 * MW_WPB + 4 ? 4 * MW_WPB + 4 : (int)r;
  }
};

}  // namespace dil
