// Host check of the message-representative block builder
// (paper_2211_12265_amd/csrc/msg_words.h), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_msg_words.py.
//
// For a prefix of PB bytes (32 or 64: tr; 66: tr || 0x00 || 0x00), every byte
// misalignment of M and every length from 0 to MAXLEN, it builds all SHAKE256
// input blocks the way the device absorption does (first block with the
// prefix words, later blocks with the next block's dwords fetched ahead) and
// compares them with the padded byte string prefix || M || 0x1F 0..0 | 0x80.
// M is placed in a heap buffer that holds exactly the dwords covering it (no
// buffer when M is empty), so the sanitizer reports any read outside them.
//
// usage: msg_words_replay PB MAXLEN
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "msg_words.h"

using namespace dil;

#define CHECK(c)                                                             \
  do {                                                                       \
    if (!(c)) {                                                              \
      fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c);        \
      abort();                                                               \
    }                                                                        \
  } while (0)

template <int PB>
static void blocks(const uint32_t *pre, const uint8_t *msg, uint64_t mlen, std::vector<uint8_t> &out) {
  using Plan = MwPlan<PB>;
  constexpr int PW = Plan::PW, DL = Plan::DL;
  const Plan pl(msg, mlen);
  uint32_t D0[MW_WPB - PW + 1], Dn[MW_WPB + 1], blk[MW_WPB];
  auto emit = [&]() {
    for (int j = 0; j < MW_WPB; j++)
      for (int b = 0; b < 4; b++) out.push_back((uint8_t)(blk[j] >> (8 * b)));
  };
  mw_fetch<MW_WPB - PW, DL>(D0, pl.base, pl.last, pl.sh, Plan::m0(0));
  if (pl.nblk > 1) mw_fetch<MW_WPB, DL>(Dn, pl.base, pl.last, pl.sh, Plan::m0(1));
  for (int j = 0; j < MW_WPB; j++) blk[j] = mw_word<PW, DL>(j, pre, D0, pl.fs, pl.r0(0), pl.nblk == 1);
  emit();
  for (uint64_t b = 1; b < pl.nblk; b++) {
    uint32_t Dc[MW_WPB + 1];
    memcpy(Dc, Dn, sizeof Dc);
    if (b + 1 < pl.nblk) mw_fetch<MW_WPB, DL>(Dn, pl.base, pl.last, pl.sh, Plan::m0(b + 1));
    for (int j = 0; j < MW_WPB; j++) blk[j] = mw_word<0, DL>(j, pre, Dc, pl.fs, pl.r0(b), b == pl.nblk - 1);
    emit();
  }
}

template <int PB>
static uint64_t run(int maxlen) {
  constexpr int PW = PB / 4;
  uint32_t pre[PW];
  uint64_t rng = 0x9E3779B97F4A7C15ULL * PB;
  auto next = [&]() {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
  };
  for (int i = 0; i < PW; i++) pre[i] = (uint32_t)next();
  uint64_t checked = 0;
  for (int sh = 0; sh < 4; sh++)
    for (int mlen = 0; mlen <= maxlen; mlen++) {
      const size_t dwords = mlen ? (size_t)((sh + mlen - 1) / 4 + 1) : 0;
      uint32_t *hull = dwords ? (uint32_t *)malloc(dwords * 4) : nullptr;
      uint8_t *msg = hull ? (uint8_t *)hull + sh : (uint8_t *)&pre[0] + sh;  // never read when M is empty
      if (hull)
        for (size_t i = 0; i < dwords * 4; i++) ((uint8_t *)hull)[i] = (uint8_t)next();
      std::vector<uint8_t> want;
      for (int i = 0; i < PW; i++)
        for (int b = 0; b < 4; b++) want.push_back((uint8_t)(pre[i] >> (8 * b)));
      for (int i = 0; i < PB % 4; i++) want.push_back(0);
      for (int i = 0; i < mlen; i++) want.push_back(msg[i]);
      want.push_back(0x1F);
      while (want.size() % MW_RATE) want.push_back(0);
      want.back() ^= 0x80;
      std::vector<uint8_t> got;
      blocks<PB>(pre, msg, (uint64_t)mlen, got);
      CHECK(got.size() == want.size());
      if (got != want) {
        fprintf(stderr, "PB=%d sh=%d mlen=%d: blocks differ\n", PB, sh, mlen);
        abort();
      }
      free(hull);
      checked++;
    }
  return checked;
}

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s PB MAXLEN\n", argv[0]);
    return 2;
  }
  const int pb = atoi(argv[1]), maxlen = atoi(argv[2]);
  uint64_t n;
  if (pb == 32) n = run<32>(maxlen);
  else if (pb == 64) n = run<64>(maxlen);
  else if (pb == 66) n = run<66>(maxlen);
  else return 2;
  printf("ok PB=%d cases=%llu\n", pb, (unsigned long long)n);
  return 0;
}
