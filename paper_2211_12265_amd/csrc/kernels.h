// Batched Dilithium kernels for gfx950 (Alg. 1-3), one-launch-per-stage form.
//
// Thread mappings:
//   sponge kernels      one lane per SHAKE stream (256-thread blocks)
//   polynomial kernels  one wavefront per task, four 16-lane groups each
//                       working on its own polynomial (64-thread blocks)
// All intermediates live in a per-task workspace in HBM (see Ws).
#pragma once
#include "common.h"
#include "ntt.h"
#include "poly.h"
#include "sponge.h"
#include "keccak_pair.h"

namespace dil {

// Per-task workspace of the staged kernels.  Rows are 256-byte aligned; the
// hash inputs mu || packed w1 are stored contiguously, in the order the hash
// consumes them, so the challenge hash reads one row.
struct Ws {
  uint8_t *muw1;     // [cap][MUW1 rounded to 256]
  uint8_t *rhop;     // [cap][64]   rho' (KeyGen: expanded secret seed; Sign: mask seed)
  uint8_t *ctilde;   // [cap][CT_STRIDE]
  int8_t *cpoly;     // [cap][256]  challenge c, dense
  int32_t *A;        // [cap][K][L][256]  A-hat, canonical
  int32_t *s1h;      // [cap][L][256]  NTT(s1)   (KeyGen: s1, s2 centred, [cap][L+K][256])
  int32_t *s2h;      // [cap][K][256]
  int32_t *t0h;      // [cap][K][256]
  int32_t *y;        // [cap][L][256]  mask, centred
  int32_t *w;        // [cap][K][256]  w = A y, canonical
  uint32_t *hmask;   // [cap][K][8]   verify: hint bits
  uint32_t *kappa;   // [cap]
  int32_t *flag;     // [cap]
  uint32_t *active0, *active1;  // [cap] task lists
  uint32_t *counters;           // [8]: next active count, error flags, attempts
  size_t cap;
  size_t muw1_stride;
  // Resident key tables: when kmap is set, A, s1h, s2h, t0h (and t1h, tr) are
  // indexed by key row kmap[task] instead of by task.
  const uint32_t *kmap;
  const int32_t *t1h;   // [keys][K][256] NTT(t1 2^d), slots layout (verify), or null
  const uint8_t *tr;    // [keys][TRB] tr = H(pk) (verify), or null
};

constexpr int CT_STRIDE = 64;  // workspace row of a ctilde (the longest, ML-DSA-87's)

// bytes hashed before the message for mu: tr (round 3), tr || 0x00 || 0x00
// (ML-DSA, empty context) or tr alone before a formatted message (ML-DSA's
// internal form)
template <int LV, bool INTERNAL>
constexpr int mu_prefix_bytes() {
  static_assert(!INTERNAL || Lv<LV>::MLDSA, "formatted messages exist at the ML-DSA levels only");
  return !Lv<LV>::MLDSA ? 32 : INTERNAL ? 64 : 66;
}

// row of the per-key arrays used by task `task`
__device__ __forceinline__ size_t kix(const Ws &ws, uint32_t task) { return ws.kmap ? ws.kmap[task] : task; }

template <int LV>
__device__ __forceinline__ size_t muw1_stride() {
  return ((size_t)P<LV>::MUW1 + 255) & ~(size_t)255;
}

// zero two small word arrays (used instead of hipMemsetAsync so that the
// launch sequence can be captured into a hipGraph)
__global__ void zero_words_k(uint32_t *a, int na, uint32_t *b, int nb) {
  int i = threadIdx.x;
  if (i < na) a[i] = 0;
  if (b && i < nb) b[i] = 0;
}

// Key-table calls: copy key_idx into the workspace with every index outside
// the table replaced by row 0 and the error word set, so no later kernel reads
// past the table; the host reports the error at its next check.
__global__ void __launch_bounds__(256) keys_check_k(const uint32_t *key_idx, uint32_t nkeys, uint32_t *out,
                                                   uint32_t count, uint32_t *err) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t k = key_idx[i];
  if (k >= nkeys) {
    k = 0;
    *err = 1u;
  }
  out[i] = k;
}

// ------------------------------------------------------------------------
// KeyGen (Alg. 1)
// ------------------------------------------------------------------------
// (rho, rho', K) = H(zeta): rho -> pk and sk, K -> sk, rho' -> workspace.
// ML-DSA hashes xi || k || l (one byte each) instead of the bare seed.
template <int LV>
__global__ void __launch_bounds__(256) kg_seed_k(const uint8_t *seeds, uint8_t *pk, uint8_t *sk, Ws ws,
                                                 uint32_t count) {
  uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  uint32_t s[50];
  const uint8_t *sd = seeds + 32 * (size_t)t;
  shake_absorb<RATE256>(s, Lv<LV>::MLDSA ? 34 : 32, [&](uint64_t pos) -> uint64_t {
    return pos < 32 ? load_le_bytes(sd + pos, 8) : (uint64_t)Lv<LV>::K | ((uint64_t)Lv<LV>::L << 8);
  });
  uint64_t *pkw = (uint64_t *)(pk + (size_t)t * P<LV>::PK);
  uint64_t *skw = (uint64_t *)(sk + (size_t)t * P<LV>::SK);
  uint64_t *rw = (uint64_t *)(ws.rhop + (size_t)t * 64);
#pragma unroll
  for (int w = 0; w < 16; w++) {
    uint64_t v = (uint64_t)s[2 * w] | ((uint64_t)s[2 * w + 1] << 32);
    if (w < 4) {
      pkw[w] = v;
      skw[w] = v;
    } else if (w < 12) {
      rw[w - 4] = v;
    } else {
      skw[w - 8] = v;  // K at sk bytes 32..63
    }
  }
}

// ExpandA: one lane per (task, i, j); rho read from rows of `rho_src` (pk or sk)
// ExpandA (Sec. 2.3 sampling; Alg. 4's rejection sampler) with wave-cooperative
// compaction: 3 bytes -> 23-bit candidate, kept if < q, in stream order, until
// 256 are kept.  Every lane squeezes its own
// SHAKE128 stream; each squeezed block is staged in LDS and the wave then
// walks the lanes whose polynomial is unfinished, testing that lane's 56
// candidates on 56 lanes at once: a ballot gives each accepted candidate its
// position in stream order, so the accepted values of one stream are stored
// as one contiguous run.  out0 is lane 0's polynomial; lane l writes
// out0 + l * N.  rows: 64 * EA_ROW words of LDS for this wavefront.  Lanes
// with valid = false run the permutations but store nothing.
constexpr int EA_ROW = RATE128 / 4 + 1;  // 43 words: odd stride, conflict-free staging
constexpr int EA_STEP = 4;                // unfinished streams tested per step
constexpr int EA_WG = 64;                 // one wavefront per workgroup (11 KiB of LDS)
// Blocks after which another permutation is always needed: a block holds
// RATE128 / 3 = 56 candidates, so at least ceil(N / 56) = 5 blocks are squeezed.
constexpr int EA_SURE = (N + RATE128 / 3 - 1) / (RATE128 / 3) - 1;

// One compaction step for up to EA_STEP streams Ls[u] (act[u]: stream u of
// the step is unfinished), split in two halves so that independent work can
// be issued between them: ea_probe reads the candidates from LDS and the
// streams' counters; ea_commit ballots, stores the accepted values and
// advances the counters.
struct EaProbe {
  uint32_t tv[EA_STEP];
  int cL[EA_STEP];
};
__device__ __forceinline__ EaProbe ea_probe(const uint32_t *rows, const int Ls[EA_STEP], int ctr, int wi,
                                            uint32_t sh) {
  EaProbe p;
#pragma unroll
  for (int u = 0; u < EA_STEP; u++) {
    const uint32_t *rL = rows + Ls[u] * EA_ROW;
    p.tv[u] = __builtin_amdgcn_alignbit(rL[wi + 1], rL[wi], sh) & 0x7FFFFFu;
    p.cL[u] = __builtin_amdgcn_readlane(ctr, Ls[u]);  // the streams' lanes are distinct
  }
  return p;
}
__device__ __forceinline__ void ea_commit(const EaProbe &p, const int Ls[EA_STEP], const bool act[EA_STEP], bool cand,
                                          int32_t *out0, int &ctr, int lane) {
#pragma unroll
  for (int u = 0; u < EA_STEP; u++) {
    const bool ok = act[u] && cand && p.tv[u] < (uint32_t)Q;
    const uint64_t m = __ballot(ok);
    const int pos =
        p.cL[u] + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (ok && pos < N) out0[(size_t)Ls[u] * N + pos] = (int32_t)p.tv[u];
    if (act[u] && lane == Ls[u]) ctr = min(N, p.cL[u] + (int)__popcll(m));
  }
}

__device__ __forceinline__ void expand_a_squeeze_wave(uint32_t s[50], int32_t *out0, uint32_t *rows, int lane,
                                                      bool valid) {
  int ctr = valid ? 0 : N;
  uint32_t *row = rows + lane * EA_ROW;
  // lane l < 56 tests candidate l of a block: bytes 3l .. 3l + 2, inside words
  // wi and wi + 1 of the staged row; the other lanes read word 0 and test nothing
  const bool cand = lane < RATE128 / 3;
  const int wi = cand ? (3 * lane) >> 2 : 0;
  const uint32_t sh = cand ? 8u * (uint32_t)((3 * lane) & 3) : 0u;
  // Blocks 0 .. EA_SURE - 1: the next permutation is certain, so it runs
  // during the compaction of the staged block (the state and the LDS rows are
  // independent): every stream is tested in 64 / EA_STEP steps, and the 24
  // rounds are spread over them, so the Keccak ALU work covers the latency of
  // the steps' LDS reads and ballots.
  static_assert(64 / EA_STEP == 16, "the round schedule below assumes 16 steps of 4 streams");
  for (int blk = 0; blk < EA_SURE; blk++) {
#pragma unroll
    for (int w = 0; w < RATE128 / 4; w++) row[w] = s[w];
    wave_sync();
    const uint64_t pending = __ballot(ctr < N);
#pragma unroll 1
    for (int it = 0; it < 8; it++) {  // two steps and three rounds per iteration
      int La[EA_STEP], Lb[EA_STEP];
      bool aa[EA_STEP], ab[EA_STEP];
#pragma unroll
      for (int u = 0; u < EA_STEP; u++) {
        La[u] = 2 * EA_STEP * it + u;
        Lb[u] = La[u] + EA_STEP;
        aa[u] = (pending >> La[u]) & 1;
        ab[u] = (pending >> Lb[u]) & 1;
      }
      const EaProbe pa = ea_probe(rows, La, ctr, wi, sh);
      keccak_round(s, 3 * it);
      keccak_round(s, 3 * it + 1);
      ea_commit(pa, La, aa, cand, out0, ctr, lane);
      const EaProbe pb = ea_probe(rows, Lb, ctr, wi, sh);
      keccak_round(s, 3 * it + 2);
      ea_commit(pb, Lb, ab, cand, out0, ctr, lane);
    }
    wave_sync();
  }
  // later blocks: compact first, then permute only if a stream is unfinished
  for (;;) {
#pragma unroll
    for (int w = 0; w < RATE128 / 4; w++) row[w] = s[w];
    wave_sync();
    // up to EA_STEP unfinished streams per step; the step is branch-free up to
    // the stores, so that its LDS reads, ballots and counter reads overlap
    uint64_t pending = __ballot(ctr < N);
    while (pending) {
      int Ls[EA_STEP];
      bool act[EA_STEP];
#pragma unroll
      for (int u = 0; u < EA_STEP; u++) {
        act[u] = pending != 0;
        Ls[u] = act[u] ? __builtin_ctzll(pending) : 0;
        pending &= pending - 1;
      }
      const EaProbe p = ea_probe(rows, Ls, ctr, wi, sh);
      ea_commit(p, Ls, act, cand, out0, ctr, lane);
    }
    wave_sync();
    if (__ballot(ctr < N) == 0) break;
    keccak_f(s);
  }
}

template <int LV>
__global__ void __launch_bounds__(EA_WG) expand_a_k(const uint8_t *rho_src, size_t rho_stride, const uint32_t *key_idx,
                                                  int32_t *A, uint32_t count) {
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L;
  uint64_t st = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  __shared__ uint32_t rows[EA_WG / 64][64 * EA_ROW];
  const bool valid = st < (uint64_t)count * K * L;
  const uint64_t sl = valid ? st : 0;  // spare lanes absorb stream 0 and store nothing
  uint32_t task = (uint32_t)(sl / (K * L));
  int ij = (int)(sl % (K * L));
  int i = ij / L, j = ij % L;
  size_t key = key_idx ? key_idx[task] : task;
  const uint64_t *rho = (const uint64_t *)(rho_src + key * rho_stride);
  uint32_t s[50];
  absorb_seed34(s, [&](int pos) { return rho[pos >> 3]; }, (uint32_t)j | ((uint32_t)i << 8));
  const int lane = threadIdx.x & 63;
  expand_a_squeeze_wave(s, A + (size_t)(st - lane) * N, rows[threadIdx.x >> 6], lane, valid);
}

// ExpandS: one lane per (task, r < L + K); centred coefficients to ws.s1h
template <int LV>
__global__ void __launch_bounds__(256) expand_s_k(Ws ws, uint32_t count) {
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L;
  uint64_t st = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (st >= (uint64_t)count * (K + L)) return;
  uint32_t task = (uint32_t)(st / (K + L));
  int r = (int)(st % (K + L));
  uint32_t s[50];
  absorb_seed66(s, ws.rhop + (size_t)task * 64, (uint32_t)r);
  expand_s_squeeze<Lv<LV>::ETA>(s, ws.s1h + (size_t)st * N);
}

// LDS layout shared by the per-task polynomial kernels
template <int LV>
struct PolyLds {
  int32_t tr[4 * NTT_LDS_GROUP];              // transposes, one region per group
  int32_t hat[(Lv<LV>::L > Lv<LV>::K ? Lv<LV>::L : Lv<LV>::K) * HAT_POLY];  // NTT-domain vector (hat_idx)
  uint32_t buf[(P<LV>::SK + 64) / 4 + 2];     // byte staging (packed rows), + pad words
};

// consecutive-layout values of the lane (16t .. 16t+15) from its strided values
template <bool PAD = true>
__device__ __forceinline__ void to_consecutive(const int32_t x[16], uint32_t v[16], int32_t *tr, int t) {
  int32_t y[16];
#pragma unroll
  for (int r = 0; r < 16; r++) y[r] = x[r];
  transpose_s2c<PAD>(y, tr, t);
#pragma unroll
  for (int r = 0; r < 16; r++) v[r] = (uint32_t)y[r];
}

// KeyGen main: t = INTT(A * NTT(s1)) + s2, Power2Round, pack pk's t1 and sk's s1, s2, t0
template <int LV>
__global__ void __launch_bounds__(64) kg_main_k(Ws ws, uint8_t *pk, uint8_t *sk, uint32_t count) {
  using PP = P<LV>;
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L, ETA = Lv<LV>::ETA;
  __shared__ PolyLds<LV> lds;
  __shared__ uint32_t pkbuf[PP::PK / 4 + 2];
  uint32_t task = blockIdx.x;
  if (task >= count) return;
  int lane = threadIdx.x, g = lane >> 4, t = lane & 15;
  int32_t *tr = lds.tr + g * NTT_LDS_GROUP;
  uint8_t *skb = (uint8_t *)lds.buf;
  uint8_t *pkb = (uint8_t *)pkbuf;
  const int32_t *S = ws.s1h + (size_t)task * (K + L) * N;
  const Tw ftw = ntt_lane_tw(t), itw = intt_lane_tw(t);
  // s1: NTT into LDS, and pack eta - s into sk
  for (int j = g; j < L; j += 4) {
    int32_t x[16];
    load_strided(x, S + j * N, t);
    uint32_t v[16];
    to_consecutive(x, v, tr, t);
#pragma unroll
    for (int r = 0; r < 16; r++) v[r] = (uint32_t)(ETA - (int32_t)v[r]);
    pack16_to_lds<PP::EBITS>(v, skb + PP::OFF_S1 + j * PP::EB, t);
    ntt16(x, ftw, tr, t);
#pragma unroll
    for (int r = 0; r < 16; r++) lds.hat[hat_idx(j, t, r)] = x[r];
  }
  wave_sync();
  for (int i = g; i < K; i += 4) {
    const int32_t *Ai = ws.A + ((size_t)task * K + i) * L * N;
    int64_t acc[16];
#pragma unroll
    for (int r = 0; r < 16; r++) acc[r] = 0;
    for (int j = 0; j < L; j++) {
      int32_t a[16];
      load_slots(a, Ai + j * N, t);
#pragma unroll
      for (int r = 0; r < 16; r++) acc[r] += (int64_t)a[r] * lds.hat[hat_idx(j, t, r)];
    }
    int32_t x[16];
#pragma unroll
    for (int r = 0; r < 16; r++) x[r] = mont_reduce(acc[r]);
    intt16(x, itw, tr, t);
    int32_t s2[16];
    load_strided(s2, S + (L + i) * N, t);
    uint32_t v[16];
    to_consecutive(s2, v, tr, t);
#pragma unroll
    for (int r = 0; r < 16; r++) v[r] = (uint32_t)(ETA - (int32_t)v[r]);
    pack16_to_lds<PP::EBITS>(v, skb + PP::OFF_S2 + i * PP::EB, t);
    int32_t t1[16], t0[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      int32_t tv = canon(x[r]) + s2[r];            // in [-eta, q + eta)
      tv += (tv >> 31) & Q;
      tv -= Q;
      tv += (tv >> 31) & Q;                        // canonical
      power2round(tv, t1[r], t0[r]);
      t0[r] = (1 << (D - 1)) - t0[r];
    }
    to_consecutive(t1, v, tr, t);
    pack16_to_lds<10>(v, pkb + 32 + i * PP::T1B, t);
    to_consecutive(t0, v, tr, t);
    pack16_to_lds<13>(v, skb + PP::OFF_T0 + i * PP::T0B, t);
  }
  wave_sync();
  // copy the packed regions out (pk[32..PK), sk[OFF_S1..SK)); rho, K, tr are written elsewhere
  uint32_t *pkg = (uint32_t *)(pk + (size_t)task * PP::PK);
  for (int w = 8 + lane; w < PP::PK / 4; w += 64) pkg[w] = pkbuf[w];
  uint32_t *skg = (uint32_t *)(sk + (size_t)task * PP::SK);
  for (int w = PP::OFF_S1 / 4 + lane; w < PP::SK / 4; w += 64) skg[w] = lds.buf[w];
}

// tr = H(pk) (TRB = 32 or 64 bytes) into sk bytes 64 .. 64 + TRB
template <int LV>
__global__ void __launch_bounds__(256) kg_tr_k(const uint8_t *pk, uint8_t *sk, uint32_t count) {
  uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const uint8_t *p = pk + (size_t)t * P<LV>::PK;
  uint32_t s[50];
  shake_absorb<RATE256>(s, P<LV>::PK, [&](uint64_t pos) { return *(const uint64_t *)(p + pos); });
  uint32_t *o = (uint32_t *)(sk + (size_t)t * P<LV>::SK + 64);
#pragma unroll
  for (int w = 0; w < P<LV>::TRB / 4; w++) o[w] = s[w];
}

// ------------------------------------------------------------------------
// Sign (Alg. 2), staged
// ------------------------------------------------------------------------
// mu and the mask seed on two lanes per task (keccak_pair.h); initialises
// kappa and the active list.
//   round 3: mu = H(tr || M); rho' = H(K || mu), or the task's 64 rnd bytes
//            themselves (randomized signing) when rnd is not null;
//   ML-DSA:  mu = H(tr || 0x00 || 0x00 || M); rho'' = H(K || rnd || mu) with
//            the task's 32 rnd bytes, or 32 zero bytes when rnd is null;
//            with INTERNAL the messages are formatted messages M' (a context
//            string or the pre-hash form, built by the caller) and mu =
//            H(tr || M').
// rnd rows are 4-byte aligned.
template <int LV, bool INTERNAL = false>
__global__ void __launch_bounds__(256) sg_prep_k(const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                                                 const uint64_t *msg_off, const uint8_t *rnd, Ws ws, uint32_t count,
                                                 uint32_t *err) {
  // the longest dependent chain of the Sign setup (up to ~30 permutations per
  // task for 4 KiB messages), sharing the CUs with ExpandA and the secret NTTs
  // launched beside it: its waves issue first
  __builtin_amdgcn_s_setprio(3);
  const uint32_t t = (uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1);
  const int half = threadIdx.x & 1;
  if (t >= count) return;  // both lanes of a pair
  size_t key = key_idx ? key_idx[t] : t;
  const uint8_t *skr = sk + key * P<LV>::SK;
  uint64_t o0 = msg_off[t], o1 = msg_off[t + 1];
  uint64_t mlen = 0;
  if (o1 >= o0) mlen = o1 - o0;
  else if (!half) atomicOr(err, 1u);  // decreasing msg_off: message treated as empty
  constexpr int TW = P<LV>::TRB / 4;
  uint32_t a[25];
  uint32_t trw[TW];
  const uint32_t *skw = (const uint32_t *)(skr + 64);  // tr inside the 8-byte aligned sk row
#pragma unroll
  for (int i = 0; i < TW; i++) trw[i] = skw[i];
  absorb_prefix_msg<mu_prefix_bytes<LV, INTERNAL>()>(a, half, trw, msg + o0, mlen);
  uint32_t mu[8];  // this lane's halves of mu's eight 8-byte words
  uint32_t *muw = (uint32_t *)(ws.muw1 + (size_t)t * muw1_stride<LV>());
#pragma unroll
  for (int i = 0; i < 8; i++) {
    mu[i] = a[i];
    muw[2 * i + half] = a[i];
  }
  uint32_t *rp = (uint32_t *)(ws.rhop + (size_t)t * 64);
  if constexpr (Lv<LV>::MLDSA) {
    // rho'' = H(K || rnd || mu): 128 bytes, one block
    const uint32_t *Kw = (const uint32_t *)(skr + 32);
    const uint32_t *rw = rnd ? (const uint32_t *)(rnd + (size_t)t * 32) : nullptr;
#pragma unroll
    for (int i = 0; i < 25; i++)
      a[i] = i < 4 ? Kw[2 * i + half] : i < 8 ? (rw ? rw[2 * (i - 4) + half] : 0u) : i < 16 ? mu[i - 8] : 0u;
    a[16] ^= half ? 0x80u << 24 : 0x1Fu;
    keccak_f_pair(a, half);
#pragma unroll
    for (int i = 0; i < 8; i++) rp[2 * i + half] = a[i];
  } else if (rnd) {
    const uint32_t *rw = (const uint32_t *)(rnd + (size_t)t * 64);
#pragma unroll
    for (int i = 0; i < 8; i++) rp[2 * i + half] = rw[2 * i + half];
  } else {
    // rho' = H(K || mu): 96 bytes, one block
    const uint32_t *Kw = (const uint32_t *)(skr + 32);
#pragma unroll
    for (int i = 0; i < 25; i++) a[i] = i < 4 ? Kw[2 * i + half] : i < 12 ? mu[i - 4] : 0u;
    if (!half) a[12] ^= 0x1Fu;
    else a[RATE256 / 8 - 1] ^= 0x80u << 24;
    keccak_f_pair(a, half);
#pragma unroll
    for (int i = 0; i < 8; i++) rp[2 * i + half] = a[i];
  }
  if (!half) {
    ws.kappa[t] = 0;
    ws.active0[t] = t;
  }
}

// NTT of the secret vectors s1, s2, t0 unpacked from sk
template <int LV>
__global__ void __launch_bounds__(64) sg_secret_k(const uint8_t *sk, const uint32_t *key_idx, Ws ws, uint32_t count) {
  using PP = P<LV>;
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L, ETA = Lv<LV>::ETA;
  __shared__ PolyLds<LV> lds;
  uint32_t task = blockIdx.x;
  if (task >= count) return;
  int lane = threadIdx.x, g = lane >> 4, t = lane & 15;
  int32_t *tr = lds.tr + g * NTT_LDS_GROUP;
  size_t key = key_idx ? key_idx[task] : task;
  const uint8_t *skr = sk + key * PP::SK;
  // stage sk bytes OFF_S1..SK into LDS (sk rows are 8-byte aligned)
  const uint32_t *skw = (const uint32_t *)(skr + PP::OFF_S1);
  constexpr int NW = (PP::SK - PP::OFF_S1) / 4;
  g2l_words<NW>(skw, lds.buf, lane);
  if (lane < 2) lds.buf[NW + lane] = 0;
  wave_sync();
  const Tw ftw = ntt_lane_tw(t);
  for (int p = g; p < L + 2 * K; p += 4) {
    uint32_t v[16];
    int32_t x[16];
    int32_t *dst;
    if (p < L + K) {
      const uint32_t *src = lds.buf + (p * PP::EB) / 4;
      unpack_strided<PP::EBITS>(src, v, t);
#pragma unroll
      for (int r = 0; r < 16; r++) x[r] = ETA - (int32_t)v[r];
      dst = p < L ? ws.s1h + ((size_t)task * L + p) * N : ws.s2h + ((size_t)task * K + (p - L)) * N;
    } else {
      int i = p - L - K;
      const uint32_t *src = lds.buf + ((L + K) * PP::EB + i * PP::T0B) / 4;
      unpack_strided<13>(src, v, t);
#pragma unroll
      for (int r = 0; r < 16; r++) x[r] = (1 << (D - 1)) - (int32_t)v[r];
      dst = ws.t0h + ((size_t)task * K + i) * N;
    }
    ntt16(x, ftw, tr, t);
    store_slots(x, dst, t);
  }
}

// ---- Sign iteration building blocks, shared by the staged kernels and the
// ---- persistent kernel (same arithmetic in both execution forms)

// ExpandMask stream i of iteration kappa (one lane)
template <int LV>
__device__ __forceinline__ void dev_expand_mask(const uint8_t *rhop, uint32_t kappa, int i, int32_t *y_out) {
  uint32_t s[50];
  absorb_seed66(s, rhop, (kappa + (uint32_t)i) & 0xFFFFu);
  expand_mask_squeeze<P<LV>::ZBITS, Lv<LV>::GAMMA1>(s, y_out);
}

// w = INTT(A-hat * NTT(y)) for one task by one wavefront: w (canonical) to
// w_out, HighBits(w) packed into w1_out (4-byte aligned, K * W1B bytes).
// hat: L * HAT_POLY words of LDS; tr: this group's transpose region; w1buf: LDS
// staging; ftw / itw: forward / inverse twiddles.
// EARLY: the group's first A-hat polynomial (row g, column 0) is requested
// before the NTT of y, and each next one before the current one is multiplied.
// The fences of the NTT's LDS transposes keep the compiler from hoisting these
// loads by itself, which leaves each load's latency exposed; requesting them
// early costs 16 registers per lane, which only the l = 4 loop kernels have.
template <int LV, bool PAD = true, bool EARLY = false, class TW>
__device__ __forceinline__ void dev_compute_w(const int32_t *y, const int32_t *A, int32_t *w_out, uint8_t *w1_out,
                                              int32_t *hat, int32_t *tr, uint32_t *w1buf, const TW &ftw,
                                              const TW &itw, int lane) {
  using PP = P<LV>;
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L;
  int g = lane >> 4, t = lane & 15;
  int32_t an[16];
  if constexpr (EARLY) {
    if (g < K) load_slots(an, A + (size_t)g * L * N, t);
  }
  for (int j = g; j < L; j += 4) {
    int32_t x[16];
    load_strided(x, y + j * N, t);
    ntt16<TW, PAD>(x, ftw, tr, t);
#pragma unroll
    for (int r = 0; r < 16; r++) hat[hat_idx(j, t, r)] = x[r];
  }
  wave_sync();
  for (int i = g; i < K; i += 4) {
    const int32_t *Ai = A + (size_t)i * L * N;
    int64_t acc[16];
#pragma unroll
    for (int r = 0; r < 16; r++) acc[r] = 0;
    if constexpr (EARLY) {
      for (int j = 0; j < L; j++) {
        int32_t a[16];
#pragma unroll
        for (int r = 0; r < 16; r++) a[r] = an[r];
        if (j + 1 < L) load_slots(an, Ai + (j + 1) * N, t);
        else if (i + 4 < K) load_slots(an, A + (size_t)(i + 4) * L * N, t);
#pragma unroll
        for (int r = 0; r < 16; r++) acc[r] += (int64_t)a[r] * hat[hat_idx(j, t, r)];
      }
    } else {
      for (int j = 0; j < L; j++) {
        int32_t a[16];
        load_slots(a, Ai + j * N, t);
#pragma unroll
        for (int r = 0; r < 16; r++) acc[r] += (int64_t)a[r] * hat[hat_idx(j, t, r)];
      }
    }
    int32_t x[16];
#pragma unroll
    for (int r = 0; r < 16; r++) x[r] = mont_reduce(acc[r]);
    intt16<TW, PAD>(x, itw, tr, t);
    int32_t w1[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      x[r] = canon(x[r]);
      w1[r] = highbits<LV>(x[r]);
    }
    store_strided(x, w_out + i * N, t);
    uint32_t v[16];
    to_consecutive<PAD>(w1, v, tr, t);
    pack16_to_lds<PP::W1BITS>(v, (uint8_t *)w1buf + i * PP::W1B, t);
  }
  wave_sync();
  uint32_t *dst = (uint32_t *)w1_out;
  for (int w = lane; w < K * PP::W1B / 4; w += 64) dst[w] = w1buf[w];
}

// SampleInBall on the lane's SHAKE256(ctilde) stream, into a per-lane 256-byte
// LDS array; positions are drawn with rejection against the loop index.
template <int TAU>
__device__ __forceinline__ void sample_in_ball(uint32_t s[50], int8_t *c, uint8_t *blockbuf) {
  // s holds the first squeezed block
  uint32_t *bw = (uint32_t *)blockbuf;
#pragma unroll
  for (int w = 0; w < RATE256 / 4; w++) bw[w] = s[w];
  uint64_t signs = (uint64_t)s[0] | ((uint64_t)s[1] << 32);
  uint32_t *cw = (uint32_t *)c;
#pragma unroll
  for (int w = 0; w < N / 4; w++) cw[w] = 0;
  int pos = 8;
  for (int i = N - TAU; i < N; i++) {
    int b;
    for (;;) {
      if (pos == RATE256) {
        keccak_f(s);
#pragma unroll
        for (int w = 0; w < RATE256 / 4; w++) bw[w] = s[w];
        pos = 0;
      }
      b = blockbuf[pos++];
      if (b <= i) break;
    }
    c[i] = c[b];
    c[b] = (int8_t)(1 - 2 * (int)(signs & 1));
    signs >>= 1;
  }
}

// ctilde = H(mu || w1) of CT bytes (mu and packed w1 8-byte aligned);
// c = SampleInBall(ctilde), seeded by all of ctilde (one lane)
template <int LV>
__device__ __forceinline__ void dev_challenge(const uint8_t *mu, const uint8_t *w1, uint32_t *ctilde_out, int8_t *c,
                                              uint8_t *blockbuf) {
  constexpr int CW = P<LV>::CT / 4;
  uint32_t s[50];
  shake_absorb<RATE256>(s, P<LV>::MUW1, [&](uint64_t pos) {
    return pos < 64 ? *(const uint64_t *)(mu + pos) : *(const uint64_t *)(w1 + (pos - 64));
  });
  uint32_t ct[CW];
#pragma unroll
  for (int i = 0; i < CW; i++) {
    ct[i] = s[i];
    ctilde_out[i] = s[i];
  }
  keccak_zero(s);
#pragma unroll
  for (int i = 0; i < CW; i++) s[i] = ct[i];
  s[CW] = 0x1Fu;
  s[2 * (RATE256 / 8 - 1) + 1] ^= 0x80u << 24;
  keccak_f(s);
  sample_in_ball<Lv<LV>::TAU>(s, c, blockbuf);
}

template <int LV>
struct CheckLds {
  int32_t tr[4 * NTT_LDS_GROUP];
  uint32_t sigbuf[P<LV>::SIG / 4 + 2];
  uint16_t hmask[Lv<LV>::K][16];
  int rowcnt[Lv<LV>::K];
};

// The rejection checks of Alg. 2 for one candidate (one wavefront):
// z = y + c s1, r0 = LowBits(w - c s2), c t0 and the hint.  c is the dense
// challenge (int8, natural order).  Returns true (wave-uniform) if the
// candidate passes all four checks; the packed signature (ctilde, z, h) is
// then in lds.sigbuf.  Polynomials whose norm already fails stop the
// evaluation early.  EARLY (as in dev_compute_w): the group's first s1-hat
// and y polynomials are requested before the NTT of c, the next ones before
// the current one's INTT, and a row's w and t0-hat together with its s2-hat.
template <int LV, bool PAD = true, bool EARLY = false, class TW>
__device__ __forceinline__ bool dev_check(const int8_t *c, const uint32_t *ctilde, const int32_t *y, const int32_t *w,
                                          const int32_t *s1h, const int32_t *s2h, const int32_t *t0h,
                                          CheckLds<LV> &lds, const TW &ftw, const TW &itw, int lane) {
  using PP = P<LV>;
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L, BETA = Lv<LV>::BETA, OMEGA = Lv<LV>::OMEGA;
  constexpr int32_t G1 = Lv<LV>::GAMMA1, G2 = Lv<LV>::GAMMA2;
  int g = lane >> 4, t = lane & 15;
  int32_t *tr = lds.tr + g * NTT_LDS_GROUP;
  uint8_t *sb = (uint8_t *)lds.sigbuf;
  // c-hat, computed by every group
  int32_t ch[16];
#pragma unroll
  for (int r = 0; r < 16; r++) ch[r] = c[t + 16 * r];
  int32_t s1n[16], yn[16];
  if constexpr (EARLY) {
    if (g < L) {
      load_slots(s1n, s1h + g * N, t);
      load_strided(yn, y + g * N, t);
    }
  }
  ntt16<TW, PAD>(ch, ftw, tr, t);
  bool bad = false;
  // z = y + c s1
  for (int j = g; j < L; j += 4) {
    int32_t s1[16], x[16], yv[16];
    if constexpr (EARLY) {
#pragma unroll
      for (int r = 0; r < 16; r++) {
        s1[r] = s1n[r];
        yv[r] = yn[r];
      }
      if (j + 4 < L) {
        load_slots(s1n, s1h + (j + 4) * N, t);
        load_strided(yn, y + (j + 4) * N, t);
      }
    } else {
      load_slots(s1, s1h + j * N, t);
    }
#pragma unroll
    for (int r = 0; r < 16; r++) x[r] = mont_mul(ch[r], s1[r]);
    intt16<TW, PAD>(x, itw, tr, t);
    if constexpr (!EARLY) load_strided(yv, y + j * N, t);
    int32_t zv[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      int32_t z = yv[r] + canon(x[r]);             // in [-gamma1 + 1, q + gamma1)
      z = z > (Q - 1) / 2 ? z - Q : z;             // centred
      bad |= (z >= G1 - BETA) || (z <= -(G1 - BETA));
      zv[r] = G1 - z;
    }
    uint32_t v[16];
    to_consecutive<PAD>(zv, v, tr, t);
    pack16_to_lds<PP::ZBITS>(v, sb + PP::OFF_Z + j * PP::ZB, t);
  }
  if (wave_any(bad)) return false;
  // r0 = LowBits(w - c s2), c t0 and the hint
  for (int i = g; i < K; i += 4) {
    int32_t s2[16], x[16], u[16], wv[16];
    load_slots(s2, s2h + i * N, t);
    if constexpr (EARLY) {
      load_strided(wv, w + i * N, t);
      load_slots(u, t0h + i * N, t);
    }
#pragma unroll
    for (int r = 0; r < 16; r++) x[r] = mont_mul(ch[r], s2[r]);
    intt16<TW, PAD>(x, itw, tr, t);
    if constexpr (!EARLY) load_strided(wv, w + i * N, t);
    int32_t r1v[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      x[r] = canon(wv[r] - canon(x[r]));           // w - c s2, canonical
      int32_t r1, r0;
      decompose<LV>(x[r], r1, r0);
      r1v[r] = r1;
      bad |= (r0 >= G2 - BETA) || (r0 <= -(G2 - BETA));
    }
    if constexpr (!EARLY) load_slots(u, t0h + i * N, t);
#pragma unroll
    for (int r = 0; r < 16; r++) u[r] = mont_mul(ch[r], u[r]);
    intt16<TW, PAD>(u, itw, tr, t);
    int cnt = 0;
#pragma unroll
    for (int r = 0; r < 16; r++) {
      int32_t ct0 = canon(u[r]);
      bad |= norm_ge(ct0, G2);
      int32_t sum = x[r] + ct0;
      sum -= (sum >= Q) ? Q : 0;                   // w - c s2 + c t0, canonical
      bool h = highbits<LV>(sum) != r1v[r];
      uint64_t m = __ballot(h);
      uint32_t m16 = (uint32_t)(m >> (16 * g)) & 0xFFFFu;
      if (t == 0) lds.hmask[i][r] = (uint16_t)m16;
      cnt += __popc(m16);
    }
    if (t == 0) lds.rowcnt[i] = cnt;
  }
  if (wave_any(bad)) return false;
  wave_sync();
  int total = 0;
  for (int i = 0; i < K; i++) total += lds.rowcnt[i];
  if (total > OMEGA) return false;
  // accepted: ctilde and the hint bytes
  if (lane < PP::CT / 4) lds.sigbuf[lane] = ctilde[lane];
  for (int b = lane; b < OMEGA + K; b += 64) sb[PP::OFF_H + b] = 0;
  wave_sync();
  for (int i = g; i < K; i += 4) {
    int pre = 0;
    for (int i2 = 0; i2 < i; i2++) pre += lds.rowcnt[i2];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      uint32_t m16 = lds.hmask[i][r];
      if ((m16 >> t) & 1u) sb[PP::OFF_H + pre + __popc(m16 & ((1u << t) - 1u))] = (uint8_t)(t + 16 * r);
      pre += __popc(m16);
    }
    if (t == 0) sb[PP::OFF_H + OMEGA + i] = (uint8_t)pre;
  }
  wave_sync();
  return true;
}

// ---- staged kernels ----
// ExpandMask: one lane per (active task, i < L)
template <int LV>
__global__ void __launch_bounds__(256) expand_mask_k(Ws ws, const uint32_t *active, uint32_t nactive) {
  constexpr int L = Lv<LV>::L;
  uint64_t st = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (st >= (uint64_t)nactive * L) return;
  uint32_t task = active[st / L];
  int i = (int)(st % L);
  dev_expand_mask<LV>(ws.rhop + (size_t)task * 64, ws.kappa[task], i, ws.y + ((size_t)task * L + i) * N);
}

// w = INTT(A * NTT(y)); w1 = HighBits(w) packed after mu
template <int LV>
__global__ void __launch_bounds__(64) sg_w_k(Ws ws, const uint32_t *active, uint32_t nactive) {
  using PP = P<LV>;
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L;
  __shared__ PolyLds<LV> lds;
  if (blockIdx.x >= nactive) return;
  uint32_t task = active[blockIdx.x];
  int lane = threadIdx.x, t = lane & 15;
  const Tw ftw = ntt_lane_tw(t), itw = intt_lane_tw(t);
  dev_compute_w<LV>(ws.y + (size_t)task * L * N, ws.A + kix(ws, task) * K * L * N, ws.w + (size_t)task * K * N,
                    ws.muw1 + (size_t)task * muw1_stride<LV>() + 64, lds.hat, lds.tr + (lane >> 4) * NTT_LDS_GROUP,
                    lds.buf, ftw, itw, lane);
  (void)PP::K;
}

// One lane's dense challenge in LDS: rows of C_ROW bytes (65 words), so that
// the lanes of a wavefront writing the same coefficient index hit 64
// different banks; copied out to a 16-byte aligned global row.
constexpr int C_ROW = N + 4;
__device__ __forceinline__ void store_c_row(const int8_t *c, int8_t *dst) {
  const uint32_t *cw = (const uint32_t *)c;
  int4 *d = (int4 *)dst;
#pragma unroll
  for (int w = 0; w < N / 16; w++) d[w] = make_int4(cw[4 * w], cw[4 * w + 1], cw[4 * w + 2], cw[4 * w + 3]);
}

// ctilde = H(mu || w1); c = SampleInBall(ctilde).  One lane per active task.
template <int LV>
__global__ void __launch_bounds__(64) sg_chal_k(Ws ws, const uint32_t *active, uint32_t nactive) {
  __shared__ int8_t cl[64][C_ROW];
  __shared__ uint32_t bb[64][RATE256 / 4];
  uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nactive) return;
  uint32_t task = active[a];
  int8_t *c = cl[threadIdx.x];
  const uint8_t *row = ws.muw1 + (size_t)task * muw1_stride<LV>();
  dev_challenge<LV>(row, row + 64, (uint32_t *)(ws.ctilde + (size_t)task * CT_STRIDE), c, (uint8_t *)bb[threadIdx.x]);
  store_c_row(c, ws.cpoly + (size_t)task * N);
}

// checks; accept -> signature row of the task, reject -> kappa += l and next round
template <int LV>
__global__ void __launch_bounds__(64) sg_check_k(Ws ws, uint8_t *sig, const uint32_t *active, uint32_t nactive,
                                                 uint32_t *next_active) {
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L;
  __shared__ CheckLds<LV> lds;
  if (blockIdx.x >= nactive) return;
  uint32_t task = active[blockIdx.x];
  int lane = threadIdx.x, t = lane & 15;
  const Tw ftw = ntt_lane_tw(t), itw = intt_lane_tw(t);
  bool ok = dev_check<LV>(ws.cpoly + (size_t)task * N, (const uint32_t *)(ws.ctilde + (size_t)task * CT_STRIDE),
                          ws.y + (size_t)task * L * N, ws.w + (size_t)task * K * N, ws.s1h + kix(ws, task) * L * N,
                          ws.s2h + kix(ws, task) * K * N, ws.t0h + kix(ws, task) * K * N, lds, ftw, itw, lane);
  if (ok) {
    l2g_bytes(lds.sigbuf, P<LV>::SIG, sig + (size_t)task * P<LV>::SIG, lane, 64);
  } else if (lane == 0) {
    ws.kappa[task] += L;
    uint32_t slot = atomicAdd(&ws.counters[0], 1u);
    next_active[slot] = task;
  }
}

// ------------------------------------------------------------------------
// Verify (Alg. 3), staged
// ------------------------------------------------------------------------
// tr = H(pk) (unless resident) and mu = H(tr || M) (ML-DSA: H(tr || 0x00 ||
// 0x00 || M), or H(tr || M') of formatted messages with INTERNAL), two lanes
// per task (keccak_pair.h)
template <int LV, bool INTERNAL = false>
__global__ void __launch_bounds__(64) vf_hash_k(const uint8_t *pk, const uint32_t *key_idx, const uint8_t *msg,
                                                const uint64_t *msg_off, Ws ws, uint32_t count, uint32_t *err) {
  using PP = P<LV>;
  __builtin_amdgcn_s_setprio(3);  // the long hash chain of Verify, beside ExpandA: its waves issue first
  const uint32_t t = (uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1);
  const int half = threadIdx.x & 1;
  if (t >= count) return;  // both lanes of a pair
  size_t key = key_idx ? key_idx[t] : t;
  constexpr int TW = PP::TRB / 4;
  uint32_t a[25];
  uint32_t trw[TW];
  if (ws.tr) {
    const uint32_t *tg = (const uint32_t *)(ws.tr + key * PP::TRB);
#pragma unroll
    for (int i = 0; i < TW; i++) trw[i] = tg[i];
  } else {
    const uint32_t *pkr = (const uint32_t *)(pk + key * PP::PK);
    shake256_absorb_pair<PP::PK>(a, half, [&](int pos) { return pkr[pos / 4 + half]; });
    // both lanes need all of tr: the partner's halves come over the DPP swap
#pragma unroll
    for (int i = 0; i < TW / 2; i++) {
      const uint32_t other = pair_swap(a[i]);
      trw[2 * i] = half ? other : a[i];
      trw[2 * i + 1] = half ? a[i] : other;
    }
  }
  uint64_t o0 = msg_off[t], o1 = msg_off[t + 1];
  uint64_t mlen = 0;
  if (o1 >= o0) mlen = o1 - o0;
  else if (!half) atomicOr(err, 1u);  // decreasing msg_off: message treated as empty
  absorb_prefix_msg<mu_prefix_bytes<LV, INTERNAL>()>(a, half, trw, msg + o0, mlen);
  uint32_t *muw = (uint32_t *)(ws.muw1 + (size_t)t * muw1_stride<LV>());
#pragma unroll
  for (int i = 0; i < 8; i++) muw[2 * i + half] = a[i];
}

// c = SampleInBall(ctilde) and strict hint decoding, one lane per task
template <int LV>
__global__ void __launch_bounds__(64) vf_prep_k(const uint8_t *sig, Ws ws, uint32_t count) {
  using PP = P<LV>;
  constexpr int K = Lv<LV>::K, OMEGA = Lv<LV>::OMEGA;
  constexpr int HB = OMEGA + K;        // hint section bytes
  constexpr int HMW = K * 8 + 1;       // mask words per lane (+1: odd stride)
  __shared__ int8_t cl[64][C_ROW];
  __shared__ uint32_t bb[64][RATE256 / 4];
  __shared__ uint8_t hbl[64][HB];
  __shared__ uint32_t hml[64][HMW];
  uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const uint8_t *sg = sig + (size_t)t * PP::SIG;
  // the hint bytes are fetched now (independent loads, one wait) and decoded from LDS at the end
  uint8_t *hb = hbl[threadIdx.x];
#pragma unroll
  for (int j = 0; j < HB; j++) hb[j] = sg[PP::OFF_H + j];
  uint32_t s[50];
  // SampleInBall(ctilde), all CT bytes of it
  keccak_zero(s);
#pragma unroll
  for (int w = 0; w < PP::CT / 8; w++) {
    uint64_t v = load_le_bytes(sg + 8 * w, 8);
    s[2 * w] = (uint32_t)v;
    s[2 * w + 1] = (uint32_t)(v >> 32);
  }
  s[PP::CT / 4] = 0x1Fu;
  s[2 * (RATE256 / 8 - 1) + 1] ^= 0x80u << 24;
  keccak_f(s);
  int8_t *c = cl[threadIdx.x];
  sample_in_ball<Lv<LV>::TAU>(s, c, (uint8_t *)bb[threadIdx.x]);
  store_c_row(c, ws.cpoly + (size_t)t * N);
  // strict hint decoding into bit masks (built in LDS, then stored row-wise)
  uint32_t *hml_t = hml[threadIdx.x];
#pragma unroll
  for (int w = 0; w < K * 8; w++) hml_t[w] = 0;
  int ok = 1, prev = 0;
  for (int i = 0; i < K; i++) {
    int cnt = hb[OMEGA + i];
    if (cnt < prev || cnt > OMEGA) {
      ok = 0;
      break;
    }
    for (int j = prev; j < cnt; j++) {
      if (j > prev && hb[j] <= hb[j - 1]) ok = 0;
      hml_t[i * 8 + (hb[j] >> 5)] |= 1u << (hb[j] & 31);
    }
    prev = cnt;
  }
  if (ok)
    for (int j = prev; j < OMEGA; j++)
      if (hb[j] != 0) ok = 0;
  uint32_t *hm = ws.hmask + (size_t)t * K * 8;
#pragma unroll
  for (int w = 0; w < K * 8; w++) hm[w] = hml_t[w];
  ws.flag[t] = ok;
}

// w1' = UseHint(h, INTT(A NTT(z) - c-hat NTT(t1 2^d))), packed after mu; z norm check
template <int LV>
__global__ void __launch_bounds__(64) vf_main_k(const uint8_t *pk, const uint32_t *key_idx, const uint8_t *sig, Ws ws,
                                                uint32_t count) {
  using PP = P<LV>;
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L, BETA = Lv<LV>::BETA;
  constexpr int32_t G1 = Lv<LV>::GAMMA1;
  // The signature's bytes are read only to unpack z; t1 (from pk) and the
  // packed w1' rows are used only after that, so the three share one region
  // (less LDS per workgroup, more resident workgroups).  pk is fetched into
  // registers up front and written to the region once z is unpacked.
  constexpr int SIGW = PP::SIG / 4 + 3, PKW = PP::PK / 4, W1W = K * PP::W1B / 4 + 1;
  constexpr int PKPER = (PKW + 63) / 64;
  __shared__ int32_t trl[4 * NTT_LDS_GROUP];
  __shared__ int32_t zh[L * HAT_POLY];
  __shared__ uint32_t region[SIGW > PKW + 2 + W1W ? SIGW : PKW + 2 + W1W];
  uint32_t *const sigw = region, *const pkw = region, *const w1b = region + PKW + 2;
  uint32_t task = blockIdx.x;
  if (task >= count) return;
  int lane = threadIdx.x, g = lane >> 4, t = lane & 15;
  int32_t *tr = trl + g * NTT_LDS_GROUP;
  size_t key = key_idx ? key_idx[task] : task;
  uint32_t pkv[PKPER];
  if (!ws.t1h) {
    const uint32_t *pkg = (const uint32_t *)(pk + key * PP::PK);
#pragma unroll
    for (int q = 0; q < PKPER; q++) {
      const int i = lane + 64 * q;
      pkv[q] = i < PKW ? pkg[i] : 0u;
    }
  }
  g2l_bytes<PP::SIG>(sig + (size_t)task * PP::SIG, sigw, lane);
  if (lane < 2) sigw[PP::SIG / 4 + 1 + lane] = 0;
  wave_sync();
  const Tw ftw = ntt_lane_tw(t), itw = intt_lane_tw(t);
  int32_t ch[16];
  {
    const int8_t *cp = ws.cpoly + (size_t)task * N;
#pragma unroll
    for (int r = 0; r < 16; r++) ch[r] = cp[t + 16 * r];
    ntt16(ch, ftw, tr, t);
  }
  bool bad = false;
  for (int j = g; j < L; j += 4) {
    uint32_t v[16];
    unpack_strided<PP::ZBITS>(sigw + (PP::OFF_Z + j * PP::ZB) / 4, v, t);
    int32_t x[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      int32_t z = G1 - (int32_t)v[r];
      bad |= (z >= G1 - BETA) || (z <= -(G1 - BETA));
      x[r] = z;
    }
    ntt16(x, ftw, tr, t);
#pragma unroll
    for (int r = 0; r < 16; r++) zh[hat_idx(j, t, r)] = x[r];
  }
  bad = wave_any(bad);
  wave_sync();
  if (!ws.t1h) {  // z is unpacked: the region now takes t1
#pragma unroll
    for (int q = 0; q < PKPER; q++) {
      const int i = lane + 64 * q;
      if (i < PKW) pkw[i] = pkv[q];
    }
    if (lane < 2) pkw[PKW + lane] = 0;
    wave_sync();
  }
  const uint32_t *hm = ws.hmask + (size_t)task * K * 8;
  for (int i = g; i < K; i += 4) {
    const int32_t *Ai = ws.A + (kix(ws, task) * K + i) * L * N;
    int64_t acc[16];
#pragma unroll
    for (int r = 0; r < 16; r++) acc[r] = 0;
    for (int j = 0; j < L; j++) {
      int32_t a[16];
      load_slots(a, Ai + j * N, t);
#pragma unroll
      for (int r = 0; r < 16; r++) acc[r] += (int64_t)a[r] * zh[hat_idx(j, t, r)];
    }
    int32_t x[16];
    if (ws.t1h) {
      load_slots(x, ws.t1h + (kix(ws, task) * K + i) * N, t);
    } else {
      uint32_t v[16];
      unpack_strided<10>(pkw + (32 + i * PP::T1B) / 4, v, t);
#pragma unroll
      for (int r = 0; r < 16; r++) x[r] = (int32_t)(v[r] << D);
      ntt16(x, ftw, tr, t);
    }
    // transpose-free: t1-hat comes out in slots layout like acc
#pragma unroll
    for (int r = 0; r < 16; r++) {
      int32_t d = mont_reduce(acc[r]) - mont_mul(ch[r], x[r]);  // in (-2q, 2q)
      d += (d <= -Q) ? Q : 0;
      d -= (d >= Q) ? Q : 0;
      x[r] = d;
    }
    intt16(x, itw, tr, t);
    int32_t w1[16];
    uint32_t hw[8];
#pragma unroll
    for (int q = 0; q < 8; q++) hw[q] = hm[i * 8 + q];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      int c = t + 16 * r;
      int32_t h = (hw[c >> 5] >> (c & 31)) & 1;
      w1[r] = use_hint<LV>(h, canon(x[r]));
    }
    uint32_t vv[16];
    to_consecutive(w1, vv, tr, t);
    pack16_to_lds<PP::W1BITS>(vv, (uint8_t *)w1b + i * PP::W1B, t);
  }
  wave_sync();
  uint32_t *dst = (uint32_t *)(ws.muw1 + (size_t)task * muw1_stride<LV>() + 64);
  for (int w = lane; w < K * PP::W1B / 4; w += 64) dst[w] = w1b[w];
  if (lane == 0 && bad) ws.flag[task] = 0;
}

// ctilde' = H(mu || w1'), verdict; two lanes per task (keccak_pair.h), the
// even lane writing the verdict
template <int LV>
__global__ void __launch_bounds__(256) vf_final_k(const uint8_t *sig, Ws ws, int32_t *verdict, uint32_t count) {
  const uint32_t t = (uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1);
  const int half = threadIdx.x & 1;
  if (t >= count) return;  // both lanes of a pair
  const uint8_t *row = ws.muw1 + (size_t)t * muw1_stride<LV>();
  uint32_t a[25];
  shake256_absorb_pair<P<LV>::MUW1>(a, half, [&](int pos) { return *(const uint32_t *)(row + pos + 4 * half); });
  const uint8_t *sg = sig + (size_t)t * P<LV>::SIG;
  uint32_t diff = 0;
#pragma unroll
  for (int w = 0; w < P<LV>::CT / 8; w++) diff |= (uint32_t)load_le_bytes(sg + 8 * w + 4 * half, 4) ^ a[w];
  diff |= pair_swap(diff);
  if (!half) verdict[t] = (ws.flag[t] && diff == 0) ? 1 : 0;
}

// ------------------------------------------------------------------------
// Resident key tables
// ------------------------------------------------------------------------
// NTT(t1 2^d) (slots layout) and tr = H(pk) for every key row of a table
template <int LV>
__global__ void __launch_bounds__(64) ks_pk_k(const uint8_t *pk, int32_t *t1h, uint32_t nkeys) {
  using PP = P<LV>;
  constexpr int K = Lv<LV>::K;
  __shared__ int32_t trl[4 * NTT_LDS_GROUP];
  __shared__ uint32_t pkw[PP::PK / 4 + 2];
  uint32_t key = blockIdx.x;
  if (key >= nkeys) return;
  int lane = threadIdx.x, g = lane >> 4, t = lane & 15;
  const uint32_t *pkg = (const uint32_t *)(pk + (size_t)key * PP::PK);
  g2l_words<PP::PK / 4>(pkg, pkw, lane);
  if (lane < 2) pkw[PP::PK / 4 + lane] = 0;
  wave_sync();
  const Tw ftw = ntt_lane_tw(t);
  for (int i = g; i < K; i += 4) {
    uint32_t v[16];
    unpack_strided<10>(pkw + (32 + i * PP::T1B) / 4, v, t);
    int32_t x[16];
#pragma unroll
    for (int r = 0; r < 16; r++) x[r] = (int32_t)(v[r] << D);
    ntt16(x, ftw, trl + g * NTT_LDS_GROUP, t);
    store_slots(x, t1h + ((size_t)key * K + i) * N, t);
  }
}

template <int LV>
__global__ void __launch_bounds__(256) ks_tr_k(const uint8_t *pk, uint8_t *tr, uint32_t nkeys) {
  uint32_t key = blockIdx.x * blockDim.x + threadIdx.x;
  if (key >= nkeys) return;
  const uint8_t *p = pk + (size_t)key * P<LV>::PK;
  uint32_t s[50];
  shake_absorb<RATE256>(s, P<LV>::PK, [&](uint64_t pos) { return *(const uint64_t *)(p + pos); });
  uint32_t *o = (uint32_t *)(tr + (size_t)key * P<LV>::TRB);
#pragma unroll
  for (int w = 0; w < P<LV>::TRB / 4; w++) o[w] = s[w];
}

// ------------------------------------------------------------------------
// Primitive microbenchmarks
// ------------------------------------------------------------------------
// c_i = INTT(NTT(a_i) o b_i): b read as NTT-domain values; canonical output.
// 256-thread blocks, 16 polynomials per block per iteration, grid-stride.
// PAD = false is the bank-conflicted transpose of the optimisation ablation.
template <bool PAD>
__global__ void __launch_bounds__(256) ntt_mul_k(const int32_t *a, const int32_t *b, int32_t *c, uint64_t count) {
  __shared__ int32_t trl[16 * NTT_LDS_GROUP];
  int g = threadIdx.x >> 4, t = threadIdx.x & 15;
  int32_t *tr = trl + g * NTT_LDS_GROUP;
  const Tw ftw = ntt_lane_tw(t), itw = intt_lane_tw(t);
  for (uint64_t p = (uint64_t)blockIdx.x * 16 + g; p < count; p += (uint64_t)gridDim.x * 16) {
    int32_t x[16], y[16];
    load_strided(x, a + p * N, t);
    load_slots(y, b + p * N, t);
    ntt16<Tw, PAD>(x, ftw, tr, t);
#pragma unroll
    for (int r = 0; r < 16; r++) x[r] = mont_mul(x[r], y[r]);
    intt16<Tw, PAD>(x, itw, tr, t);
#pragma unroll
    for (int r = 0; r < 16; r++) x[r] = canon(x[r]);
    store_strided(x, c + p * N, t);
  }
}

// ExpandA rejection sampling of one polynomial per lane from a 34-byte input
__global__ void __launch_bounds__(EA_WG) expand_a_seed_k(const uint8_t *seeds, int32_t *out, uint64_t count) {
  uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  __shared__ uint32_t rows[EA_WG / 64][64 * EA_ROW];
  const bool valid = p < count;
  const uint8_t *sd = seeds + 34 * (valid ? p : 0);
  uint32_t s[50];
  uint32_t nonce = (uint32_t)sd[32] | ((uint32_t)sd[33] << 8);
  absorb_seed34(s, [&](int pos) { return load_le_bytes(sd + pos, 8); }, nonce);
  const int lane = threadIdx.x & 63;
  expand_a_squeeze_wave(s, out + (p - lane) * N, rows[threadIdx.x >> 6], lane, valid);
}

}  // namespace dil
