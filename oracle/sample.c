/*
 * Oracle samplers (Sec. 2.3 "Sampling"; Alg. 1 ExpandA/ExpandS, Alg. 2
 * ExpandMask/SampleInBall) and the generic bit packing used by every encoding.
 * TEST INFRASTRUCTURE ONLY (see dil_oracle.h).
 *
 * Each sampler squeezes its whole stream from a plain SHAKE call and consumes
 * it sequentially, one candidate at a time, in stream order.
 * Readings [R] (the paper gives only the output ranges):
 *   ExpandA      stream SHAKE128(rho || j || i) for row i, column j; 3 bytes
 *                b0 b1 b2 -> t = b0 + 2^8 b1 + 2^16 (b2 mod 128); keep t < q
 *                until 256 kept; the values are NTT-domain coefficients.
 *   ExpandS      s1[r] = SHAKE256(rho' || LE16(r)), s2[r] = SHAKE256(rho' || LE16(l + r));
 *                low nibble then high nibble of each byte; eta = 2: keep < 15,
 *                coefficient 2 - (v mod 5); eta = 4: keep < 9, coefficient 4 - v.
 *   ExpandMask   y_i = SHAKE256(rho' || LE16(kappa + i)) read LSB-first as
 *                18-bit (gamma1 = 2^17) or 20-bit (gamma1 = 2^19) values v;
 *                coefficient gamma1 - v.
 *   SampleInBall SHAKE256(ctilde): 8 bytes form a little-endian sign word s;
 *                for i = 256 - tau .. 255 draw bytes until b <= i, then
 *                c_i = c_b, c_b = (-1)^(s & 1), s >>= 1.
 * Pinned (tests/test_oracle_samplers.py, statistically, from properties of a
 * uniform byte stream that hold whatever the byte order):
 *   ExpandA      accepted / examined candidates = q / 2^23 (the 23-bit mask);
 *                values uniform on [0, q).
 *   ExpandS      accepted / examined nibbles = 15/16 (eta = 2) or 9/16 (eta = 4);
 *                coefficients uniform on [-eta, eta].
 *   SampleInBall exactly tau entries +-1; the support is a uniform tau-subset of
 *                the 256 positions, which is the textbook property of the
 *                Fisher-Yates draw with b <= i (b < i biases the positions).
 *   ExpandMask   range [-gamma1 + 1, gamma1], stream i of kappa = nonce kappa + i.
 * parity unpinned: the byte and nibble order inside each stream, the nonce
 *   encodings, ExpandMask's orientation (gamma1 - v rather than v - gamma1 + 1)
 *   and SampleInBall's sign-bit source; the paper fixes none of them and no
 *   official round-3 byte streams (KATs) are available here.
 */
#include "dil_oracle.h"
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

void dil_ref_bitpack(const uint32_t *v, size_t n, int b, uint8_t *out) {
  memset(out, 0, (n * b + 7) / 8);
  for (size_t i = 0; i < n; i++)
    for (int t = 0; t < b; t++) {
      size_t bit = i * b + t;
#if defined(DIL_PLANT) && DIL_PLANT == 9
      if ((v[i] >> t) & 1) out[bit / 8] |= (uint8_t)(0x80u >> (bit % 8)); /* planted: MSB-first packing */
#else
      if ((v[i] >> t) & 1) out[bit / 8] |= (uint8_t)(1u << (bit % 8));
#endif
    }
}

void dil_ref_bitunpack(const uint8_t *in, size_t n, int b, uint32_t *v) {
  for (size_t i = 0; i < n; i++) {
    uint32_t x = 0;
    for (int t = 0; t < b; t++) {
      size_t bit = i * b + t;
      x |= (uint32_t)((in[bit / 8] >> (bit % 8)) & 1) << t;
    }
    v[i] = x;
  }
}

/* rejection sampling needs an unbounded stream; squeeze generously and grow on demand */
typedef struct {
  uint8_t *buf;
  size_t len, pos;
  int xof128;
  uint8_t seed[80];
  size_t seedlen;
} stream_t;

static void stream_open(stream_t *s, int xof128, const uint8_t *seed, size_t seedlen, size_t first) {
  s->xof128 = xof128;
  memcpy(s->seed, seed, seedlen);
  s->seedlen = seedlen;
  s->len = first;
  s->pos = 0;
  s->buf = (uint8_t *)malloc(first);
  if (xof128) dil_ref_shake128(seed, seedlen, s->buf, first);
  else dil_ref_shake256(seed, seedlen, s->buf, first);
}

static uint8_t stream_byte(stream_t *s) {
  if (s->pos == s->len) { /* re-squeeze a longer prefix: SHAKE output is a prefix-stable stream */
    size_t nl = s->len * 2;
    uint8_t *nb = (uint8_t *)malloc(nl);
    if (s->xof128) dil_ref_shake128(s->seed, s->seedlen, nb, nl);
    else dil_ref_shake256(s->seed, s->seedlen, nb, nl);
    free(s->buf);
    s->buf = nb;
    s->len = nl;
  }
  return s->buf[s->pos++];
}

static void stream_close(stream_t *s) { free(s->buf); }

size_t dil_ref_expand_a_poly_counted(const uint8_t seed34[34], int32_t out[ORN]) {
  stream_t s;
  stream_open(&s, 1, seed34, 34, 840);
  int ctr = 0;
  size_t candidates = 0;
  while (ctr < ORN) {
    uint32_t b0 = stream_byte(&s), b1 = stream_byte(&s), b2 = stream_byte(&s);
#if defined(DIL_PLANT) && DIL_PLANT == 15
    uint32_t t = b0 | (b1 << 8) | (b2 << 16); /* planted: the 23-bit mask dropped */
#else
    uint32_t t = b0 | (b1 << 8) | ((b2 & 0x7F) << 16);
#endif
    candidates++;
    if (t < ORQ) out[ctr++] = (int32_t)t;
  }
  stream_close(&s);
  return candidates;
}

void dil_ref_expand_a_poly(const uint8_t seed34[34], int32_t out[ORN]) { (void)dil_ref_expand_a_poly_counted(seed34, out); }

int dil_ref_params(int level, ref_params *p);

void dil_ref_expand_a(int level, const uint8_t rho[32], int32_t *A) {
  ref_params P;
  if (dil_ref_params(level, &P)) return;
  uint8_t seed[34];
  memcpy(seed, rho, 32);
  for (int i = 0; i < P.k; i++)
    for (int j = 0; j < P.l; j++) {
      seed[32] = (uint8_t)j;
      seed[33] = (uint8_t)i;
      dil_ref_expand_a_poly(seed, A + ((size_t)i * P.l + j) * ORN);
    }
}

typedef struct {
  const uint8_t *seeds;
  int32_t *out;
  size_t lo, hi;
} ea_job;

static void *ea_worker(void *arg) {
  ea_job *j = (ea_job *)arg;
  for (size_t p = j->lo; p < j->hi; p++) dil_ref_expand_a_poly(j->seeds + 34 * p, j->out + ORN * p);
  return NULL;
}

void dil_ref_expand_a_polys(const uint8_t *seeds34, int32_t *out, size_t count, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if ((size_t)nthreads > count) nthreads = count ? (int)count : 1;
  pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
  ea_job *jobs = (ea_job *)calloc(nthreads, sizeof(ea_job));
  for (int t = 0; t < nthreads; t++) {
    jobs[t].seeds = seeds34; jobs[t].out = out;
    jobs[t].lo = count * t / nthreads;
    jobs[t].hi = count * (t + 1) / nthreads;
    pthread_create(&th[t], NULL, ea_worker, &jobs[t]);
  }
  for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
}

size_t dil_ref_expand_s_poly_counted(int eta, const uint8_t rhop[64], uint16_t nonce, int32_t out[ORN]) {
  uint8_t seed[66];
  memcpy(seed, rhop, 64);
  seed[64] = (uint8_t)(nonce & 0xFF);
  seed[65] = (uint8_t)(nonce >> 8);
  stream_t s;
  stream_open(&s, 0, seed, 66, 272);
  int ctr = 0;
  size_t nibbles = 0;
  while (ctr < ORN) {
    uint8_t b = stream_byte(&s);
    uint32_t half[2] = {b & 0x0Fu, (uint32_t)b >> 4};
    for (int h = 0; h < 2 && ctr < ORN; h++) {
      uint32_t v = half[h];
      nibbles++;
#if defined(DIL_PLANT) && DIL_PLANT == 16
      if (eta == 2 && v < 16) out[ctr++] = 2 - (int32_t)(v % 5); /* planted: eta = 2 threshold 16 */
#else
      if (eta == 2 && v < 15) out[ctr++] = 2 - (int32_t)(v % 5);
#endif
      else if (eta == 4 && v < 9) out[ctr++] = 4 - (int32_t)v;
    }
  }
  stream_close(&s);
  return nibbles;
}

void dil_ref_expand_s(int level, const uint8_t rhop[64], int32_t *s) {
  ref_params P;
  if (dil_ref_params(level, &P)) return;
  for (int r = 0; r < P.l + P.k; r++) (void)dil_ref_expand_s_poly_counted(P.eta, rhop, (uint16_t)r, s + (size_t)r * ORN);
}

void dil_ref_expand_mask(int level, const uint8_t rhop[64], uint32_t kappa, int32_t *y) {
  ref_params P;
  if (dil_ref_params(level, &P)) return;
  int b = P.z_bits;
  for (int i = 0; i < P.l; i++) {
    uint16_t nonce = (uint16_t)((kappa + (uint32_t)i) & 0xFFFF);
    uint8_t seed[66];
    memcpy(seed, rhop, 64);
    seed[64] = (uint8_t)(nonce & 0xFF);
    seed[65] = (uint8_t)(nonce >> 8);
    size_t nbytes = (size_t)ORN * b / 8;
    uint8_t *buf = (uint8_t *)malloc(nbytes);
    dil_ref_shake256(seed, 66, buf, nbytes);
    uint32_t v[ORN];
    dil_ref_bitunpack(buf, ORN, b, v);
    for (int c = 0; c < ORN; c++) y[(size_t)i * ORN + c] = P.gamma1 - (int32_t)v[c];
    free(buf);
  }
}

void dil_ref_sample_in_ball(int level, const uint8_t *ctilde, int32_t c[ORN]) {
  ref_params P;
  if (dil_ref_params(level, &P)) return;
  stream_t s;
#if defined(DIL_PLANT) && DIL_PLANT == 23
  stream_open(&s, 0, ctilde, 32, 136);  /* planted: only the first 32 bytes of ctilde seed it */
#else
  stream_open(&s, 0, ctilde, (size_t)P.ct_bytes, 136);  /* ML-DSA: the whole lambda/4-byte ctilde seeds it */
#endif
  uint64_t signs = 0;
  for (int i = 0; i < 8; i++) signs |= (uint64_t)stream_byte(&s) << (8 * i);
  for (int i = 0; i < ORN; i++) c[i] = 0;
  for (int i = ORN - P.tau; i < ORN; i++) {
    int b;
#if defined(DIL_PLANT) && DIL_PLANT == 19
    do { b = stream_byte(&s); } while (b >= i); /* planted: positions drawn with b < i */
#else
    do { b = stream_byte(&s); } while (b > i);
#endif
    c[i] = c[b];
#if defined(DIL_PLANT) && DIL_PLANT == 10
    c[b] = (signs & 1) ? -1 : 1;
    if (i == ORN - 1) c[b] = 0; /* planted: last position dropped */
#else
    c[b] = (signs & 1) ? -1 : 1;
#endif
    signs >>= 1;
  }
  stream_close(&s);
}
