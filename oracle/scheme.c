/*
 * Oracle Dilithium.Gen / Sign / Verify (Alg. 1, 2, 3), parameters (Tab. 1),
 * encodings, and threaded batch drivers.
 * TEST INFRASTRUCTURE ONLY (see dil_oracle.h).
 *
 * Readings [R] (the paper fixes field order only; byte layouts follow the
 * public round-3 v3.1 specification):
 *   (rho, rho', K) = SHAKE256(zeta, 128 B) split 32 | 64 | 32 (Alg. 1; L1 = 256, L2 = 512 bits)
 *   tr = SHAKE256(pk, 32 B); mu = SHAKE256(tr || M, 64 B); rho' = SHAKE256(K || mu, 64 B);
 *   ctilde = SHAKE256(mu || packed w1, 32 B)            (Alg. 2, Alg. 3)
 *   pk  = rho || t1 (10-bit)                             sizes 1312 / 1952 / 2592
 *   sk  = rho || K || tr || s1 || s2 (eta - s, 3 or 4 bits) || t0 (2^12 - t0, 13 bits)
 *                                                        sizes 2528 / 4000 / 4864
 *   sig = ctilde || z (gamma1 - z, 18 or 20 bits) || h   sizes 2420 / 3293 / 4595
 *   w1  6 bits (gamma2 = (q-1)/88) or 4 bits (gamma2 = (q-1)/32)
 *   h   omega index bytes (ascending per polynomial) then k cumulative counts;
 *       Verify decodes strictly: counts non-decreasing and <= omega, indices
 *       strictly increasing within a polynomial, unused index bytes zero.
 *   Sign reduces t = A s1 + s2 to [0, q) before Power2Round; Sign's output is
 *   the first kappa in 0, l, 2l, ... whose candidate passes all four checks.
 *
 * ML-DSA (levels 44/65/87, FIPS 204 -- not in the paper, which covers round 3;
 * the standard is not available here, so these readings are from its published
 * algorithm, pinned by hashlib recomputation and the scheme properties only):
 *   parameters k, l, eta, tau, gamma1, gamma2, beta, omega of levels 2/3/5;
 *   lambda = 128 / 192 / 256, ctilde of lambda / 4 = 32 / 48 / 64 bytes
 *   (rho, rho', K) = SHAKE256(xi || k || l, 128 B)   (one byte each for k and l)
 *   tr = SHAKE256(pk, 64 B); sk = rho || K || tr (64 B) || s1 || s2 || t0
 *                                                        sizes 2560 / 4032 / 4896
 *   mu = SHAKE256(tr || 0x00 || 0x00 || M, 64 B)   (pure signing, empty context)
 *   rho'' = SHAKE256(K || rnd || mu, 64 B), rnd 32 bytes (zeros: deterministic)
 *   ctilde = SHAKE256(mu || packed w1, lambda / 4); SampleInBall absorbs all of it
 *   sig = ctilde || z || h                              sizes 2420 / 3309 / 4627
 *   ExpandA / ExpandS / ExpandMask, the encodings of t1, s, t0, z, w1 and h, the
 *   strict hint decoding and the rejection conditions are those of round 3.
 */
#include "dil_oracle.h"
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

int dil_ref_params(int level, ref_params *p) {
  memset(p, 0, sizeof *p);
  p->level = level;
  p->tr_bytes = 32;
  p->ct_bytes = 32;
  if (level == 44 || level == 65 || level == 87) {  /* ML-DSA-44 / 65 / 87 */
    const int base = level == 44 ? 2 : level == 65 ? 3 : 5;
    dil_ref_params(base, p);
    p->level = level;
    p->mldsa = 1;
    p->tr_bytes = 64;
    p->ct_bytes = level == 44 ? 32 : level == 65 ? 48 : 64;
    p->sk_bytes = 64 + (size_t)p->tr_bytes + (size_t)(p->l + p->k) * ORN * p->eta_bits / 8 + (size_t)p->k * ORN * 13 / 8;
    p->sig_bytes = (size_t)p->ct_bytes + (size_t)p->l * ORN * p->z_bits / 8 + p->omega + p->k;
    return 0;
  }
  switch (level) {
    case 2:
      p->k = 4; p->l = 4; p->eta = 2; p->tau = 39; p->gamma1 = 1 << 17; p->gamma2 = 95232;
      p->beta = 78; p->omega = 80;
      break;
    case 3:
      p->k = 6; p->l = 5; p->eta = 4; p->tau = 49; p->gamma1 = 1 << 19; p->gamma2 = 261888;
      p->beta = 196; p->omega = 55;
      break;
    case 5:
      p->k = 8; p->l = 7; p->eta = 2; p->tau = 60; p->gamma1 = 1 << 19; p->gamma2 = 261888;
      p->beta = 120; p->omega = 75;
      break;
    default:
      return -1;
  }
  p->z_bits = p->gamma1 == (1 << 17) ? 18 : 20;
  p->w1_bits = ((ORQ - 1) / (2 * p->gamma2)) == 44 ? 6 : 4;
  p->eta_bits = p->eta == 2 ? 3 : 4;
  p->w1_poly_bytes = (size_t)ORN * p->w1_bits / 8;
  p->pk_bytes = 32 + (size_t)p->k * ORN * 10 / 8;
  p->sk_bytes = 96 + (size_t)(p->l + p->k) * ORN * p->eta_bits / 8 + (size_t)p->k * ORN * 13 / 8;
  p->sig_bytes = 32 + (size_t)p->l * ORN * p->z_bits / 8 + p->omega + p->k;
  return 0;
}

static int64_t modq(int64_t x) {
  int64_t r = x % ORQ;
  return r < 0 ? r + ORQ : r;
}
static int32_t centred(int64_t x) { /* mod+- q, in (-(q-1)/2, (q-1)/2] */
  int64_t r = modq(x);
  return (int32_t)(r > (ORQ - 1) / 2 ? r - ORQ : r);
}
static int32_t iabs(int32_t x) { return x < 0 ? -x : x; }

/* ---- polynomial-vector helpers on canonical coefficients ---- */
static void to_canon(const int32_t *in, int32_t *out, size_t n) {
  for (size_t i = 0; i < n; i++) out[i] = (int32_t)modq(in[i]);
}
static void pointwise_acc(int32_t *acc, const int32_t *a, const int32_t *b) {
  for (int i = 0; i < ORN; i++) acc[i] = (int32_t)modq(acc[i] + modq((int64_t)a[i] * b[i]));
}
static void pointwise(int32_t *out, const int32_t *a, const int32_t *b) {
  for (int i = 0; i < ORN; i++) out[i] = (int32_t)modq((int64_t)a[i] * b[i]);
}

/* ---- encodings ---- */
static void pack_vals(const int32_t *v, int n, int b, uint8_t *out) {
  uint32_t *u = (uint32_t *)malloc(sizeof(uint32_t) * n);
  for (int i = 0; i < n; i++) u[i] = (uint32_t)v[i];
  dil_ref_bitpack(u, n, b, out);
  free(u);
}
static void unpack_vals(const uint8_t *in, int n, int b, int32_t *v) {
  uint32_t *u = (uint32_t *)malloc(sizeof(uint32_t) * n);
  dil_ref_bitunpack(in, n, b, u);
  for (int i = 0; i < n; i++) v[i] = (int32_t)u[i];
  free(u);
}

static void pack_eta(const ref_params *P, const int32_t *s /* centred */, uint8_t *out) {
  int32_t t[ORN];
  for (int i = 0; i < ORN; i++) t[i] = P->eta - s[i];
  pack_vals(t, ORN, P->eta_bits, out);
}
static void unpack_eta(const ref_params *P, const uint8_t *in, int32_t *s) {
  unpack_vals(in, ORN, P->eta_bits, s);
  for (int i = 0; i < ORN; i++) s[i] = P->eta - s[i];
}
static void pack_t0(const int32_t *t0, uint8_t *out) {
  int32_t t[ORN];
#if defined(DIL_PLANT) && DIL_PLANT == 14
  for (int i = 0; i < ORN; i++) t[i] = (1 << 12) + t0[i]; /* planted: t0 offset with the wrong sign */
#else
  for (int i = 0; i < ORN; i++) t[i] = (1 << 12) - t0[i];
#endif
  pack_vals(t, ORN, 13, out);
}
static void unpack_t0(const uint8_t *in, int32_t *t0) {
  unpack_vals(in, ORN, 13, t0);
  for (int i = 0; i < ORN; i++) t0[i] = (1 << 12) - t0[i];
}
static void pack_z(const ref_params *P, const int32_t *z, uint8_t *out) {
  int32_t t[ORN];
  for (int i = 0; i < ORN; i++) t[i] = P->gamma1 - z[i];
  pack_vals(t, ORN, P->z_bits, out);
}
static void unpack_z(const ref_params *P, const uint8_t *in, int32_t *z) {
  unpack_vals(in, ORN, P->z_bits, z);
  for (int i = 0; i < ORN; i++) z[i] = P->gamma1 - z[i];
}
static void pack_hint(const ref_params *P, const int32_t *h /* k*256 of 0/1 */, uint8_t *out) {
  memset(out, 0, P->omega + P->k);
  /* Sign calls this only with at most omega ones (Alg. 2's [h] <= omega
     condition); the guards keep a broken caller inside the buffer */
  int cnt = 0;
  for (int i = 0; i < P->k; i++) {
    for (int j = 0; j < ORN; j++)
      if (h[i * ORN + j]) {
        if (cnt < P->omega) out[cnt] = (uint8_t)j;
        cnt++;
      }
    out[P->omega + i] = (uint8_t)(cnt > 255 ? 255 : cnt);
  }
}
/* strict decoding; returns 0 ok, 1 malformed */
static int unpack_hint(const ref_params *P, const uint8_t *in, int32_t *h) {
  memset(h, 0, sizeof(int32_t) * P->k * ORN);
  int prev = 0;
  for (int i = 0; i < P->k; i++) {
    int cnt = in[P->omega + i];
    if (cnt < prev || cnt > P->omega) return 1;
    for (int j = prev; j < cnt; j++) {
      if (j > prev && in[j] <= in[j - 1]) return 1;
      h[i * ORN + in[j]] = 1;
    }
    prev = cnt;
  }
  for (int j = prev; j < P->omega; j++)
    if (in[j] != 0) return 1;
  return 0;
}

/* ---- Alg. 1 ---- */
int dil_ref_keygen(int level, const uint8_t zeta[32], uint8_t *pk, uint8_t *sk) {
  ref_params P;
  if (dil_ref_params(level, &P)) return -1;
  const int k = P.k, l = P.l;
  uint8_t seed[128], in[34];
  memcpy(in, zeta, 32);
  in[32] = (uint8_t)k;  /* ML-DSA only: the k and l bytes after the seed */
  in[33] = (uint8_t)l;
#if defined(DIL_PLANT) && DIL_PLANT == 20
  dil_ref_shake256(in, 32, seed, 128); /* planted: ML-DSA's k and l bytes left out of the seed expansion */
#else
  dil_ref_shake256(in, P.mldsa ? 34 : 32, seed, 128);
#endif
  const uint8_t *rho = seed, *rhop = seed + 32, *K = seed + 96;
  int32_t *A = (int32_t *)malloc(sizeof(int32_t) * k * l * ORN);
  int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (k + l) * ORN);
  int32_t *s1hat = (int32_t *)malloc(sizeof(int32_t) * l * ORN);
  int32_t *t1 = (int32_t *)malloc(sizeof(int32_t) * k * ORN);
  int32_t *t0 = (int32_t *)malloc(sizeof(int32_t) * k * ORN);
  dil_ref_expand_a(level, rho, A);
  dil_ref_expand_s(level, rhop, s);
  to_canon(s, s1hat, (size_t)l * ORN);
  for (int j = 0; j < l; j++) dil_ref_ntt(s1hat + j * ORN);
  for (int i = 0; i < k; i++) {
    int32_t acc[ORN];
    memset(acc, 0, sizeof acc);
    for (int j = 0; j < l; j++) pointwise_acc(acc, A + (i * l + j) * ORN, s1hat + j * ORN);
    dil_ref_intt(acc);
    for (int c = 0; c < ORN; c++) acc[c] = (int32_t)modq((int64_t)acc[c] + s[(l + i) * ORN + c]);
    dil_ref_power2round(acc, t1 + i * ORN, t0 + i * ORN, ORN);
  }
  memcpy(pk, rho, 32);
  for (int i = 0; i < k; i++) pack_vals(t1 + i * ORN, ORN, 10, pk + 32 + i * 320);
  uint8_t tr[64];
  dil_ref_shake256(pk, P.pk_bytes, tr, (size_t)P.tr_bytes);
  memcpy(sk, rho, 32);
  memcpy(sk + 32, K, 32);
  memcpy(sk + 64, tr, (size_t)P.tr_bytes);
  size_t eb = (size_t)ORN * P.eta_bits / 8, off = 64 + (size_t)P.tr_bytes;
  for (int j = 0; j < l; j++, off += eb) pack_eta(&P, s + j * ORN, sk + off);
  for (int i = 0; i < k; i++, off += eb) pack_eta(&P, s + (l + i) * ORN, sk + off);
  for (int i = 0; i < k; i++, off += 416) pack_t0(t0 + i * ORN, sk + off);
  free(A); free(s); free(s1hat); free(t1); free(t0);
  return 0;
}

static void pack_w1(const ref_params *P, const int32_t *w1, uint8_t *out) {
  for (int i = 0; i < P->k; i++) pack_vals(w1 + i * ORN, ORN, P->w1_bits, out + i * P->w1_poly_bytes);
}

/* ML-DSA's internal signing and verification take the formatted message M'
   (for the pure form 0x00 || |ctx| || ctx || M; for the pre-hash form 0x01 ||
   |ctx| || ctx || OID || PH(M)) and hash mu = H(tr || M', 64) */
static void mu_internal(const uint8_t tr[64], const uint8_t *mprime, size_t len, uint8_t mu[64]) {
#if defined(DIL_PLANT) && DIL_PLANT == 24
  dil_ref_mldsa_mu(tr, mprime, len, mu); /* planted: the formatted message formatted again */
#else
  uint8_t *buf = (uint8_t *)malloc(64 + len + 1);
  memcpy(buf, tr, 64);
  memcpy(buf + 64, mprime, len);
  dil_ref_shake256(buf, 64 + len, mu, 64);
  free(buf);
#endif
}

/* ML-DSA: mu = H(tr || IntegerToBytes(0, 1) || IntegerToBytes(|ctx|, 1) || ctx || M, 64)
   with an empty context ctx */
void dil_ref_mldsa_mu(const uint8_t tr[64], const uint8_t *msg, size_t mlen, uint8_t mu[64]) {
  uint8_t *buf = (uint8_t *)malloc(66 + mlen);
  memcpy(buf, tr, 64);
  buf[64] = 0;  /* pure ML-DSA, not the pre-hash variant */
  buf[65] = 0;  /* context length 0 */
  memcpy(buf + 66, msg, mlen);
#if defined(DIL_PLANT) && DIL_PLANT == 21
  memmove(buf + 64, buf + 66, mlen); /* planted: the two zero bytes before M dropped */
  dil_ref_shake256(buf, 64 + mlen, mu, 64);
#else
  dil_ref_shake256(buf, 66 + mlen, mu, 64);
#endif
  free(buf);
}

/* ---- Alg. 2 ---- */
/* Iteration cap of the rejection loop: a correct signer needs more than a few
   hundred iterations with negligible probability; the cap turns a broken
   variant (the planted-mistake tests) into a returned error instead of a hang. */
static int g_sign_cap = 100000;
void dil_ref_set_sign_cap(int cap) { g_sign_cap = cap > 0 ? cap : 100000; }

/* rnd == NULL: deterministic Sign, rho' = H(K || mu) (Alg. 2 as printed).
   rnd != NULL: the randomized variant of the round-3 scheme, rho' = the 64
   caller-supplied bytes; every other step is unchanged. */
static int sign_core(int level, int internal, const uint8_t *sk, const uint8_t *msg, size_t mlen, const uint8_t *rnd,
                     uint8_t *sig) {
  ref_params P;
  if (dil_ref_params(level, &P)) return -1;
  const int k = P.k, l = P.l;
  const uint8_t *rho = sk, *K = sk + 32, *tr = sk + 64;
  const size_t eb = (size_t)ORN * P.eta_bits / 8, so = 64 + (size_t)P.tr_bytes;  /* s1 offset in sk */
  int32_t *A = (int32_t *)malloc(sizeof(int32_t) * k * l * ORN);
  int32_t *s1h = (int32_t *)malloc(sizeof(int32_t) * l * ORN);
  int32_t *s2h = (int32_t *)malloc(sizeof(int32_t) * k * ORN);
  int32_t *t0h = (int32_t *)malloc(sizeof(int32_t) * k * ORN);
  int32_t *y = (int32_t *)malloc(sizeof(int32_t) * l * ORN);
  int32_t *yh = (int32_t *)malloc(sizeof(int32_t) * l * ORN);
  int32_t *w = (int32_t *)malloc(sizeof(int32_t) * k * ORN);
  int32_t *w1 = (int32_t *)malloc(sizeof(int32_t) * k * ORN);
  int32_t *z = (int32_t *)malloc(sizeof(int32_t) * l * ORN);
  int32_t *h = (int32_t *)malloc(sizeof(int32_t) * k * ORN);
  uint8_t *buf = (uint8_t *)malloc(130 + (size_t)k * P.w1_poly_bytes + mlen);

  /* round 3: mu = H(tr || M), rho' = H(K || mu) (or the caller's 64 bytes);
     ML-DSA: mu = H(tr || 0 || 0 || M), rho'' = H(K || rnd || mu), rnd 32 bytes */
  uint8_t mu[64], rhop[64];
  if (P.mldsa) {
    if (internal) mu_internal(tr, msg, mlen, mu);
    else dil_ref_mldsa_mu(tr, msg, mlen, mu);
    memcpy(buf, K, 32);
    if (rnd) memcpy(buf + 32, rnd, 32);
    else memset(buf + 32, 0, 32);
    memcpy(buf + 64, mu, 64);
#if defined(DIL_PLANT) && DIL_PLANT == 22
    memmove(buf + 32, buf + 64, 64); /* planted: rnd left out of rho'' = H(K || mu) */
    dil_ref_shake256(buf, 96, rhop, 64);
#else
    dil_ref_shake256(buf, 128, rhop, 64);
#endif
  } else {
    memcpy(buf, tr, 32);
    memcpy(buf + 32, msg, mlen);
    dil_ref_shake256(buf, 32 + mlen, mu, 64);
    if (rnd) {
      memcpy(rhop, rnd, 64);
    } else {
      memcpy(buf, K, 32);
      memcpy(buf + 32, mu, 64);
      dil_ref_shake256(buf, 96, rhop, 64);
    }
  }

  dil_ref_expand_a(level, rho, A);
  for (int j = 0; j < l; j++) {
    int32_t t[ORN];
    unpack_eta(&P, sk + so + j * eb, t);
    to_canon(t, s1h + j * ORN, ORN);
    dil_ref_ntt(s1h + j * ORN);
  }
  for (int i = 0; i < k; i++) {
    int32_t t[ORN];
    unpack_eta(&P, sk + so + (l + i) * eb, t);
    to_canon(t, s2h + i * ORN, ORN);
    dil_ref_ntt(s2h + i * ORN);
    unpack_t0(sk + so + (l + k) * eb + i * 416, t);
    to_canon(t, t0h + i * ORN, ORN);
    dil_ref_ntt(t0h + i * ORN);
  }

  uint32_t kappa = 0;
  int iters = 0;
  for (;;) {
    if (iters >= g_sign_cap) {
      memset(sig, 0, P.sig_bytes);
      iters = -2;
      break;
    }
    iters++;
    dil_ref_expand_mask(level, rhop, kappa, y);
    kappa += (uint32_t)l;
    to_canon(y, yh, (size_t)l * ORN);
    for (int j = 0; j < l; j++) dil_ref_ntt(yh + j * ORN);
    for (int i = 0; i < k; i++) {
      int32_t *acc = w + i * ORN;
      memset(acc, 0, sizeof(int32_t) * ORN);
      for (int j = 0; j < l; j++) pointwise_acc(acc, A + (i * l + j) * ORN, yh + j * ORN);
      dil_ref_intt(acc);
    }
    int32_t r0tmp[ORN];
    for (int i = 0; i < k; i++) dil_ref_decompose(w + i * ORN, w1 + i * ORN, r0tmp, ORN, P.gamma2);
    memcpy(buf, mu, 64);
    pack_w1(&P, w1, buf + 64);
    uint8_t ctilde[64];
    dil_ref_shake256(buf, 64 + (size_t)k * P.w1_poly_bytes, ctilde, (size_t)P.ct_bytes);
    int32_t c[ORN], ch[ORN];
    dil_ref_sample_in_ball(level, ctilde, c);
    to_canon(c, ch, ORN);
    dil_ref_ntt(ch);

    /* z = y + c s1 */
    int reject = 0;
    for (int j = 0; j < l && !reject; j++) {
      int32_t t[ORN];
      pointwise(t, ch, s1h + j * ORN);
      dil_ref_intt(t);
      for (int cidx = 0; cidx < ORN; cidx++) {
        z[j * ORN + cidx] = centred((int64_t)y[j * ORN + cidx] + t[cidx]);
#if defined(DIL_PLANT) && DIL_PLANT == 11
        if (iabs(z[j * ORN + cidx]) >= P.gamma1) reject = 1; /* planted: beta dropped from the z bound */
#else
        if (iabs(z[j * ORN + cidx]) >= P.gamma1 - P.beta) reject = 1;
#endif
      }
    }
    if (reject) continue;
    /* r0 = LowBits(w - c s2) */
    int32_t *wcs2 = (int32_t *)malloc(sizeof(int32_t) * k * ORN);
    for (int i = 0; i < k && !reject; i++) {
      int32_t t[ORN], r1[ORN], r0[ORN];
      pointwise(t, ch, s2h + i * ORN);
      dil_ref_intt(t);
      for (int cidx = 0; cidx < ORN; cidx++) wcs2[i * ORN + cidx] = (int32_t)modq((int64_t)w[i * ORN + cidx] - t[cidx]);
      dil_ref_decompose(wcs2 + i * ORN, r1, r0, ORN, P.gamma2);
      for (int cidx = 0; cidx < ORN; cidx++)
        if (iabs(r0[cidx]) >= P.gamma2 - P.beta) reject = 1;
    }
    if (reject) { free(wcs2); continue; }
    /* c t0, hint */
    int hcount = 0;
    for (int i = 0; i < k && !reject; i++) {
      int32_t t[ORN], negct0[ORN], r[ORN];
      pointwise(t, ch, t0h + i * ORN);
      dil_ref_intt(t);
      for (int cidx = 0; cidx < ORN; cidx++) {
#if !(defined(DIL_PLANT) && DIL_PLANT == 18) /* planted (18): the ||c t0|| >= gamma2 rejection dropped */
        if (iabs(centred(t[cidx])) >= P.gamma2) reject = 1;
#endif
        negct0[cidx] = (int32_t)modq(-(int64_t)t[cidx]);
#if defined(DIL_PLANT) && DIL_PLANT == 13
        r[cidx] = (int32_t)modq((int64_t)wcs2[i * ORN + cidx] - t[cidx]); /* planted: wrong sign of c t0 */
#else
        r[cidx] = (int32_t)modq((int64_t)wcs2[i * ORN + cidx] + t[cidx]);
#endif
      }
      dil_ref_make_hint(negct0, r, h + i * ORN, ORN, P.gamma2);
      for (int cidx = 0; cidx < ORN; cidx++) hcount += h[i * ORN + cidx];
    }
    free(wcs2);
#if defined(DIL_PLANT) && DIL_PLANT == 17
    if (reject) continue; /* planted: the [h] > omega rejection dropped */
#else
    if (reject || hcount > P.omega) continue;
#endif
    const size_t ct = (size_t)P.ct_bytes, zb = (size_t)ORN * P.z_bits / 8;
    memcpy(sig, ctilde, ct);
    for (int j = 0; j < l; j++) pack_z(&P, z + j * ORN, sig + ct + j * zb);
    pack_hint(&P, h, sig + ct + l * zb);
    break;
  }
  free(A); free(s1h); free(s2h); free(t0h); free(y); free(yh); free(w); free(w1); free(z); free(h); free(buf);
  return iters;
}

int dil_ref_sign(int level, const uint8_t *sk, const uint8_t *msg, size_t mlen, uint8_t *sig) {
  return sign_core(level, 0, sk, msg, mlen, NULL, sig);
}

int dil_ref_sign_rnd(int level, const uint8_t *sk, const uint8_t *msg, size_t mlen, const uint8_t *rnd,
                     uint8_t *sig) {
  return sign_core(level, 0, sk, msg, mlen, rnd, sig);
}

int dil_ref_mldsa_sign_internal(int level, const uint8_t *sk, const uint8_t *mprime, size_t len, const uint8_t *rnd,
                                uint8_t *sig) {
  ref_params P;
  if (dil_ref_params(level, &P) || !P.mldsa) return -1;
  return sign_core(level, 1, sk, mprime, len, rnd, sig);
}

/* ---- Alg. 3 ---- */
static int verify_core(int level, int internal, const uint8_t *pk, const uint8_t *msg, size_t mlen,
                       const uint8_t *sig) {
  ref_params P;
  if (dil_ref_params(level, &P)) return -1;
  const int k = P.k, l = P.l;
  const size_t zb = (size_t)ORN * P.z_bits / 8, ct = (size_t)P.ct_bytes;
  int32_t *z = (int32_t *)malloc(sizeof(int32_t) * l * ORN);
  int32_t *h = (int32_t *)malloc(sizeof(int32_t) * k * ORN);
  int32_t *A = (int32_t *)malloc(sizeof(int32_t) * k * l * ORN);
  int32_t *w1 = (int32_t *)malloc(sizeof(int32_t) * k * ORN);
  uint8_t *buf = (uint8_t *)malloc(130 + (size_t)k * P.w1_poly_bytes + mlen);
  int ok = 1;
  for (int j = 0; j < l; j++) unpack_z(&P, sig + ct + j * zb, z + j * ORN);
  if (unpack_hint(&P, sig + ct + l * zb, h)) ok = 0;
  for (int i = 0; i < l * ORN && ok; i++)
    if (iabs(z[i]) >= P.gamma1 - P.beta) ok = 0;
  if (ok) {
    uint8_t tr[64], mu[64], c2[64];
    dil_ref_shake256(pk, P.pk_bytes, tr, (size_t)P.tr_bytes);
    if (P.mldsa && internal) {
      mu_internal(tr, msg, mlen, mu);
    } else if (P.mldsa) {
      dil_ref_mldsa_mu(tr, msg, mlen, mu);
    } else {
      memcpy(buf, tr, 32);
      memcpy(buf + 32, msg, mlen);
      dil_ref_shake256(buf, 32 + mlen, mu, 64);
    }
    dil_ref_expand_a(level, pk, A);
    int32_t c[ORN], ch[ORN];
    dil_ref_sample_in_ball(level, sig, c);
    to_canon(c, ch, ORN);
    dil_ref_ntt(ch);
    int32_t *zh = (int32_t *)malloc(sizeof(int32_t) * l * ORN);
    to_canon(z, zh, (size_t)l * ORN);
    for (int j = 0; j < l; j++) dil_ref_ntt(zh + j * ORN);
    for (int i = 0; i < k; i++) {
      int32_t acc[ORN], t1[ORN], t[ORN];
      memset(acc, 0, sizeof acc);
      for (int j = 0; j < l; j++) pointwise_acc(acc, A + (i * l + j) * ORN, zh + j * ORN);
      unpack_vals(pk + 32 + i * 320, ORN, 10, t1);
      for (int cidx = 0; cidx < ORN; cidx++) t1[cidx] = (int32_t)modq((int64_t)t1[cidx] << 13);
      dil_ref_ntt(t1);
      pointwise(t, ch, t1);
#if !(defined(DIL_PLANT) && DIL_PLANT == 12) /* planted (12): the c t1 2^d term dropped */
      for (int cidx = 0; cidx < ORN; cidx++) acc[cidx] = (int32_t)modq((int64_t)acc[cidx] - t[cidx]);
#endif
      dil_ref_intt(acc);
      dil_ref_use_hint(h + i * ORN, acc, w1 + i * ORN, ORN, P.gamma2);
    }
    free(zh);
    memcpy(buf, mu, 64);
    pack_w1(&P, w1, buf + 64);
    dil_ref_shake256(buf, 64 + (size_t)k * P.w1_poly_bytes, c2, ct);
    if (memcmp(c2, sig, ct) != 0) ok = 0;
  }
  free(z); free(h); free(A); free(w1); free(buf);
  return ok;
}

int dil_ref_verify(int level, const uint8_t *pk, const uint8_t *msg, size_t mlen, const uint8_t *sig) {
  return verify_core(level, 0, pk, msg, mlen, sig);
}

int dil_ref_mldsa_verify_internal(int level, const uint8_t *pk, const uint8_t *mprime, size_t len,
                                  const uint8_t *sig) {
  ref_params P;
  if (dil_ref_params(level, &P) || !P.mldsa) return -1;
  return verify_core(level, 1, pk, mprime, len, sig);
}

/* ---- threaded batch drivers (tasks are independent) ---- */
typedef struct {
  int op, level, internal;
  const uint8_t *in_key, *msg, *sig_in, *seeds, *rnd;
  const uint32_t *key_idx;
  const uint64_t *msg_off;
  uint8_t *pk, *sk, *sig;
  int32_t *verdict, *iters;
  size_t lo, hi;
  ref_params P;
} batch_job;

static void *batch_worker(void *arg) {
  batch_job *j = (batch_job *)arg;
  for (size_t t = j->lo; t < j->hi; t++) {
    if (j->op == 0) {
      dil_ref_keygen(j->level, j->seeds + 32 * t, j->pk + j->P.pk_bytes * t, j->sk + j->P.sk_bytes * t);
    } else {
      size_t key = j->key_idx ? j->key_idx[t] : t;
      const uint8_t *m = j->msg + j->msg_off[t];
      size_t mlen = (size_t)(j->msg_off[t + 1] - j->msg_off[t]);
      if (j->op == 1) {
        int it = sign_core(j->level, j->internal, j->in_key + j->P.sk_bytes * key, m, mlen,
                           j->rnd ? j->rnd + (j->P.mldsa ? 32 : 64) * (size_t)t : NULL,
                           j->sig + j->P.sig_bytes * t);
        if (j->iters) j->iters[t] = it;
      } else {
        j->verdict[t] = verify_core(j->level, j->internal, j->in_key + j->P.pk_bytes * key, m, mlen,
                                    j->sig_in + j->P.sig_bytes * t);
      }
    }
  }
  return NULL;
}

static int run_batch(batch_job *proto, uint32_t count, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if ((uint32_t)nthreads > count) nthreads = count ? (int)count : 1;
  pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
  batch_job *jobs = (batch_job *)calloc(nthreads, sizeof(batch_job));
  for (int t = 0; t < nthreads; t++) {
    jobs[t] = *proto;
    jobs[t].lo = (size_t)count * t / nthreads;
    jobs[t].hi = (size_t)count * (t + 1) / nthreads;
    pthread_create(&th[t], NULL, batch_worker, &jobs[t]);
  }
  for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
  return 0;
}

int dil_ref_keygen_batch(int level, const uint8_t *seeds, uint8_t *pk, uint8_t *sk, uint32_t count, int nthreads) {
  batch_job j;
  memset(&j, 0, sizeof j);
  if (dil_ref_params(level, &j.P)) return -1;
  j.op = 0; j.level = level; j.seeds = seeds; j.pk = pk; j.sk = sk;
  return run_batch(&j, count, nthreads);
}

int dil_ref_sign_batch_ex(int level, int internal, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                          const uint64_t *msg_off, const uint8_t *rnd, uint8_t *sig, uint32_t count, int nthreads,
                          int32_t *iters) {
  batch_job j;
  memset(&j, 0, sizeof j);
  if (dil_ref_params(level, &j.P) || (internal && !j.P.mldsa)) return -1;
  j.internal = internal;
  for (uint32_t t = 0; t < count; t++)
    if (msg_off[t + 1] < msg_off[t]) return -1;
  j.op = 1; j.level = level; j.in_key = sk; j.key_idx = key_idx; j.msg = msg; j.msg_off = msg_off;
  j.sig = sig; j.iters = iters; j.rnd = rnd;
  return run_batch(&j, count, nthreads);
}

int dil_ref_sign_batch_rnd(int level, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                           const uint64_t *msg_off, const uint8_t *rnd, uint8_t *sig, uint32_t count, int nthreads,
                           int32_t *iters) {
  return dil_ref_sign_batch_ex(level, 0, sk, key_idx, msg, msg_off, rnd, sig, count, nthreads, iters);
}

int dil_ref_sign_batch(int level, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                       const uint64_t *msg_off, uint8_t *sig, uint32_t count, int nthreads, int32_t *iters) {
  return dil_ref_sign_batch_rnd(level, sk, key_idx, msg, msg_off, NULL, sig, count, nthreads, iters);
}

int dil_ref_verify_batch_ex(int level, int internal, const uint8_t *pk, const uint32_t *key_idx, const uint8_t *msg,
                            const uint64_t *msg_off, const uint8_t *sig, int32_t *verdict, uint32_t count,
                            int nthreads) {
  batch_job j;
  memset(&j, 0, sizeof j);
  if (dil_ref_params(level, &j.P) || (internal && !j.P.mldsa)) return -1;
  j.internal = internal;
  for (uint32_t t = 0; t < count; t++)
    if (msg_off[t + 1] < msg_off[t]) return -1;
  j.op = 2; j.level = level; j.in_key = pk; j.key_idx = key_idx; j.msg = msg; j.msg_off = msg_off;
  j.sig_in = sig; j.verdict = verdict;
  return run_batch(&j, count, nthreads);
}

int dil_ref_verify_batch(int level, const uint8_t *pk, const uint32_t *key_idx, const uint8_t *msg,
                         const uint64_t *msg_off, const uint8_t *sig, int32_t *verdict, uint32_t count,
                         int nthreads) {
  return dil_ref_verify_batch_ex(level, 0, pk, key_idx, msg, msg_off, sig, verdict, count, nthreads);
}
