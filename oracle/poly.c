/*
 * Oracle ring arithmetic in R_q = Z_q[X]/(X^256 + 1), q = 8380417 (Sec. 2.2).
 * TEST INFRASTRUCTURE ONLY (see dil_oracle.h).
 *
 * Representation: canonical int32 in [0, q).  Every product is formed in
 * int64 and reduced with '%' followed by canonicalisation.
 *
 * NTT reading [R] (the printed formula in Sec. 2.2 swaps i and j, which would
 * give a twisted cyclic transform): with psi = 1753, a primitive 512-th root
 * of unity mod q, output slot j holds f evaluated at psi^(2 brv8(j) + 1):
 *     fhat_j = sum_i f_i psi^((2 brv8(j) + 1) i),
 *     f_i    = 256^-1 sum_j fhat_j psi^(-(2 brv8(j) + 1) i),
 * so that f * g = INTT(NTT f o NTT g) is the negacyclic product.  The fast
 * transforms below are the textbook in-place radix-2 forms (Cooley-Tukey
 * forward, Gentleman-Sande inverse) whose block k uses psi^brv8(k); tests pin
 * them to the O(n^2) definition and to schoolbook negacyclic multiplication.
 */
#include "dil_oracle.h"
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define PSI 1753

static int64_t modq(int64_t x) {
  int64_t r = x % ORQ;
  return r < 0 ? r + ORQ : r;
}

static int64_t powmod(int64_t b, int64_t e) {
  int64_t r = 1;
  b = modq(b);
  while (e > 0) {
    if (e & 1) r = modq(r * b);
    b = modq(b * b);
    e >>= 1;
  }
  return r;
}

static int brv8(int k) {
  int r = 0;
  for (int i = 0; i < 8; i++)
    if (k & (1 << i)) r |= 1 << (7 - i);
  return r;
}

void dil_ref_ntt(int32_t a[ORN]) {
  int k = 0;
  for (int len = 128; len >= 1; len >>= 1) {
    for (int start = 0; start < ORN; start += 2 * len) {
      k++;
#if defined(DIL_PLANT) && DIL_PLANT == 3
      int64_t zeta = powmod(PSI, k); /* planted: twiddle index not bit-reversed */
#else
      int64_t zeta = powmod(PSI, brv8(k));
#endif
      for (int j = start; j < start + len; j++) {
        int64_t t = modq(zeta * a[j + len]);
        int64_t u = a[j];
        a[j + len] = (int32_t)modq(u - t);
        a[j] = (int32_t)modq(u + t);
      }
    }
  }
}

void dil_ref_intt(int32_t a[ORN]) {
  for (int len = 1; len <= 128; len <<= 1) {
    for (int start = 0; start < ORN; start += 2 * len) {
      int k = 128 / len + start / (2 * len); /* the block index the forward pass used */
      int64_t zeta_inv = powmod(PSI, 512 - brv8(k));
      for (int j = start; j < start + len; j++) {
        int64_t x = a[j], y = a[j + len];
        a[j] = (int32_t)modq(x + y);
        a[j + len] = (int32_t)modq(modq(x - y) * zeta_inv);
      }
    }
  }
#if defined(DIL_PLANT) && DIL_PLANT == 4
  int64_t ninv = 1; /* planted: 1/n dropped */
#else
  int64_t ninv = powmod(ORN, ORQ - 2); /* 256^-1 mod q by Fermat */
#endif
  for (int i = 0; i < ORN; i++) a[i] = (int32_t)modq(a[i] * ninv);
}

void dil_ref_ntt_definition(const int32_t a[ORN], int32_t out[ORN]) {
  for (int j = 0; j < ORN; j++) {
    int64_t root = powmod(PSI, 2 * brv8(j) + 1);
    int64_t acc = 0, p = 1;
    for (int i = 0; i < ORN; i++) {
      acc = modq(acc + modq((int64_t)a[i] * p));
      p = modq(p * root);
    }
    out[j] = (int32_t)acc;
  }
}

void dil_ref_poly_mul_schoolbook(const int32_t a[ORN], const int32_t b[ORN], int32_t out[ORN]) {
  int64_t acc[ORN];
  memset(acc, 0, sizeof acc);
  for (int i = 0; i < ORN; i++)
    for (int j = 0; j < ORN; j++) {
      int64_t p = modq((int64_t)a[i] * b[j]);
      if (i + j < ORN) acc[i + j] = modq(acc[i + j] + p);
      else acc[i + j - ORN] = modq(acc[i + j - ORN] - p); /* X^256 = -1 */
    }
  for (int i = 0; i < ORN; i++) out[i] = (int32_t)acc[i];
}

typedef struct {
  const int32_t *a, *b;
  int32_t *c;
  size_t lo, hi;
} nm_job;

static void *ntt_mul_worker(void *arg) {
  nm_job *j = (nm_job *)arg;
  int32_t t[ORN];
  for (size_t p = j->lo; p < j->hi; p++) {
    memcpy(t, j->a + p * ORN, sizeof t);
    dil_ref_ntt(t);
    for (int i = 0; i < ORN; i++) t[i] = (int32_t)modq((int64_t)t[i] * j->b[p * ORN + i]);
    dil_ref_intt(t);
    memcpy(j->c + p * ORN, t, sizeof t);
  }
  return NULL;
}

void dil_ref_ntt_mul_batch(const int32_t *a, const int32_t *b, int32_t *c, size_t count, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if ((size_t)nthreads > count) nthreads = count ? (int)count : 1;
  pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
  nm_job *jobs = (nm_job *)calloc(nthreads, sizeof(nm_job));
  for (int t = 0; t < nthreads; t++) {
    jobs[t].a = a; jobs[t].b = b; jobs[t].c = c;
    jobs[t].lo = count * t / nthreads;
    jobs[t].hi = count * (t + 1) / nthreads;
    pthread_create(&th[t], NULL, ntt_mul_worker, &jobs[t]);
  }
  for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
}
