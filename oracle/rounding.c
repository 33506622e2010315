/*
 * Oracle bit extraction and hints (Sec. 2.3, "Bits Extraction and Hints").
 * TEST INFRASTRUCTURE ONLY (see dil_oracle.h).
 *
 * mod+- alpha returns the representative in (-floor((alpha+1)/2), floor(alpha/2)]
 * (Sec. 2.1, Notation).  Each function is written from its definition:
 *   Power2Round(r, d=13): r0 = r+ mod+- 2^13, r1 = (r+ - r0) / 2^13.
 *   Decompose(r, alpha=2 gamma2): r0 = r+ mod+- alpha; if r+ - r0 = q - 1 then
 *       (r1, r0) = (0, r0 - 1) else r1 = (r+ - r0) / alpha.
 *   HighBits -> r1, LowBits -> r0  [R: the prose names them the other way
 *       round, their use in Alg. 2 fixes this order].
 *   MakeHint(z, r) = [HighBits(r) != HighBits(r + z)]  [R: the printed
 *       definition compares with an undefined v1; read as HighBits(r + z)].
 *   UseHint(h, r): m = (q-1)/alpha; r1 if h = 0, else (r1 + 1) mod+ m when
 *       r0 > 0 and (r1 - 1) mod+ m when r0 <= 0.
 * Pinned by exhaustive identities over [0, q) and the hint-correctness property.
 */
#include "dil_oracle.h"

static int64_t modp(int64_t x, int64_t m) { /* mod+ : [0, m) */
  int64_t r = x % m;
  return r < 0 ? r + m : r;
}

static int64_t modpm(int64_t x, int64_t alpha) { /* mod+- : (-floor((a+1)/2), floor(a/2)] */
  int64_t r = modp(x, alpha);
#if defined(DIL_PLANT) && DIL_PLANT == 5
  if (r >= alpha / 2) r -= alpha; /* planted: tie goes to the negative side */
#else
  if (r > alpha / 2) r -= alpha;
#endif
  return r;
}

static void p2r(int64_t r, int32_t *r1, int32_t *r0) {
  int64_t rp = modp(r, ORQ);
  int64_t a0 = modpm(rp, 1 << 13);
  *r0 = (int32_t)a0;
  *r1 = (int32_t)((rp - a0) >> 13);
}

static void decomp(int64_t r, int64_t gamma2, int32_t *r1, int32_t *r0) {
  int64_t alpha = 2 * gamma2;
  int64_t rp = modp(r, ORQ);
  int64_t lo = modpm(rp, alpha);
#if defined(DIL_PLANT) && DIL_PLANT == 6
  if (0) { /* planted: Decompose special case dropped */
#else
  if (rp - lo == ORQ - 1) {
#endif
    *r1 = 0;
    *r0 = (int32_t)(lo - 1);
  } else {
    *r1 = (int32_t)((rp - lo) / alpha);
    *r0 = (int32_t)lo;
  }
}

void dil_ref_power2round(const int32_t *r, int32_t *r1, int32_t *r0, size_t n) {
  for (size_t i = 0; i < n; i++) p2r(r[i], &r1[i], &r0[i]);
}

void dil_ref_decompose(const int32_t *r, int32_t *r1, int32_t *r0, size_t n, int32_t gamma2) {
  for (size_t i = 0; i < n; i++) decomp(r[i], gamma2, &r1[i], &r0[i]);
}

void dil_ref_make_hint(const int32_t *z, const int32_t *r, int32_t *h, size_t n, int32_t gamma2) {
  for (size_t i = 0; i < n; i++) {
    int32_t a1, a0, b1, b0;
    decomp(r[i], gamma2, &a1, &a0);
#if defined(DIL_PLANT) && DIL_PLANT == 7
    decomp((int64_t)r[i] - z[i], gamma2, &b1, &b0); /* planted: wrong sign of z */
#else
    decomp((int64_t)r[i] + z[i], gamma2, &b1, &b0);
#endif
    h[i] = a1 != b1;
  }
}

void dil_ref_use_hint(const int32_t *h, const int32_t *r, int32_t *out, size_t n, int32_t gamma2) {
  int64_t m = (ORQ - 1) / (2 * gamma2);
  for (size_t i = 0; i < n; i++) {
    int32_t r1, r0;
    decomp(r[i], gamma2, &r1, &r0);
    if (h[i] == 0) out[i] = r1;
#if defined(DIL_PLANT) && DIL_PLANT == 8
    else if (r0 >= 0) out[i] = (int32_t)modp((int64_t)r1 + 1, m); /* planted: r0 = 0 takes the + branch */
#else
    else if (r0 > 0) out[i] = (int32_t)modp((int64_t)r1 + 1, m);
#endif
    else out[i] = (int32_t)modp((int64_t)r1 - 1, m);
  }
}
