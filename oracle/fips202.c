/*
 * Oracle Keccak-f[1600] and SHAKE128/256, written from the FIPS 202 definitions.
 * TEST INFRASTRUCTURE ONLY (see dil_oracle.h).
 *
 * The paper fixes SHAKE128/256 as the XOF and SHAKE256 as the hash H
 * (Sec. 2.3, "Sampling").  Everything here is the standard's text:
 *   state      5x5 lanes of 64 bits; lane (x, y) is state word x + 5y and the
 *              byte string S maps to lanes little-endian (S[8(x+5y)+i] is byte i);
 *   round      theta, rho, pi, chi, iota, 24 rounds;
 *   rc(t)      output bit of the degree-8 LFSR x^8 + x^6 + x^5 + x^4 + 1;
 *   RC[ir]     bit 2^j - 1 = rc(j + 7 ir), j = 0..6;
 *   rho offset for (x, y) visited by (x, y) <- (y, 2x + 3y) from (1, 0):
 *              (t+1)(t+2)/2 mod 64 at step t;
 *   SHAKE      pad M || 1111 || 10*1, rate 168 (SHAKE128) or 136 (SHAKE256).
 * Pinned exactly by Python hashlib in the oracle tests.
 */
#include "dil_oracle.h"
#include <pthread.h>
#include <string.h>

static uint64_t g_rc[24];
static int g_rho[25];
static pthread_once_t g_once = PTHREAD_ONCE_INIT;

/* rc(t): FIPS 202 Algorithm 5 */
static int rc_bit(int t) {
  if (t % 255 == 0) return 1;
  unsigned R = 1; /* R[0] = 1, R[1..7] = 0; bit i of the integer is R[i] */
  for (int i = 1; i <= t % 255; i++) {
    R <<= 1;                 /* R = 0 || R  (9 bits) */
    unsigned r8 = (R >> 8) & 1;
    R ^= r8 << 0;
    R ^= r8 << 4;
    R ^= r8 << 5;
    R ^= r8 << 6;
    R &= 0xFF;               /* Trunc_8 */
  }
  return R & 1;
}

static void keccak_init_once(void) {
  for (int ir = 0; ir < 24; ir++) {
    uint64_t rc = 0;
    for (int j = 0; j <= 6; j++)
      if (rc_bit(j + 7 * ir)) rc |= (uint64_t)1 << ((1 << j) - 1);
    g_rc[ir] = rc;
  }
  memset(g_rho, 0, sizeof g_rho);
  int x = 1, y = 0;
  for (int t = 0; t < 24; t++) {
    g_rho[x + 5 * y] = ((t + 1) * (t + 2) / 2) % 64;
#if defined(DIL_PLANT) && DIL_PLANT == 1
    if (t == 7) g_rho[x + 5 * y] = (g_rho[x + 5 * y] + 1) % 64; /* planted: one wrong rotation offset */
#endif
    int nx = y, ny = (2 * x + 3 * y) % 5;
    x = nx; y = ny;
  }
}

static void keccak_init(void) { pthread_once(&g_once, keccak_init_once); }

static uint64_t rotl64(uint64_t v, int n) {
  n &= 63;
  if (n == 0) return v;
  return (v << n) | (v >> (64 - n));
}

void dil_ref_keccak_f1600(uint64_t A[25]) {
  keccak_init();
  for (int ir = 0; ir < 24; ir++) {
    uint64_t C[5], D[5], B[25];
    /* theta */
    for (int x = 0; x < 5; x++)
      C[x] = A[x] ^ A[x + 5] ^ A[x + 10] ^ A[x + 15] ^ A[x + 20];
    for (int x = 0; x < 5; x++)
      D[x] = C[(x + 4) % 5] ^ rotl64(C[(x + 1) % 5], 1);
    for (int y = 0; y < 5; y++)
      for (int x = 0; x < 5; x++) A[x + 5 * y] ^= D[x];
    /* rho and pi: B[y, 2x+3y] = rot(A[x, y], r[x, y])  (equivalently A'[x,y] = A[x+3y, x]) */
    for (int y = 0; y < 5; y++)
      for (int x = 0; x < 5; x++) {
        int X = y, Y = (2 * x + 3 * y) % 5;
        B[X + 5 * Y] = rotl64(A[x + 5 * y], g_rho[x + 5 * y]);
      }
    /* chi */
    for (int y = 0; y < 5; y++)
      for (int x = 0; x < 5; x++)
#if defined(DIL_PLANT) && DIL_PLANT == 2
        A[x + 5 * y] = B[x + 5 * y] ^ (B[(x + 1) % 5 + 5 * y] & (~B[(x + 2) % 5 + 5 * y])); /* planted: chi operands swapped */
#else
        A[x + 5 * y] = B[x + 5 * y] ^ ((~B[(x + 1) % 5 + 5 * y]) & B[(x + 2) % 5 + 5 * y]);
#endif
    /* iota */
    A[0] ^= g_rc[ir];
  }
}

/* byte-level view of the state: byte i of the 200-byte string S */
static void xor_byte(uint64_t A[25], size_t i, uint8_t b) {
  A[i / 8] ^= (uint64_t)b << (8 * (i % 8));
}
static uint8_t get_byte(const uint64_t A[25], size_t i) {
  return (uint8_t)(A[i / 8] >> (8 * (i % 8)));
}

static void shake(size_t rate, const uint8_t *in, size_t inlen, uint8_t *out, size_t outlen) {
  uint64_t A[25];
  memset(A, 0, sizeof A);
  size_t pos = 0;
  for (size_t i = 0; i < inlen; i++) {
    xor_byte(A, pos++, in[i]);
    if (pos == rate) { dil_ref_keccak_f1600(A); pos = 0; }
  }
  /* SHAKE domain bits 1111 then the first pad bit: 0x1F; the final pad bit: 0x80 */
  xor_byte(A, pos, 0x1F);
  xor_byte(A, rate - 1, 0x80);
  dil_ref_keccak_f1600(A);
  pos = 0;
  for (size_t i = 0; i < outlen; i++) {
    if (pos == rate) { dil_ref_keccak_f1600(A); pos = 0; }
    out[i] = get_byte(A, pos++);
  }
}

void dil_ref_shake128(const uint8_t *in, size_t inlen, uint8_t *out, size_t outlen) {
  shake(168, in, inlen, out, outlen);
}
void dil_ref_shake256(const uint8_t *in, size_t inlen, uint8_t *out, size_t outlen) {
  shake(136, in, inlen, out, outlen);
}
