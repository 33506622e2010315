/*
 * Plain CPU oracle for batched CRYSTALS-Dilithium (round-3 parameter sets 2/3/5)
 * and its FIPS 204 form ML-DSA-44/65/87 (levels 44/65/87).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * definition that the GPU path is checked against.  Only the test suite, the
 * package's smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never calls it and shares no code, header, table or constant
 * with it.
 *
 * Arithmetic is plain int64 with '%' followed by explicit canonicalisation:
 * no Montgomery, no Barrett, no vector instructions.  Keccak round constants
 * and rotation offsets are derived at start-up from their FIPS 202
 * definitions (the rc LFSR and the triangular-number rule), not typed in.
 *
 * Citations name the paper's sections, algorithms and tables
 * ("Alg. 2" = Dilithium.Sign, "Tab. 1" = parameter sets, "Sec. 2.3" =
 * Preliminaries / Dilithium, "Sec. 2.2" = ring arithmetic and the NTT).
 * Where the paper is silent the oracle follows the public round-3 (v3.1)
 * Dilithium specification's byte conventions; each such reading is marked
 * [R] and listed in the design notes.
 *
 * Parity pins (tests under tests/test_oracle_*.py):
 *   SHAKE128/256            exact vs Python hashlib (FIPS 202)
 *   NTT / INTT              fast == O(n^2) definition; INTT(NTT(x)) == x;
 *                           INTT(NTT f o NTT g) == schoolbook negacyclic product
 *   Power2Round, Decompose  exhaustive identities over all of [0, q)
 *   MakeHint / UseHint      hint-correctness property over all r
 *   encodings               pack o unpack == identity, sizes
 *   samplers                ExpandA acceptance q / 2^23 (the 23-bit mask),
 *                           ExpandS acceptance 15/16 and 9/16 and uniform
 *                           coefficients, SampleInBall's uniform support
 *                           (the b <= i draw), ranges and weights
 *   scheme                  Verify(Sign) == 1, all single-bit flips rejected,
 *                           mean Sign loop count vs Sec. 2.3, and on crafted
 *                           secret keys every emitted signature keeps
 *                           ||c t0|| < gamma2 and at most omega hints
 * ML-DSA (levels 44/65/87) follows FIPS 204, which is neither in the paper nor
 * available here: its readings are those of section "ML-DSA" in scheme.c, pinned
 * by hashlib recomputation of the seed expansion, tr, mu and rho'' and by the
 * scheme properties; parity unpinned against the FIPS 204 known-answer tests.
 * parity unpinned: the exact byte streams of ExpandA / ExpandS / ExpandMask /
 *   SampleInBall and the encodings against the official round-3 known-answer
 *   tests (neither the specification nor its KAT files are available): the
 *   byte and nibble order inside the sampler streams, the nonce encodings,
 *   ExpandMask's orientation gamma1 - v, SampleInBall's sign-bit source and
 *   the key / signature byte layouts are readings [R].
 */
#ifndef DIL_ORACLE_H
#define DIL_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#define ORQ 8380417
#define ORN 256

typedef struct {
  int level, k, l, eta, tau, beta, omega;
  int32_t gamma1, gamma2;
  int z_bits, w1_bits, eta_bits;
  size_t pk_bytes, sk_bytes, sig_bytes, w1_poly_bytes;
  int mldsa;     /* 0: round-3 Dilithium (levels 2/3/5); 1: FIPS 204 ML-DSA (44/65/87) */
  int tr_bytes;  /* 32 (round 3) or 64 (ML-DSA) */
  int ct_bytes;  /* ctilde: 32 (round 3); lambda / 4 = 32 / 48 / 64 (ML-DSA) */
} ref_params;

/* parameter set for level 2/3/5 (Tab. 1), or 44/65/87 for ML-DSA-44/65/87 (the
   same k, l, eta, tau, gamma1, gamma2, beta, omega as levels 2/3/5; the FIPS 204
   differences are tr_bytes, ct_bytes and the hash inputs of the scheme functions);
   returns 0 on success, -1 otherwise */
int dil_ref_params(int level, ref_params *p);
/* ML-DSA's message representative mu = H(tr || 0 || 0 || M, 64): the pure
   signing interface with an empty context string (FIPS 204, not in the paper) */
void dil_ref_mldsa_mu(const uint8_t tr[64], const uint8_t *msg, size_t mlen, uint8_t mu[64]);

/* Keccak / SHAKE (Sec. 2.3 "Sampling": SHAKE128/256 as XOF, SHAKE256 as H) */
void dil_ref_keccak_f1600(uint64_t st[25]);
void dil_ref_shake128(const uint8_t *in, size_t inlen, uint8_t *out, size_t outlen);
void dil_ref_shake256(const uint8_t *in, size_t inlen, uint8_t *out, size_t outlen);

/* ring arithmetic (Sec. 2.2) on canonical coefficients in [0, q) */
void dil_ref_ntt(int32_t a[ORN]);
void dil_ref_intt(int32_t a[ORN]);
void dil_ref_ntt_definition(const int32_t a[ORN], int32_t out[ORN]);
void dil_ref_poly_mul_schoolbook(const int32_t a[ORN], const int32_t b[ORN], int32_t out[ORN]);
/* c_i = INTT(NTT(a_i) o b_i), b_i read as NTT-domain values; count polys, nthreads workers */
void dil_ref_ntt_mul_batch(const int32_t *a, const int32_t *b, int32_t *c, size_t count, int nthreads);

/* rounding and hints (Sec. 2.3 "Bits Extraction and Hints"), elementwise over n values */
void dil_ref_power2round(const int32_t *r, int32_t *r1, int32_t *r0, size_t n);
void dil_ref_decompose(const int32_t *r, int32_t *r1, int32_t *r0, size_t n, int32_t gamma2);
void dil_ref_make_hint(const int32_t *z, const int32_t *r, int32_t *h, size_t n, int32_t gamma2);
void dil_ref_use_hint(const int32_t *h, const int32_t *r, int32_t *out, size_t n, int32_t gamma2);

/* samplers (Sec. 2.3 "Sampling", Alg. 1-2); outputs canonical in [0, q) except where noted */
void dil_ref_expand_a(int level, const uint8_t rho[32], int32_t *A /* k*l*256 */);
void dil_ref_expand_a_poly(const uint8_t seed34[34], int32_t out[ORN]);
void dil_ref_expand_a_polys(const uint8_t *seeds34, int32_t *out, size_t count, int nthreads);
void dil_ref_expand_s(int level, const uint8_t rhop[64], int32_t *s /* (l+k)*256, centred */);
/* one ExpandA / ExpandS polynomial, returning how much of its stream the rejection
   sampler examined: 3-byte candidates (ExpandA) or nibbles (ExpandS); pins the
   acceptance rates q / 2^23, 15/16 (eta = 2) and 9/16 (eta = 4) */
size_t dil_ref_expand_a_poly_counted(const uint8_t seed34[34], int32_t out[ORN]);
size_t dil_ref_expand_s_poly_counted(int eta, const uint8_t rhop[64], uint16_t nonce, int32_t out[ORN] /* centred */);
void dil_ref_expand_mask(int level, const uint8_t rhop[64], uint32_t kappa, int32_t *y /* l*256, centred */);
/* ctilde: 32 bytes (round 3) or the ct_bytes of the ML-DSA level */
void dil_ref_sample_in_ball(int level, const uint8_t *ctilde, int32_t c[ORN] /* centred */);

/* generic b-bit LSB-first packing of n coefficients (values must lie in [0, 2^b)) */
void dil_ref_bitpack(const uint32_t *v, size_t n, int b, uint8_t *out);
void dil_ref_bitunpack(const uint8_t *in, size_t n, int b, uint32_t *v);

/* scheme (Alg. 1-3), single task */
int dil_ref_keygen(int level, const uint8_t zeta[32], uint8_t *pk, uint8_t *sk);
/* returns the number of loop iterations used (>= 1), -1 on bad level, or -2 (all-zero
   signature) when the loop reaches the iteration cap (default 100000, see set_sign_cap) */
void dil_ref_set_sign_cap(int cap);
int dil_ref_sign(int level, const uint8_t *sk, const uint8_t *msg, size_t mlen, uint8_t *sig);
/* the randomized variant of round-3 Sign: rho' is the 64 caller-supplied bytes rnd
   instead of H(K || mu); at the ML-DSA levels rnd is the 32-byte hedging input of
   rho'' = H(K || rnd || mu) (dil_ref_sign uses 32 zero bytes); same return values */
int dil_ref_sign_rnd(int level, const uint8_t *sk, const uint8_t *msg, size_t mlen, const uint8_t *rnd,
                     uint8_t *sig);
/* returns 1 accept, 0 reject, -1 bad level */
int dil_ref_verify(int level, const uint8_t *pk, const uint8_t *msg, size_t mlen, const uint8_t *sig);
/* ML-DSA's internal signing / verification (levels 44 / 65 / 87 only, -1
   otherwise): the caller passes the formatted message M' and mu = H(tr || M',
   64); M' = 0x00 || |ctx| || ctx || M is the pure form with context ctx (the
   functions above use ctx empty), M' = 0x01 || |ctx| || ctx || OID || PH(M)
   the pre-hash form.  rnd: 32 bytes or NULL (zeros). */
int dil_ref_mldsa_sign_internal(int level, const uint8_t *sk, const uint8_t *mprime, size_t len, const uint8_t *rnd,
                                uint8_t *sig);
int dil_ref_mldsa_verify_internal(int level, const uint8_t *pk, const uint8_t *mprime, size_t len,
                                  const uint8_t *sig);

/* batched drivers: same argument conventions as the GPU C-ABI but host pointers, no stream.
   key_idx may be NULL (task i uses key i).  msg_off has count+1 entries (CSR).
   iters (optional) receives the Sign loop count per task.  Return 0, or -1 on bad input. */
int dil_ref_keygen_batch(int level, const uint8_t *seeds, uint8_t *pk, uint8_t *sk, uint32_t count, int nthreads);
int dil_ref_sign_batch(int level, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                       const uint64_t *msg_off, uint8_t *sig, uint32_t count, int nthreads, int32_t *iters);
/* as dil_ref_sign_batch, task t signing with rho' = rnd[64 t .. 64 t + 64) (rnd NULL: deterministic);
   at the ML-DSA levels rnd rows are 32 bytes (rnd[32 t .. 32 t + 32)) */
int dil_ref_sign_batch_rnd(int level, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                           const uint64_t *msg_off, const uint8_t *rnd, uint8_t *sig, uint32_t count, int nthreads,
                           int32_t *iters);
/* the batch drivers with internal = 1: messages are formatted messages M'
   (ML-DSA levels only; -1 otherwise) */
int dil_ref_sign_batch_ex(int level, int internal, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                          const uint64_t *msg_off, const uint8_t *rnd, uint8_t *sig, uint32_t count, int nthreads,
                          int32_t *iters);
int dil_ref_verify_batch_ex(int level, int internal, const uint8_t *pk, const uint32_t *key_idx, const uint8_t *msg,
                            const uint64_t *msg_off, const uint8_t *sig, int32_t *verdict, uint32_t count,
                            int nthreads);
int dil_ref_verify_batch(int level, const uint8_t *pk, const uint32_t *key_idx, const uint8_t *msg,
                         const uint64_t *msg_off, const uint8_t *sig, int32_t *verdict, uint32_t count,
                         int nthreads);
#endif
