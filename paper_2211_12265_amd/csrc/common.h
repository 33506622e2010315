// Shared definitions for the gfx950 Dilithium kernels: parameter sets (Tab. 1),
// Montgomery constants derived at compile time, and small device helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dil {

constexpr int32_t Q = 8380417;
constexpr int N = 256;
constexpr int D = 13;

// ---- compile-time modular helpers (used only to derive constants) ----
constexpr int64_t cmod(int64_t x, int64_t m) { return ((x % m) + m) % m; }
constexpr int64_t cpow(int64_t b, int64_t e, int64_t m) {
  int64_t r = 1;
  b = cmod(b, m);
  while (e > 0) {
    if (e & 1) r = (r * b) % m;
    b = (b * b) % m;
    e >>= 1;
  }
  return r;
}
// q^-1 mod 2^32 by Newton iteration on the 2-adic inverse
constexpr uint32_t qinv32() {
  uint32_t x = 1;
  for (int i = 0; i < 6; i++) x = x * (2u - (uint32_t)Q * x);
  return x;
}
constexpr int32_t QINV = (int32_t)qinv32();
static_assert((uint32_t)Q * (uint32_t)QINV == 1u, "q * qinv != 1 mod 2^32");
constexpr int64_t R_MOD_Q = cmod((int64_t)1 << 32, Q);            // 2^32 mod q
constexpr int32_t to_mont(int64_t c) { return (int32_t)cmod(cmod(c, Q) * R_MOD_Q, Q); }
constexpr int64_t PSI = 1753;                                       // primitive 512-th root of unity mod q
constexpr int brv8(int k) {
  int r = 0;
  for (int i = 0; i < 8; i++)
    if (k & (1 << i)) r |= 1 << (7 - i);
  return r;
}
// forward twiddle for butterfly block k (1..255): psi^brv8(k), Montgomery form
constexpr int32_t zeta_m(int k) { return to_mont(cpow(PSI, brv8(k), Q)); }
// inverse twiddle for block k: psi^-brv8(k), Montgomery form
constexpr int32_t zinv_m(int k) { return to_mont(cpow(PSI, 512 - brv8(k), Q)); }
// INTT output scale: inputs carry the 2^-32 of one Montgomery product, so the last
// layer multiplies by 2^32 / 256 (i.e. Montgomery form of 2^64 / 256).
constexpr int64_t INV256 = cpow(256, Q - 2, Q);
constexpr int64_t SCALE_PLAIN = cmod(R_MOD_Q * INV256, Q);          // 2^32/256 mod q
constexpr int32_t SCALE_M = to_mont(SCALE_PLAIN);
constexpr int32_t zinv_scaled_m(int k) { return to_mont(cmod(cpow(PSI, 512 - brv8(k), Q) * SCALE_PLAIN, Q)); }

// ---- level parameters (Tab. 1) ----
template <int LV> struct Lv;
// MLDSA: the FIPS 204 form (not in the paper); CT: bytes of ctilde
template <> struct Lv<2> {
  static constexpr int K = 4, L = 4, ETA = 2, TAU = 39, BETA = 78, OMEGA = 80;
  static constexpr int32_t GAMMA1 = 1 << 17, GAMMA2 = (Q - 1) / 88;
  static constexpr bool MLDSA = false;
  static constexpr int CT = 32;
};
template <> struct Lv<3> {
  static constexpr int K = 6, L = 5, ETA = 4, TAU = 49, BETA = 196, OMEGA = 55;
  static constexpr int32_t GAMMA1 = 1 << 19, GAMMA2 = (Q - 1) / 32;
  static constexpr bool MLDSA = false;
  static constexpr int CT = 32;
};
template <> struct Lv<5> {
  static constexpr int K = 8, L = 7, ETA = 2, TAU = 60, BETA = 120, OMEGA = 75;
  static constexpr int32_t GAMMA1 = 1 << 19, GAMMA2 = (Q - 1) / 32;
  static constexpr bool MLDSA = false;
  static constexpr int CT = 32;
};
// ML-DSA-44 / 65 / 87 (FIPS 204): the lattice parameters of levels 2 / 3 / 5,
// a 64-byte tr and a ctilde of lambda / 4 bytes; the key seed, mu and the mask
// seed rho'' hash other inputs (see the KeyGen and Sign setup kernels)
template <> struct Lv<44> : Lv<2> {
  static constexpr bool MLDSA = true;
  static constexpr int CT = 32;
};
template <> struct Lv<65> : Lv<3> {
  static constexpr bool MLDSA = true;
  static constexpr int CT = 48;
};
template <> struct Lv<87> : Lv<5> {
  static constexpr bool MLDSA = true;
  static constexpr int CT = 64;
};
// derived sizes (encodings follow the round-3 v3.1 byte layout)
template <int LV> struct P : Lv<LV> {
  using B = Lv<LV>;
  static constexpr int ZBITS = B::GAMMA1 == (1 << 17) ? 18 : 20;
  static constexpr int W1BITS = (Q - 1) / (2 * B::GAMMA2) == 44 ? 6 : 4;
  static constexpr int EBITS = B::ETA == 2 ? 3 : 4;
  static constexpr int M_HB = (Q - 1) / (2 * B::GAMMA2);            // number of HighBits values
  static constexpr int ZB = N * ZBITS / 8;                           // packed z poly
  static constexpr int W1B = N * W1BITS / 8;                         // packed w1 poly
  static constexpr int EB = N * EBITS / 8;                           // packed eta poly
  static constexpr int T1B = 320, T0B = 416;
  static constexpr int TRB = B::MLDSA ? 64 : 32;                     // tr bytes
  static constexpr int CT = B::CT;                                   // ctilde bytes
  static constexpr int PK = 32 + B::K * T1B;
  static constexpr int OFF_S1 = 64 + TRB;                            // sk = rho || K || tr || s1 || s2 || t0
  static constexpr int OFF_S2 = OFF_S1 + B::L * EB, OFF_T0 = OFF_S1 + (B::L + B::K) * EB;
  static constexpr int SK = OFF_T0 + B::K * T0B;
  static constexpr int SIG = CT + B::L * ZB + B::OMEGA + B::K;       // sig = ctilde || z || h
  static constexpr int OFF_Z = CT, OFF_H = CT + B::L * ZB;
  static constexpr int MUW1 = 64 + B::K * W1B;                       // mu || packed w1
};
static_assert(P<2>::PK == 1312 && P<2>::SK == 2528 && P<2>::SIG == 2420, "L2 sizes");
static_assert(P<3>::PK == 1952 && P<3>::SK == 4000 && P<3>::SIG == 3293, "L3 sizes");
static_assert(P<5>::PK == 2592 && P<5>::SK == 4864 && P<5>::SIG == 4595, "L5 sizes");
static_assert(P<44>::PK == 1312 && P<44>::SK == 2560 && P<44>::SIG == 2420, "ML-DSA-44 sizes");
static_assert(P<65>::PK == 1952 && P<65>::SK == 4032 && P<65>::SIG == 3309, "ML-DSA-65 sizes");
static_assert(P<87>::PK == 2592 && P<87>::SK == 4896 && P<87>::SIG == 4627, "ML-DSA-87 sizes");

// ---- device arithmetic ----
// Montgomery reduction of a 64-bit value: returns a * 2^-32 mod q in (-q, q),
// valid for |a| < 2^31 q.  Three VALU ops on gfx950: the product/accumulate
// (v_mad_i64_i32), the low multiply by q^-1 and one more v_mad_i64_i32.
__device__ __forceinline__ int32_t mont_reduce(int64_t a) {
  int32_t t = (int32_t)a * QINV;
  return (int32_t)((a - (int64_t)t * Q) >> 32);
}
__device__ __forceinline__ int32_t mont_mul(int32_t a, int32_t b) { return mont_reduce((int64_t)a * b); }
// canonical representative in [0, q) of x in (-q, q)
__device__ __forceinline__ int32_t canon(int32_t x) { return x + ((x >> 31) & Q); }
}  // namespace dil
