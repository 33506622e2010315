"""Oracle ML-DSA-44 / 65 / 87 (FIPS 204 form of the scheme of Sec. 2, levels 44 / 65 / 87).

FIPS 204 is neither in the paper nor available here, and there are no known-answer files: parity
against the standard stays unpinned.  What is pinned, independently of the oracle's scheme code:
  * the object sizes of the three parameter sets;
  * every hash input that differs from round 3, recomputed with hashlib: the KeyGen seed
    expansion H(xi || k || l, 128), tr = H(pk, 64), mu = H(tr || 0 || 0 || M, 64),
    rho'' = H(K || rnd || mu, 64) and ctilde = H(mu || w1Encode(w1), lambda / 4);
  * the key and signature layouts, by recomputing t = A s1 + s2, y = z - c s1, w = A y and the
    hint from the primitives (schoolbook products, Power2Round, Decompose, MakeHint, ExpandA,
    ExpandS, ExpandMask: each pinned on its own for round 3);
  * SampleInBall seeded by the whole ctilde (tau entries of +-1; every byte of ctilde matters);
  * the scheme properties: Verify(Sign) accepts, bit flips and the other variant reject, the
    deterministic signer is the hedged one with rnd = 0;
  * internal signing on a formatted message M' (mu = H(tr || M')): with M' = 0 || |ctx| || ctx
    || M it is pure signing with context ctx (recomputed with hashlib for a non-empty ctx), the
    empty context gives the pure signatures, and another context rejects."""
import hashlib

import numpy as np
import pytest

from paper_2211_12265_amd import workload

Q = 8380417
N = 256
D = 13
LEVELS = [44, 65, 87]
# (pk, sk, sig) bytes of ML-DSA-44 / 65 / 87
SIZES = {44: (1312, 2560, 2420), 65: (1952, 4032, 3309), 87: (2592, 4896, 4627)}
LAMBDA = {44: 128, 65: 192, 87: 256}
BASE = {44: 2, 65: 3, 87: 5}


def _h(data: bytes, n: int) -> bytes:
    return hashlib.shake_256(data).digest(n)


def _mul(a: np.ndarray, b: np.ndarray, orc) -> np.ndarray:
    """product in Z_q[X]/(X^256 + 1), coefficients in [0, q)"""
    return np.mod(orc.poly_mul_schoolbook(np.mod(a, Q), np.mod(b, Q)).astype(np.int64), Q)


def _centred(a: np.ndarray) -> np.ndarray:
    a = np.mod(a.astype(np.int64), Q)
    return np.where(a > Q // 2, a - Q, a)


def _matrix(orc, level: int, rho: bytes) -> np.ndarray:
    """A in the coefficient domain (ExpandA samples the NTT domain directly, Sec. 2.3)"""
    ah = orc.expand_a(level, rho)
    return np.stack([np.stack([orc.intt(ah[i, j]) for j in range(ah.shape[1])]) for i in range(ah.shape[0])]).astype(np.int64)


def _decode_hint(p: dict, data: np.ndarray) -> np.ndarray:
    """omega position bytes, then k running counts (strict decoding is pinned for round 3)"""
    k, om = p["k"], p["omega"]
    h = np.zeros((k, N), np.int64)
    start = 0
    for i in range(k):
        end = int(data[om + i])
        for j in range(start, end):
            h[i, int(data[j])] = 1
        start = end
    return h


@pytest.mark.parametrize("level", LEVELS)
def test_parameter_sets(orc, level):
    p, b = orc.params(level), orc.params(BASE[level])
    assert p["mldsa"] == 1 and b["mldsa"] == 0
    for f in ("k", "l", "eta", "tau", "beta", "omega", "gamma1", "gamma2", "z_bits", "w1_bits", "pk_bytes"):
        assert p[f] == b[f], f
    assert (p["pk_bytes"], p["sk_bytes"], p["sig_bytes"]) == SIZES[level]
    assert p["tr_bytes"] == 64 and p["ct_bytes"] == LAMBDA[level] // 4
    with pytest.raises(ValueError):
        orc.params(45)


@pytest.mark.parametrize("level", LEVELS)
def test_keygen_recomputed(orc, level):
    p = orc.params(level)
    k, l, eta = p["k"], p["l"], p["eta"]
    xi = workload.random_bytes("test/mldsa-xi", level, (32,)).tobytes()
    pk, sk = orc.keygen(level, xi)
    seed = _h(xi + bytes([k, l]), 128)
    rho, rhop, K = seed[:32], seed[32:96], seed[96:]
    assert pk[:32] == rho and sk[:32] == rho and sk[32:64] == K
    assert sk[64:128] == _h(pk, 64)
    # s1, s2 from ExpandS(rho'), t = A s1 + s2, (t1, t0) = Power2Round(t)
    s = orc.expand_s(level, rhop).astype(np.int64)
    A = _matrix(orc, level, rho)
    eb = N * p["eta_bits"] // 8
    off = 128
    for j in range(l + k):
        v = orc.bitunpack(sk[off + j * eb: off + (j + 1) * eb], N, p["eta_bits"]).astype(np.int64)
        assert np.array_equal(eta - v, s[j]), j
    off += (l + k) * eb
    for i in range(k):
        t = s[l + i].copy()
        for j in range(l):
            t = t + _mul(A[i, j], s[j], orc)
        t = np.mod(t, Q)
        t1 = (t + (1 << (D - 1)) - 1) >> D
        t0 = t - (t1 << D)
        assert pk[32 + 320 * i: 32 + 320 * (i + 1)] == orc.bitpack(t1, 10)
        assert sk[off + 416 * i: off + 416 * (i + 1)] == orc.bitpack((1 << (D - 1)) - t0, 13)
    assert off + 416 * k == len(sk)


@pytest.mark.parametrize("level", LEVELS)
@pytest.mark.parametrize("hedged,ctx", [(False, b""), (True, b""), (False, b"context string"), (True, b"\x01" * 255)])
def test_sign_recomputed(orc, level, hedged, ctx):
    """Every ML-DSA-specific step of Sign recomputed from the signature it emits (a non-empty
    context through internal signing of the formatted message)."""
    p = orc.params(level)
    k, l, ct = p["k"], p["l"], p["ct_bytes"]
    xi = workload.random_bytes("test/mldsa-xi", 100 + level, (32,)).tobytes()
    pk, sk = orc.keygen(level, xi)
    msg = workload.random_bytes("test/mldsa-m", level, (77,)).tobytes()
    rnd = workload.random_bytes("test/mldsa-rnd", level, (32,)).tobytes() if hedged else bytes(32)
    mprime = bytes([0, len(ctx)]) + ctx + msg
    sm = mprime if ctx else msg
    sig, iters = orc.sign_batch(level, np.frombuffer(sk, np.uint8)[None], np.frombuffer(sm, np.uint8),
                                np.array([0, len(sm)], np.uint64),
                                rnd=np.frombuffer(rnd, np.uint8)[None] if hedged else None, internal=bool(ctx))
    sig, it = sig[0].tobytes(), int(iters[0])
    assert len(sig) == p["sig_bytes"] and it >= 1
    tr, K = sk[64:128], sk[32:64]
    mu = _h(tr + mprime, 64)
    if not ctx:
        assert orc.mldsa_mu(tr, msg) == mu
    rhopp = _h(K + rnd + mu, 64)
    ctilde = sig[:ct]
    c = orc.sample_in_ball(level, ctilde).astype(np.int64)
    zb = N * p["z_bits"] // 8
    z = np.stack([p["gamma1"] - orc.bitunpack(sig[ct + j * zb: ct + (j + 1) * zb], N, p["z_bits"]).astype(np.int64)
                  for j in range(l)])
    assert np.abs(z).max() < p["gamma1"] - p["beta"]
    eb = N * p["eta_bits"] // 8
    s = np.stack([p["eta"] - orc.bitunpack(sk[128 + j * eb: 128 + (j + 1) * eb], N, p["eta_bits"]).astype(np.int64)
                  for j in range(l + k)])
    # y = z - c s1 is ExpandMask(rho'', kappa) with kappa = l * (iterations - 1)
    y = np.stack([_centred(z[j] - _mul(c, s[j], orc)) for j in range(l)])
    assert np.array_equal(y, orc.expand_mask(level, rhopp, l * (it - 1)))
    # ctilde = H(mu || w1Encode(HighBits(A y)), lambda / 4)
    A = _matrix(orc, level, pk[:32])
    w = np.stack([np.mod(sum(_mul(A[i, j], y[j], orc) for j in range(l)), Q) for i in range(k)])
    w1, _ = orc.decompose(w.reshape(-1).astype(np.int32), p["gamma2"])
    w1 = w1.reshape(k, N)
    assert _h(mu + b"".join(orc.bitpack(w1[i], p["w1_bits"]) for i in range(k)), ct) == ctilde
    # h = MakeHint(-c t0, w - c s2 + c t0)
    off = 128 + (l + k) * eb
    t0 = np.stack([(1 << (D - 1)) - orc.bitunpack(sk[off + 416 * i: off + 416 * (i + 1)], N, 13).astype(np.int64)
                   for i in range(k)])
    ct0 = np.stack([_mul(c, t0[i], orc) for i in range(k)])
    cs2 = np.stack([_mul(c, s[l + i], orc) for i in range(k)])
    r = np.mod(w - cs2 + ct0, Q)
    hint = orc.make_hint(np.mod(-ct0, Q).reshape(-1).astype(np.int32), r.reshape(-1).astype(np.int32), p["gamma2"])
    assert np.array_equal(_decode_hint(p, np.frombuffer(sig[ct + l * zb:], np.uint8)), hint.reshape(k, N))
    assert orc.mldsa_verify_internal(level, pk, mprime, sig) == 1
    assert orc.verify(level, pk, msg, sig) == (0 if ctx else 1)


@pytest.mark.parametrize("level", LEVELS)
def test_sample_in_ball_whole_ctilde(orc, level):
    p = orc.params(level)
    ct = p["ct_bytes"]
    base = workload.random_bytes("test/mldsa-ct", level, (ct,)).tobytes()
    c = orc.sample_in_ball(level, base)
    assert np.count_nonzero(c) == p["tau"] and set(np.unique(c)) <= {-1, 0, 1}
    # SampleInBall absorbs ctilde whole: the ball of SHAKE256(ctilde), not of a prefix
    if ct == 32:
        assert np.array_equal(c, orc.sample_in_ball(BASE[level], base))
    for pos in (0, ct // 2, ct - 1):
        other = bytearray(base)
        other[pos] ^= 1
        assert not np.array_equal(c, orc.sample_in_ball(level, bytes(other))), pos


@pytest.mark.parametrize("level", LEVELS)
def test_round_trip_and_rejections(orc, level):
    p = orc.params(level)
    n = 8
    pk, sk = orc.keygen_batch(level, workload.keygen_seeds(n, seed=level))
    msg, off = workload.messages(workload.uniform_lengths(n, 0, 200, seed=level), seed=level)
    sig, iters = orc.sign_batch(level, sk, msg, off)
    assert orc.verify_batch(level, pk, msg, off, sig).tolist() == [1] * n
    # deterministic Sign is the hedged one with rnd = 0; a nonzero rnd gives another valid signature
    sig0, it0 = orc.sign_batch(level, sk, msg, off, rnd=np.zeros((n, 32), np.uint8))
    assert np.array_equal(sig, sig0) and np.array_equal(iters, it0)
    rnd = workload.random_bytes("test/mldsa-rnd", level, (n, 32))
    sig_r, _ = orc.sign_batch(level, sk, msg, off, rnd=rnd)
    assert not np.array_equal(sig_r, sig)
    assert orc.verify_batch(level, pk, msg, off, sig_r).tolist() == [1] * n
    with pytest.raises(ValueError):
        orc.sign_batch(level, sk, msg, off, rnd=np.zeros((n, 64), np.uint8))
    # sampled single-bit flips of signature 0
    nbits = p["sig_bytes"] * 8
    bits = np.unique(np.concatenate([np.arange(0, nbits, 11), np.arange(nbits - 8 * (p["omega"] + p["k"]), nbits)]))
    flipped = np.repeat(sig[:1], bits.size, axis=0)
    flipped[np.arange(bits.size), bits // 8] ^= (1 << (bits % 8)).astype(np.uint8)
    m0 = msg[int(off[0]):int(off[1])]
    v = orc.verify_batch(level, pk, np.tile(m0, bits.size), np.arange(bits.size + 1, dtype=np.uint64) * m0.size,
                         flipped, key_idx=np.zeros(bits.size, np.uint32))
    assert v.sum() == 0
    # the same bytes do not verify as a round-3 signature (level 44 shares every size with level 2)
    if level == 44:
        assert orc.verify_batch(2, pk, msg, off, sig).sum() == 0
        pk2, sk2 = orc.keygen_batch(2, workload.keygen_seeds(n, seed=level))
        assert not np.array_equal(pk2, pk)
        sig2, _ = orc.sign_batch(2, sk2, msg, off)
        assert orc.verify_batch(44, pk2, msg, off, sig2).sum() == 0


@pytest.mark.parametrize("level", LEVELS)
def test_internal_mode_batches(orc, level):
    """Batch drivers on formatted messages: the empty context reproduces pure signing and
    verification, a context binds the signature to it, and round-3 levels have no internal mode."""
    n = 6
    pk, sk = orc.keygen_batch(level, workload.keygen_seeds(n, seed=500 + level))
    lens = workload.uniform_lengths(n, 0, 150, seed=level)
    msg, off = workload.messages(lens, seed=level)
    msgs = [msg[int(off[i]):int(off[i + 1])].tobytes() for i in range(n)]

    def csr(parts):
        buf = np.frombuffer(b"".join(parts), np.uint8) if sum(map(len, parts)) else np.zeros(0, np.uint8)
        return buf, np.concatenate([[0], np.cumsum([len(x) for x in parts])]).astype(np.uint64)

    pure, _ = orc.sign_batch(level, sk, msg, off)
    fm, foff = csr([orc.mldsa_format(m) for m in msgs])
    assert np.array_equal(orc.sign_batch(level, sk, fm, foff, internal=True)[0], pure)
    assert orc.verify_batch(level, pk, fm, foff, pure, internal=True).tolist() == [1] * n
    cm, coff = csr([orc.mldsa_format(m, b"app-%d" % i) for i, m in enumerate(msgs)])
    csig, _ = orc.sign_batch(level, sk, cm, coff, internal=True)
    assert orc.verify_batch(level, pk, cm, coff, csig, internal=True).tolist() == [1] * n
    assert orc.verify_batch(level, pk, msg, off, csig).tolist() == [0] * n          # context dropped
    assert orc.verify_batch(level, pk, fm, foff, csig, internal=True).tolist() == [0] * n
    with pytest.raises(ValueError):
        orc.sign_batch(BASE[level], sk[:, :orc.params(BASE[level])["sk_bytes"]], msg, off, internal=True)
