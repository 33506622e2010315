"""The randomized variant of round-3 Sign in the oracle: rho' comes from the caller instead of
H(K || mu) (Alg. 2 computes it deterministically; the randomized variant keeps every other
step).  Pins that do not use the oracle's own hash: with rho' computed here by hashlib as
SHAKE256(K || SHAKE256(tr || M)), the randomized path must reproduce the deterministic
signature byte for byte; random rho' values give signatures that verify, differ from the
deterministic ones and are reproducible for the same rho'."""
import hashlib

import numpy as np
import pytest

from paper_2211_12265_amd import workload


def _setup(orc, level, n, seed):
    pk, sk = orc.keygen_batch(level, workload.keygen_seeds(n, seed=seed))
    lens = workload.uniform_lengths(n, 0, 400, seed=seed)
    msg, off = workload.messages(lens, seed=seed)
    return pk, sk, msg, off


def _rhop_det(sk_row: bytes, m: bytes) -> bytes:
    tr, K = sk_row[64:96], sk_row[32:64]
    mu = hashlib.shake_256(tr + m).digest(64)
    return hashlib.shake_256(K + mu).digest(64)


@pytest.mark.parametrize("level", [2, 3, 5])
def test_rnd_equal_to_deterministic_rhop_reproduces_signature(orc, level):
    n = 12
    pk, sk, msg, off = _setup(orc, level, n, seed=40 + level)
    rnd = np.stack([np.frombuffer(_rhop_det(sk[i].tobytes(), msg[int(off[i]):int(off[i + 1])].tobytes()), np.uint8)
                    for i in range(n)])
    det, it_det = orc.sign_batch(level, sk, msg, off)
    ran, it_ran = orc.sign_batch(level, sk, msg, off, rnd=rnd)
    assert np.array_equal(det, ran) and np.array_equal(it_det, it_ran)


@pytest.mark.parametrize("level", [2, 3, 5])
def test_random_rhop_signatures_verify_and_differ(orc, level):
    n = 16
    pk, sk, msg, off = _setup(orc, level, n, seed=50 + level)
    rnd1 = workload.random_bytes("dil/rnd", 1, (n, 64))
    rnd2 = workload.random_bytes("dil/rnd", 2, (n, 64))
    det, _ = orc.sign_batch(level, sk, msg, off)
    s1, _ = orc.sign_batch(level, sk, msg, off, rnd=rnd1)
    s1b, _ = orc.sign_batch(level, sk, msg, off, rnd=rnd1)
    s2, _ = orc.sign_batch(level, sk, msg, off, rnd=rnd2)
    assert np.array_equal(s1, s1b)
    assert orc.verify_batch(level, pk, msg, off, s1).tolist() == [1] * n
    assert orc.verify_batch(level, pk, msg, off, s2).tolist() == [1] * n
    assert all(not np.array_equal(s1[i], det[i]) and not np.array_equal(s1[i], s2[i]) for i in range(n))


def test_rnd_shape_checked(orc):
    pk, sk, msg, off = _setup(orc, 2, 3, seed=60)
    with pytest.raises(ValueError):
        orc.sign_batch(2, sk, msg, off, rnd=np.zeros((2, 64), np.uint8))
