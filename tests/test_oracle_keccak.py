"""Oracle Keccak-f[1600] / SHAKE pinned exactly against Python hashlib (FIPS 202)."""
import hashlib

import numpy as np
import pytest

from paper_2211_12265_amd import workload


LENGTHS = sorted(set(list(range(0, 210)) + [271, 272, 273, 335, 336, 337, 407, 408, 409, 503, 504, 505, 999, 1000]))


@pytest.mark.parametrize("which", ["128", "256"])
def test_shake_matches_hashlib(orc, which):
    data = workload.random_bytes("test/shake", 0, (1000,)).tobytes()
    for n in LENGTHS:
        m = data[:n]
        for outlen in (1, 32, 135, 136, 137, 167, 168, 169, 700):
            if which == "128":
                assert orc.shake128(m, outlen) == hashlib.shake_128(m).digest(outlen), (n, outlen)
            else:
                assert orc.shake256(m, outlen) == hashlib.shake_256(m).digest(outlen), (n, outlen)


def test_shake_long_output(orc):
    m = b"dilithium"
    assert orc.shake128(m, 5000) == hashlib.shake_128(m).digest(5000)
    assert orc.shake256(m, 5000) == hashlib.shake_256(m).digest(5000)


def test_permutation_via_one_block(orc):
    # SHAKE256 of the empty string is one permutation of the padded zero state;
    # reproduce it with the exported permutation and the FIPS 202 padding.
    st = np.zeros(25, dtype=np.uint64)
    st[0] ^= np.uint64(0x1F)
    st[136 // 8 - 1] ^= np.uint64(0x80) << np.uint64(56)
    out = orc.keccak_f1600(st)
    assert out.tobytes()[:136] == hashlib.shake_256(b"").digest(136)
