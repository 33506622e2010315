"""Oracle Power2Round / Decompose / MakeHint / UseHint pinned by exhaustive identities
over all of [0, q) (Sec. 2.3, 'Bits Extraction and Hints')."""
import numpy as np
import pytest

Q = 8380417
ALL = np.arange(Q, dtype=np.int32)


def test_power2round_exhaustive(orc):
    r1, r0 = orc.power2round(ALL)
    assert np.array_equal(r1.astype(np.int64) * 8192 + r0, ALL.astype(np.int64))
    assert r0.min() > -4096 and r0.max() <= 4096      # mod+- 2^13 range (Sec. 2.1)
    assert r1.min() >= 0 and r1.max() <= 1023          # t1 fits 10 bits
    assert (r0 == 4096).any() and (r0 == -4095).any()


@pytest.mark.parametrize("gamma2,m", [(95232, 44), (261888, 16)])
def test_decompose_exhaustive(orc, gamma2, m):
    alpha = 2 * gamma2
    assert (Q - 1) % alpha == 0 and (Q - 1) // alpha == m
    r1, r0 = orc.decompose(ALL, gamma2)
    r1 = r1.astype(np.int64); r0 = r0.astype(np.int64)
    assert np.array_equal((r1 * alpha + r0) % Q, ALL.astype(np.int64))
    assert r1.min() >= 0 and r1.max() == m - 1
    assert np.abs(r0).max() <= gamma2
    special = ALL.astype(np.int64) > Q - 1 - gamma2
    assert np.all(r1[special] == 0)
    assert np.all(r0[special] == ALL[special].astype(np.int64) - Q)
    assert np.all(r0[~special] > -gamma2)


@pytest.mark.parametrize("gamma2", [95232, 261888])
def test_hint_correctness_property(orc, gamma2):
    # UseHint(MakeHint(z, r), r) == HighBits(r + z) for every r in [0, q) and |z| <= gamma2
    zs = [0, 1, -1, gamma2, -gamma2, gamma2 - 1, -(gamma2 - 1), 12345, -54321]
    rng = np.random.default_rng(7)
    for zval in zs + [None, None]:
        if zval is None:
            z = rng.integers(-gamma2, gamma2 + 1, size=Q, dtype=np.int32)
        else:
            z = np.full(Q, zval, dtype=np.int32)
        h = orc.make_hint(z, ALL, gamma2)
        got = orc.use_hint(h, ALL, gamma2)
        rz = ((ALL.astype(np.int64) + z) % Q).astype(np.int32)
        hb, _ = orc.decompose(rz, gamma2)
        assert np.array_equal(got, hb), zval


def test_make_hint_matches_definition_pointwise(orc):
    gamma2 = 95232
    rng = np.random.default_rng(8)
    r = rng.integers(0, Q, size=200000, dtype=np.int32)
    z = rng.integers(-gamma2, gamma2 + 1, size=r.size, dtype=np.int32)
    h = orc.make_hint(z, r, gamma2)
    a1, _ = orc.decompose(r, gamma2)
    b1, _ = orc.decompose(((r.astype(np.int64) + z) % Q).astype(np.int32), gamma2)
    assert np.array_equal(h, (a1 != b1).astype(np.int32))
    assert 0 < h.sum() < r.size
