"""Oracle samplers (Sec. 2.3 'Sampling', Alg. 4): ranges, counts, acceptance rates and
distributions.  The acceptance rates pin ExpandA's 23-bit mask and ExpandS's thresholds, the
support statistic pins SampleInBall's b <= i draw.  Exact byte streams against the official
round-3 KATs (byte and nibble order, nonce encodings, ExpandMask's orientation, the sign-bit
source) are parity unpinned."""
import numpy as np
import pytest

import oracle_pins
from paper_2211_12265_amd import workload

Q = 8380417


def test_expand_a_range_and_shape(orc):
    rho = workload.random_bytes("test/rho", 0, (32,)).tobytes()
    for level, (k, l) in {2: (4, 4), 3: (6, 5), 5: (8, 7)}.items():
        A = orc.expand_a(level, rho)
        assert A.shape == (k, l, 256)
        assert A.min() >= 0 and A.max() < Q
        # distinct streams per (i, j)
        flat = A.reshape(k * l, 256)
        assert len({row.tobytes() for row in flat}) == k * l


def test_expand_a_uniform_statistics(orc):
    seeds = workload.expand_a_inputs(4096, seed=1)
    polys = orc.expand_a_polys(seeds)
    x = polys.astype(np.float64) / Q
    assert abs(x.mean() - 0.5) < 0.002
    hist, _ = np.histogram(x, bins=16, range=(0, 1))
    assert hist.min() > 0.95 * hist.mean() and hist.max() < 1.05 * hist.mean()
    # matrix entries for one rho equal the per-poly entry point with (j, i) nonces
    A = orc.expand_a(2, seeds[0, :32].tobytes())
    for idx in range(16):
        j, i = idx % 4, (idx // 4) % 4
        assert np.array_equal(A[i, j], polys[idx])


@pytest.mark.parametrize("level,eta", [(2, 2), (3, 4), (5, 2)])
def test_expand_s_range(orc, level, eta):
    s = orc.expand_s(level, workload.random_bytes("test/rhop", level, (64,)).tobytes())
    assert s.min() >= -eta and s.max() <= eta
    vals, counts = np.unique(s, return_counts=True)
    assert list(vals) == list(range(-eta, eta + 1))
    # uniform on [-eta, eta]
    assert counts.min() > 0.6 * counts.mean()


@pytest.mark.parametrize("level,g1", [(2, 1 << 17), (3, 1 << 19), (5, 1 << 19)])
def test_expand_mask_range(orc, level, g1):
    rhop = workload.random_bytes("test/rhop", level, (64,)).tobytes()
    y0 = orc.expand_mask(level, rhop, 0)
    y1 = orc.expand_mask(level, rhop, y0.shape[0])
    assert y0.min() >= -g1 + 1 and y0.max() <= g1
    assert not np.array_equal(y0, y1)
    # y_i of kappa = l equals y_{i-1}-style shift: stream i of kappa is nonce kappa + i
    ya = orc.expand_mask(level, rhop, 1)
    assert np.array_equal(ya[0], y0[1])


@pytest.mark.parametrize("level,tau", [(2, 39), (3, 49), (5, 60)])
def test_sample_in_ball_weight(orc, level, tau):
    for t in range(50):
        c = orc.sample_in_ball(level, workload.random_bytes("test/ct", t, (32,)).tobytes())
        assert np.count_nonzero(c) == tau
        assert set(np.unique(c[c != 0])) <= {-1, 1}


def test_expand_a_acceptance_rate():
    # rejected candidates over 4096 streams: q / 2^23 acceptance, within 4 standard deviations
    assert oracle_pins.expand_a_acceptance(streams=4096, seed=1) == []
    assert oracle_pins.expand_a_acceptance(streams=4096, seed=5) == []


@pytest.mark.parametrize("eta", [2, 4])
def test_expand_s_acceptance_rate_and_distribution(eta):
    # 15/16 (eta = 2) or 9/16 (eta = 4) of the nibbles kept; coefficients uniform on [-eta, eta]
    assert oracle_pins.expand_s_acceptance(eta, streams=4096, seed=2) == []


@pytest.mark.parametrize("level", [2, 5])
def test_sample_in_ball_support_uniform(level):
    # the nonzero positions form a uniform tau-subset (Fisher-Yates with b <= i)
    assert oracle_pins.sample_in_ball_support(level, samples=60000, seed=3) == []
