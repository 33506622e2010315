"""Planted mistakes: each variant of the oracle built with -DDIL_PLANT=<n> (a wrong rotation
offset, swapped chi operands, a non-bit-reversed twiddle, a dropped 1/n, a wrong mod+- tie, a
dropped Decompose special case, a wrong sign in MakeHint, a wrong UseHint branch, MSB-first
packing, a dropped challenge position, a dropped beta, a dropped c t1 term, a wrong c t0 sign,
a wrong t0 offset, ExpandA's 23-bit mask dropped, ExpandS's eta = 2 threshold moved to 16, Sign's
[h] > omega rejection dropped, Sign's ||c t0|| >= gamma2 rejection dropped, SampleInBall drawing
b < i; and in the ML-DSA form: the k / l bytes left out of KeyGen's seed expansion, the two zero
bytes of mu dropped, rnd left out of rho'', SampleInBall seeded by 32 bytes of a longer ctilde,
the internal form's formatted message formatted again)
must fail at least one of the oracle's pins.  Everything runs on the CPU."""
import hashlib
import os

import numpy as np
import pytest

import oracle
import oracle_pins
from paper_2211_12265_amd import workload

Q = 8380417
PLANTS = list(range(1, 25))


def _schoolbook(a, b):
    full = np.zeros(511, dtype=object)
    for i in range(256):
        full[i:i + 256] += int(a[i]) * b.astype(object)
    out = full[:256] - np.concatenate([full[256:], [0]])
    return np.array([int(x) % Q for x in out], dtype=np.int32)


def pins_hold(stop_early: bool = False):
    """A fast subset of the oracle pins; returns the list of failing pin names (with stop_early,
    only the first: a planted mistake has to fail one of them, and a broken signer makes the
    later signing pins run to their iteration caps)."""
    failed = []
    data = workload.random_bytes("test/mut", 0, (400,)).tobytes()
    for n in (0, 1, 135, 136, 167, 168, 300):
        if oracle.shake128(data[:n], 200) != hashlib.shake_128(data[:n]).digest(200) or \
           oracle.shake256(data[:n], 200) != hashlib.shake_256(data[:n]).digest(200):
            failed.append("shake")
            break
    polys = workload.uniform_polys(2, seed=9)
    a, b = polys[0], polys[1]
    if not np.array_equal(oracle.ntt(a), oracle.ntt_definition(a)):
        failed.append("ntt-definition")
    if not np.array_equal(oracle.intt(oracle.ntt(a)), a):
        failed.append("ntt-roundtrip")
    prod = oracle.intt((oracle.ntt(a).astype(np.int64) * oracle.ntt(b) % Q).astype(np.int32))
    if not np.array_equal(prod, _schoolbook(a, b)):
        failed.append("schoolbook")
    allr = np.arange(Q, dtype=np.int32)
    r1, r0 = oracle.power2round(allr)
    if not (np.array_equal(r1.astype(np.int64) * 8192 + r0, allr) and r0.min() > -4096 and r0.max() <= 4096):
        failed.append("power2round")
    g2 = 95232
    d1, d0 = oracle.decompose(allr, g2)
    special = allr > Q - 1 - g2
    if not (np.array_equal((d1.astype(np.int64) * 2 * g2 + d0) % Q, allr) and d1.max() == 43 and
            np.all(d1[special] == 0) and np.abs(d0).max() <= g2):
        failed.append("decompose")
    rng = np.random.default_rng(1)
    r = np.concatenate([rng.integers(0, Q, 200000, dtype=np.int32), np.arange(Q - 2 * g2, Q, dtype=np.int32),
                        np.arange(0, 4 * g2, 7, dtype=np.int32)])
    for zv in (g2, -g2, 0, 1, -1):
        z = np.full(r.size, zv, np.int32)
        got = oracle.use_hint(oracle.make_hint(z, r, g2), r, g2)
        hb, _ = oracle.decompose(((r.astype(np.int64) + z) % Q).astype(np.int32), g2)
        if not np.array_equal(got, hb):
            failed.append("hint")
            break
    v = rng.integers(0, 1 << 13, 256).astype(np.uint32)
    bits = ((v[:, None] >> np.arange(13, dtype=np.uint32)) & 1).astype(np.uint8).reshape(-1)
    if oracle.bitpack(v, 13) != np.packbits(bits, bitorder="little").tobytes():
        failed.append("packbits")
    c = oracle.sample_in_ball(2, b"\x07" * 32)
    if np.count_nonzero(c) != 39:
        failed.append("sample-in-ball")
    oracle.lib().dil_ref_set_sign_cap(300)   # a correct signer exceeds this with probability ~1e-35
    try:
        for level in (2,):
            pk, sk = oracle.keygen_batch(level, workload.keygen_seeds(6, seed=5), nthreads=4)
            msg, off = workload.messages(workload.fixed_lengths(6, 32), seed=5)
            sig, it = oracle.sign_batch(level, sk, msg, off, nthreads=4)
            if (it < 1).any() or oracle.verify_batch(level, pk, msg, off, sig, nthreads=4).tolist() != [1] * 6:
                failed.append("round-trip")
        # the ML-DSA form's hash inputs, under the same iteration cap
        for level in (44, 87):
            if failed and stop_early:
                break
            failed += oracle_pins.mldsa_hash_inputs(level)
    finally:
        oracle.lib().dil_ref_set_sign_cap(0)
    if failed and stop_early:
        return failed
    # sampler acceptance rates and distributions, Sign's output conditions on crafted keys
    for name, pin in (("expand-a-acceptance", lambda: oracle_pins.expand_a_acceptance(streams=2048)),
                      ("expand-s-acceptance", lambda: oracle_pins.expand_s_acceptance(2, streams=2048)),
                      ("sign-ct0-bound", lambda: oracle_pins.sign_ct0_bound(2)),
                      ("sign-hint-bound", lambda: oracle_pins.sign_hint_bound(2)),
                      ("sample-in-ball-support", lambda: oracle_pins.sample_in_ball_support(2, samples=60000))):
        if pin():
            failed.append(name)
            if stop_early:
                return failed
    return failed


def test_unmodified_oracle_passes_the_fast_pins():
    assert pins_hold() == []


@pytest.mark.parametrize("plant", PLANTS)
def test_planted_mistake_is_caught(tmp_path, plant):
    path = oracle.build(force=True, out=str(tmp_path / f"liboracle_plant{plant}.so"),
                        defines=[f"DIL_PLANT={plant}"])
    saved = oracle._LIB
    try:
        oracle._LIB = oracle.bind(path)
        failed = pins_hold(stop_early=True)
    finally:
        oracle._LIB = saved
    assert failed, f"planted mistake {plant} passed every pin"
