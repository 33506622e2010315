"""Oracle encodings: LSB-first bit packing pinned to numpy's little-endian packbits,
pack o unpack identity, and the byte sizes implied by Tab. 1."""
import json
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "params_table1.json")))


@pytest.mark.parametrize("b", [3, 4, 6, 10, 13, 18, 20])
def test_bitpack_is_lsb_first(orc, b):
    rng = np.random.default_rng(b)
    v = rng.integers(0, 1 << b, size=256, dtype=np.uint32)
    bits = ((v[:, None] >> np.arange(b, dtype=np.uint32)) & 1).astype(np.uint8).reshape(-1)
    expect = np.packbits(bits, bitorder="little").tobytes()
    assert orc.bitpack(v, b) == expect
    assert np.array_equal(orc.bitunpack(expect, 256, b), v)


@pytest.mark.parametrize("b", [3, 4, 6, 10, 13])
def test_pack_unpack_every_value(orc, b):
    v = np.arange(1 << b, dtype=np.uint32)
    v = np.resize(v, ((v.size + 255) // 256) * 256)
    assert np.array_equal(orc.bitunpack(orc.bitpack(v, b), v.size, b), v)


def test_params_match_table1(orc):
    for lv, g in GOLD["levels"].items():
        p = orc.params(int(lv))
        for key in ("k", "l", "tau", "gamma1", "gamma2", "eta", "beta", "omega"):
            assert p[key] == g[key], (lv, key)
        assert p["beta"] == p["tau"] * p["eta"]
        assert (GOLD["q"] - 1) % (2 * p["gamma2"]) == 0


def test_sizes(orc):
    expect = {2: (1312, 2528, 2420), 3: (1952, 4000, 3293), 5: (2592, 4864, 4595)}
    for lv, (pk, sk, sig) in expect.items():
        p = orc.params(lv)
        assert (p["pk_bytes"], p["sk_bytes"], p["sig_bytes"]) == (pk, sk, sig)
        pkb, skb = orc.keygen(lv, bytes(32))
        assert len(pkb) == pk and len(skb) == sk
