"""GPU parity at the ML-DSA levels 44 / 65 / 87 (FIPS 204 form; the oracle's readings and pins are
in tests/test_oracle_mldsa.py): KeyGen, deterministic and hedged Sign (staged and persistent
forms) and Verify through the C-ABI, bit-exact against the oracle on the same seeded inputs,
including message lengths around the block boundaries of mu's 66-byte prefix, key tables, a
10,000-task batch in the benchmark's launch configuration, and the rejections that hold at any
size (flipped signatures, the round-3 variant of the same bytes)."""
import hashlib

import numpy as np
import pytest

import oracle
from paper_2211_12265_amd import workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LEVELS = [44, 65, 87]
# lengths where mu's input tr || 0 || 0 || M crosses a SHAKE256 block (136 - 66 = 70, 206, 342)
EDGE_LENGTHS = [0, 1, 2, 3, 69, 70, 71, 72, 205, 206, 207, 341, 342, 343]


@pytest.fixture(scope="module", params=["staged", "persistent"])
def sctx(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import dilithium as dl
    c = dl.Context(0, mode=dl.MODE_STAGED if request.param == "staged" else dl.MODE_PERSISTENT)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import dilithium as dl
    c = dl.Context(0, mode=dl.MODE_PERSISTENT)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _keygen(ctx, level, seeds):
    from paper_2211_12265_amd import dilithium as dl
    pkl, skl, _ = dl.sizes(level)
    n = seeds.shape[0]
    pk = torch.zeros((n, pkl), dtype=torch.uint8, device="cuda")
    sk = torch.zeros((n, skl), dtype=torch.uint8, device="cuda")
    ctx.keygen(level, dev(seeds), pk, sk)
    torch.cuda.synchronize()
    return pk, sk


def _sign(ctx, level, sk, msg, off, key_idx=None, rnd=None):
    from paper_2211_12265_amd import dilithium as dl
    n = off.size - 1
    sig = torch.zeros((n, dl.sizes(level)[2]), dtype=torch.uint8, device="cuda")
    ctx.sign(level, sk, dev(msg), dev(off.astype(np.int64)), sig,
             key_idx=None if key_idx is None else dev(key_idx.astype(np.int32)),
             rnd=None if rnd is None else dev(rnd))
    torch.cuda.synchronize()
    return sig


def _verify(ctx, level, pk, msg, off, sig, key_idx=None):
    n = off.size - 1
    v = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    ctx.verify(level, pk, dev(msg), dev(off.astype(np.int64)), sig, v,
               key_idx=None if key_idx is None else dev(key_idx.astype(np.int32)))
    torch.cuda.synchronize()
    return v.cpu().numpy()


@pytest.mark.parametrize("level", LEVELS)
def test_sizes(level):
    from paper_2211_12265_amd import dilithium as dl
    p = oracle.params(level)
    assert dl.sizes(level) == (p["pk_bytes"], p["sk_bytes"], p["sig_bytes"])


@pytest.mark.parametrize("level", LEVELS)
def test_keygen_parity(ctx, level):
    seeds = workload.keygen_seeds(64, seed=200 + level)
    pk, sk = _keygen(ctx, level, seeds)
    opk, osk = oracle.keygen_batch(level, seeds)
    assert np.array_equal(pk.cpu().numpy(), opk)
    assert np.array_equal(sk.cpu().numpy(), osk)


@pytest.mark.parametrize("level", LEVELS)
def test_sign_verify_parity(sctx, level):
    n = 64
    pk, sk = _keygen(sctx, level, workload.keygen_seeds(n, seed=210 + level))
    lens = workload.uniform_lengths(n, 0, 700, seed=level)
    lens[:len(EDGE_LENGTHS)] = EDGE_LENGTHS
    msg, off = workload.messages(lens, seed=level)
    sig = _sign(sctx, level, sk, msg, off)
    osig, iters = oracle.sign_batch(level, sk.cpu().numpy(), msg, off)
    got = sig.cpu().numpy()
    bad = [i for i in range(n) if not np.array_equal(got[i], osig[i])]
    assert not bad, f"signature mismatch for tasks {bad[:8]} (iters {iters[bad[:8]]})"
    assert _verify(sctx, level, pk, msg, off, sig).tolist() == [1] * n
    # the deterministic signer is the hedged one with rnd = 0
    zero = np.zeros((n, 32), np.uint8)
    assert np.array_equal(_sign(sctx, level, sk, msg, off, rnd=zero).cpu().numpy(), got)


@pytest.mark.parametrize("level", LEVELS)
def test_hedged_sign_parity(sctx, level):
    n = 40
    pk, sk = _keygen(sctx, level, workload.keygen_seeds(n, seed=220 + level))
    lens = workload.uniform_lengths(n, 0, 300, seed=221 + level)
    lens[:4] = [0, 70, 71, 206]
    msg, off = workload.messages(lens, seed=221 + level)
    rnd = workload.random_bytes("dil/mldsa-rnd", level, (n, 32))
    sig = _sign(sctx, level, sk, msg, off, rnd=rnd)
    osig, _ = oracle.sign_batch(level, sk.cpu().numpy(), msg, off, rnd=rnd)
    assert np.array_equal(sig.cpu().numpy(), osig)
    assert not np.array_equal(osig, oracle.sign_batch(level, sk.cpu().numpy(), msg, off)[0])
    assert _verify(sctx, level, pk, msg, off, sig).tolist() == [1] * n


def test_rnd_rows_and_persistent_shapes(ctx):
    from paper_2211_12265_amd import dilithium as dl
    level = 65
    pk, sk = _keygen(ctx, level, workload.keygen_seeds(2, seed=230))
    msg, off = workload.messages(workload.fixed_lengths(2, 32), seed=230)
    sig = torch.zeros((2, dl.sizes(level)[2]), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):   # ML-DSA takes 32 rnd bytes per task
        ctx.sign(level, sk, dev(msg), dev(off.astype(np.int64)), sig, rnd=dev(np.zeros((2, 64), np.uint8)))
    buf = torch.zeros(2 * 32 + 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(dl.DilError):  # misaligned rnd rows
        ctx.sign(level, sk, dev(msg), dev(off.astype(np.int64)), sig, rnd=buf[1:1 + 64].view(2, 32))
    for waves in (1, 2):             # the loop kernel is built in the four-wavefront shape only
        ctx.set_param("persist.waves", waves)
        try:
            with pytest.raises(dl.DilError):
                ctx.sign(level, sk, dev(msg), dev(off.astype(np.int64)), sig)
        finally:
            ctx.set_param("persist.waves", 4)
    torch.cuda.synchronize()


@pytest.mark.parametrize("level", LEVELS)
def test_key_idx_and_keyset(sctx, level):
    from paper_2211_12265_amd import dilithium as dl
    nkeys, n = 5, 24
    pk, sk = _keygen(sctx, level, workload.keygen_seeds(nkeys, seed=240 + level))
    kidx = np.random.default_rng(level).integers(0, nkeys, size=n).astype(np.uint32)
    msg, off = workload.messages(workload.uniform_lengths(n, 0, 400, seed=level + 240), seed=level + 240)
    osig, _ = oracle.sign_batch(level, sk.cpu().numpy(), msg, off, key_idx=kidx)
    assert np.array_equal(_sign(sctx, level, sk, msg, off, key_idx=kidx).cpu().numpy(), osig)
    ks = dl.KeySet(sctx, level, pk=pk, sk=sk)
    try:
        sig = torch.zeros((n, dl.sizes(level)[2]), dtype=torch.uint8, device="cuda")
        ks.sign(sctx, dev(kidx.astype(np.int32)), dev(msg), dev(off.astype(np.int64)), sig)
        torch.cuda.synchronize()
        assert np.array_equal(sig.cpu().numpy(), osig)
        bad = osig.copy()
        bad[::3, 50] ^= 1
        v = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        ks.verify(sctx, dev(kidx.astype(np.int32)), dev(msg), dev(off.astype(np.int64)), dev(bad), v)
        torch.cuda.synchronize()
        expect = oracle.verify_batch(level, pk.cpu().numpy(), msg, off, bad, key_idx=kidx)
        assert np.array_equal(v.cpu().numpy(), expect) and expect.sum() == n - len(range(0, n, 3))
    finally:
        ks.close()


@pytest.mark.parametrize("level", LEVELS)
def test_verify_rejections(ctx, level):
    pk, sk = _keygen(ctx, level, workload.keygen_seeds(1, seed=250 + level))
    msg, off = workload.messages(workload.fixed_lengths(1, 40), seed=250)
    sig = _sign(ctx, level, sk, msg, off).cpu().numpy()
    p = oracle.params(level)
    nbits = sig.shape[1] * 8
    bits = np.unique(np.concatenate([np.arange(0, 8 * p["ct_bytes"]), np.arange(0, nbits, 7),
                                     np.arange(nbits - 8 * (p["omega"] + p["k"]), nbits)]))
    flipped = np.repeat(sig, bits.size, axis=0)
    flipped[np.arange(bits.size), bits // 8] ^= (1 << (bits % 8)).astype(np.uint8)
    offs = np.arange(bits.size + 1, dtype=np.uint64) * 40
    kidx = np.zeros(bits.size, np.uint32)
    v = _verify(ctx, level, pk, np.tile(msg, bits.size), offs, dev(flipped), key_idx=kidx)
    assert v.sum() == 0
    assert np.array_equal(v, oracle.verify_batch(level, pk.cpu().numpy(), np.tile(msg, bits.size), offs, flipped,
                                                 key_idx=kidx))


def test_round3_and_mldsa_do_not_cross_verify(ctx):
    """Level 44 and level 2 share every size: each rejects the other's signatures."""
    n = 8
    msg, off = workload.messages(workload.uniform_lengths(n, 0, 200, seed=260), seed=260)
    pk44, sk44 = _keygen(ctx, 44, workload.keygen_seeds(n, seed=260))
    pk2, sk2 = _keygen(ctx, 2, workload.keygen_seeds(n, seed=260))
    s44, s2 = _sign(ctx, 44, sk44, msg, off), _sign(ctx, 2, sk2, msg, off)
    assert _verify(ctx, 44, pk44, msg, off, s44).tolist() == [1] * n
    assert _verify(ctx, 2, pk44, msg, off, s44).tolist() == [0] * n
    assert _verify(ctx, 44, pk2, msg, off, s2).tolist() == [0] * n


def test_tr_by_hashlib(ctx):
    """The GPU key's tr is H(pk, 64), recomputed by hashlib."""
    level = 87
    pk, sk = _keygen(ctx, level, workload.keygen_seeds(3, seed=270))
    pkh, skh = pk.cpu().numpy(), sk.cpu().numpy()
    for i in range(3):
        assert skh[i, 64:128].tobytes() == hashlib.shake_256(pkh[i].tobytes()).digest(64)


@pytest.mark.parametrize("level", [44, 65, 87])
def test_ten_thousand_tasks(level):
    """A 10,000-task batch in the benchmark's launch configuration (recorded schedule, graph
    replay, automatic tail batches; 32-byte messages at level 44, uniform 32..4096-byte ones at
    65 / 87): every key and signature equals the oracle's and every signature verifies."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import autotune
    from paper_2211_12265_amd import dilithium as dl
    n = 10000
    c = dl.Context(0, mode=dl.MODE_PERSISTENT)
    try:
        c.set_param("graph", 1)
        mix = "fixed32" if level == 44 else "uniform"
        autotune.apply_schedule(c, autotune.cached_schedule(level, n, mix))
        seeds = workload.keygen_seeds(n, seed=level)
        lens = workload.fixed_lengths(n, 32) if mix == "fixed32" else workload.uniform_lengths(n, 32, 4096, seed=level)
        msg, off = workload.messages(lens, seed=level)
        opk, osk = oracle.keygen_batch(level, seeds)
        osig, _ = oracle.sign_batch(level, osk, msg, off)
        pk, sk = _keygen(c, level, seeds)
        assert np.array_equal(pk.cpu().numpy(), opk) and np.array_equal(sk.cpu().numpy(), osk)
        sig = _sign(c, level, sk, msg, off)
        got = sig.cpu().numpy()
        bad = np.flatnonzero((got != osig).any(axis=1))
        assert bad.size == 0, f"{bad.size} signatures differ, first {bad[:8]}"
        assert _verify(c, level, pk, msg, off, sig).sum() == n
    finally:
        c.close()


def _csr(parts):
    buf = np.frombuffer(b"".join(parts), np.uint8).copy() if sum(map(len, parts)) else np.zeros(0, np.uint8)
    return buf, np.concatenate([[0], np.cumsum([len(x) for x in parts])]).astype(np.uint64)


@pytest.mark.parametrize("level", LEVELS)
def test_formatted_messages_parity(sctx, level):
    """"mldsa.internal": Sign and Verify of formatted messages M' (context strings of 0..255
    bytes) equal the oracle's internal functions, the empty context reproduces pure signing,
    a signature does not verify under another context, and key tables take the same form."""
    from paper_2211_12265_amd import dilithium as dl
    n = 40
    pk, sk = _keygen(sctx, level, workload.keygen_seeds(n, seed=260 + level))
    lens = workload.uniform_lengths(n, 0, 300, seed=261 + level)
    msg, off = workload.messages(lens, seed=261 + level)
    msgs = [msg[int(off[i]):int(off[i + 1])].tobytes() for i in range(n)]
    ctxs = [workload.random_bytes("test/mldsa-ctx", 7 * i + level, (i * 37 % 256,)).tobytes() for i in range(n)]
    fm, foff = _csr([oracle.mldsa_format(m, c) for m, c in zip(msgs, ctxs)])
    em, eoff = _csr([oracle.mldsa_format(m) for m in msgs])
    rnd = workload.random_bytes("dil/mldsa-rnd", 100 + level, (n, 32))
    osig, _ = oracle.sign_batch(level, sk.cpu().numpy(), fm, foff, internal=True)
    ohedged, _ = oracle.sign_batch(level, sk.cpu().numpy(), fm, foff, rnd=rnd, internal=True)
    pure = _sign(sctx, level, sk, msg, off).cpu().numpy()
    sctx.set_param("mldsa.internal", 1)
    try:
        got = _sign(sctx, level, sk, fm, foff)
        assert np.array_equal(got.cpu().numpy(), osig)
        assert np.array_equal(_sign(sctx, level, sk, fm, foff, rnd=rnd).cpu().numpy(), ohedged)
        assert np.array_equal(_sign(sctx, level, sk, em, eoff).cpu().numpy(), pure)
        assert _verify(sctx, level, pk, fm, foff, got).tolist() == [1] * n
        assert _verify(sctx, level, pk, em, eoff, got).tolist() == [int(not c) for c in ctxs]
        ks = dl.KeySet(sctx, level, pk=pk, sk=sk)
        try:
            sig = torch.zeros((n, dl.sizes(level)[2]), dtype=torch.uint8, device="cuda")
            ks.sign(sctx, None, dev(fm), dev(foff.astype(np.int64)), sig)
            v = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            ks.verify(sctx, None, dev(fm), dev(foff.astype(np.int64)), sig, v)
            v_na = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            ks.verify(sctx, None, dev(fm), dev(foff.astype(np.int64)), sig, v_na, noalloc=True)
            torch.cuda.synchronize()
            assert np.array_equal(sig.cpu().numpy(), osig)
            assert v.cpu().numpy().tolist() == [1] * n and v_na.cpu().numpy().tolist() == [1] * n
        finally:
            ks.close()
    finally:
        sctx.set_param("mldsa.internal", 0)
    # pure mode again on the same context
    assert np.array_equal(_sign(sctx, level, sk, msg, off).cpu().numpy(), pure)


def test_formatted_messages_only_at_mldsa_levels(ctx):
    from paper_2211_12265_amd import dilithium as dl
    pk, sk = _keygen(ctx, 2, workload.keygen_seeds(2, seed=270))
    msg, off = workload.messages(workload.fixed_lengths(2, 32), seed=270)
    with pytest.raises(dl.DilError):
        ctx.set_param("mldsa.internal", 2)
    ctx.set_param("mldsa.internal", 1)
    try:
        with pytest.raises(dl.DilError):
            _sign(ctx, 2, sk, msg, off)
        with pytest.raises(dl.DilError):
            _verify(ctx, 2, pk, msg, off, torch.zeros((2, dl.sizes(2)[2]), dtype=torch.uint8, device="cuda"))
    finally:
        ctx.set_param("mldsa.internal", 0)
    torch.cuda.synchronize()
