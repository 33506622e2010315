"""Serving loop: mixed-level Sign/Verify requests through the continuous-batching
loop give exactly the oracle's outputs, every result is the same alone and in the
mix (deterministic signing: tolerance 0 bytes), a memory budget below one batch
makes requests wait for later batches instead of failing, and batches overlap."""
import numpy as np
import pytest

import oracle
from paper_2211_12265_amd import workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd import serving as sv
    ctx = dl.Context(0, mode=dl.MODE_PERSISTENT)
    keys = {2: 12, 3: 7, 5: 5}
    keysets, host = {}, {}
    for lv, nk in keys.items():
        pkl, skl, _ = dl.sizes(lv)
        seeds = workload.keygen_seeds(nk, seed=200 + lv)
        pk = torch.zeros((nk, pkl), dtype=torch.uint8, device="cuda")
        sk = torch.zeros((nk, skl), dtype=torch.uint8, device="cuda")
        ctx.keygen(lv, torch.from_numpy(seeds).cuda(), pk, sk)
        keysets[lv] = dl.KeySet(ctx, lv, pk=pk, sk=sk)
        host[lv] = (pk.cpu().numpy(), sk.cpu().numpy())
    reqs = sv.build_requests(300, lam=20000.0, keys_per_level=keys, seed=7)
    flipped = sv.attach_signatures(reqs, ctx, keysets, flip_rate=0.1, seed=7)
    yield dl, sv, ctx, keysets, host, reqs, flipped
    for ks in keysets.values():
        ks.close()
    ctx.close()


@pytest.mark.parametrize("engine", ["python", "native"])
def test_serving_matches_oracle(setup, engine):
    dl, sv, ctx, keysets, host, reqs, flipped = setup
    cls = sv.Server if engine == "python" else sv.NativeServer
    server = cls(keysets, n_streams=3, max_batch=64, mem_budget=2 << 30, max_msg_bytes=1 << 20)
    res = server.serve(reqs)
    server.close()
    assert np.isfinite(res.t_done).all()
    _check_against_oracle(sv, host, reqs, flipped, res)


def _check_against_oracle(sv, host, reqs, flipped, res):
    for lv in np.unique(reqs.level).tolist():
        pk, sk = host[lv]
        s = np.nonzero((reqs.level == lv) & (reqs.op == sv.SIGN))[0]
        if s.size:
            lens = reqs.msg_off[s + 1] - reqs.msg_off[s]
            msg = sv._gather(reqs.msg, reqs.msg_off[s], lens)
            off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
            osig, _ = oracle.sign_batch(lv, sk, msg, off, key_idx=reqs.key[s].astype(np.uint32))
            got = np.stack([res.sig[int(r)] for r in s])
            assert np.array_equal(got, osig)
        v = np.nonzero((reqs.level == lv) & (reqs.op == sv.VERIFY))[0]
        if v.size:
            lens = reqs.msg_off[v + 1] - reqs.msg_off[v]
            msg = sv._gather(reqs.msg, reqs.msg_off[v], lens)
            off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
            ss = sv.sig_size(lv)
            sigs = sv._gather(reqs.sig_in, reqs.sig_off[v], np.full(v.size, ss)).reshape(-1, ss)
            ov = oracle.verify_batch(lv, pk, msg, off, sigs, key_idx=reqs.key[v].astype(np.uint32))
            assert np.array_equal(res.verdict[v], ov)
            assert np.array_equal(ov == 0, flipped[v])


@pytest.mark.parametrize("engine", ["python", "native"])
def test_same_alone_and_in_mix(setup, engine):
    dl, sv, ctx, keysets, host, reqs, flipped = setup
    cls = sv.Server if engine == "python" else sv.NativeServer
    server = cls(keysets, n_streams=4, max_batch=128, mem_budget=2 << 30, max_msg_bytes=1 << 20)
    mixed = server.serve(reqs)
    for r in range(len(reqs)):
        one = sv.Requests(np.zeros(1), reqs.op[r:r + 1], reqs.level[r:r + 1], reqs.key[r:r + 1],
                          reqs.msg[reqs.msg_off[r]:reqs.msg_off[r + 1]].copy(),
                          np.array([0, reqs.msg_off[r + 1] - reqs.msg_off[r]], np.int64))
        if reqs.op[r] == sv.VERIFY:
            ss = sv.sig_size(int(reqs.level[r]))
            one.sig_in = reqs.sig_in[reqs.sig_off[r]:reqs.sig_off[r] + ss].copy()
            one.sig_off = np.array([0], np.int64)
        alone = server.serve(one)
        if reqs.op[r] == sv.SIGN:
            assert np.array_equal(alone.sig[0], mixed.sig[int(r)])
        else:
            assert alone.verdict[0] == mixed.verdict[r]
    server.close()


@pytest.mark.parametrize("engine", ["python", "native"])
def test_out_of_range_key_rejected_before_any_work(setup, engine):
    """A request naming a key row past its level's table is refused on the host (the device
    reads key rows without bounds checks), and the engine then still serves a valid trace."""
    dl, sv, ctx, keysets, host, reqs, flipped = setup
    cls = sv.Server if engine == "python" else sv.NativeServer
    server = cls(keysets, n_streams=2, max_batch=64, mem_budget=2 << 30, max_msg_bytes=1 << 20)
    bad = sv.Requests(**vars(reqs))
    bad.key = reqs.key.copy()
    bad.key[int(np.argmax(reqs.level == 5))] = keysets[5].n_keys
    with pytest.raises((ValueError, dl.DilError)) as err:
        server.serve(bad)
    if engine == "native":
        assert err.value.code == -1   # DIL_EINVAL
    res = server.serve(reqs)
    server.close()
    assert np.isfinite(res.t_done).all()
    v = reqs.op == sv.VERIFY
    assert np.array_equal(res.verdict[v] == 0, flipped[v])


@pytest.mark.parametrize("engine", ["python", "native"])
def test_budget_below_one_batch_queues_requests(setup, engine):
    """With a memory budget that holds the workspaces of only a few requests per (level, op),
    every request still completes with the oracle's output: the ones that do not fit a batch
    wait for a later one.  The budget is a quarter of what the engine reserves for full
    batches, so the per-group cap falls below the batch size."""
    dl, sv, ctx, keysets, host, reqs, flipped = setup
    cls = sv.Server if engine == "python" else sv.NativeServer
    full = cls(keysets, n_streams=3, max_batch=64, mem_budget=64 << 30, max_msg_bytes=1 << 20)
    first = full.serve(reqs)
    full.close()
    assert first.group_cap == 64
    big = first.reserved_bytes
    server = cls(keysets, n_streams=3, max_batch=64, mem_budget=big // 4, max_msg_bytes=1 << 20)
    res = server.serve(reqs)
    server.close()
    assert 1 <= res.group_cap < 64 and res.reserved_bytes <= big // 4
    assert np.isfinite(res.t_done).all()
    grp = 2 * np.searchsorted([2, 3, 5], reqs.level) + reqs.op
    largest = int(np.bincount(grp).max())
    assert res.batches >= -(-largest // res.group_cap)
    _check_against_oracle(sv, host, reqs, flipped, res)
    # a budget below one request per group is refused when the engine is created
    with pytest.raises(dl.DilError):
        cls(keysets, n_streams=3, max_batch=64, mem_budget=1 << 20, max_msg_bytes=1 << 20)


@pytest.mark.parametrize("engine", ["python", "native"])
def test_batches_overlap(setup, engine):
    """Every request at t = 0 with small batches: a lane is launched while another batch is
    still in flight (the engine counts such launches)."""
    dl, sv, ctx, keysets, host, reqs, flipped = setup
    cls = sv.Server if engine == "python" else sv.NativeServer
    server = cls(keysets, n_streams=4, max_batch=16, mem_budget=2 << 30, max_msg_bytes=1 << 20)
    burst = sv.Requests(**vars(reqs))
    burst.t_arrival = np.zeros(len(reqs))
    res = server.serve(burst)
    server.close()
    assert res.batches >= len(reqs) // 16
    assert res.overlapped > 0
    _check_against_oracle(sv, host, reqs, flipped, res)


@pytest.mark.parametrize("front", ["Service", "NativeService"])
def test_service_submit_and_wait_from_threads(front):
    """The interactive front ends (`Service` over the Python engine, `NativeService` over
    dil_server_start / submit / poll / wait / stop): three threads submit mixed Sign / Verify
    requests at levels 2 and ML-DSA-65 while earlier batches run; every ticket's result equals
    the oracle's (signature bytes, verdict), results are handed out once, and bad requests are
    refused at submission."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import threading
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd import serving as sv
    ctx = dl.Context(0, mode=dl.MODE_PERSISTENT)
    keysets, host = {}, {}
    for lv, nk in ((2, 6), (65, 4)):
        seeds = workload.keygen_seeds(nk, seed=300 + lv)
        pk, sk = oracle.keygen_batch(lv, seeds)
        host[lv] = (pk, sk)
        keysets[lv] = dl.KeySet(ctx, lv, pk=torch.from_numpy(pk).cuda(), sk=torch.from_numpy(sk).cuda())
    rng = np.random.default_rng(31)
    n = 240
    level = rng.choice([2, 65], size=n)
    op = (rng.random(n) < 0.6).astype(int)      # 60% verify
    key = np.array([rng.integers(0, 6 if lv == 2 else 4) for lv in level])
    lens = workload.uniform_lengths(n, 0, 400, seed=31)
    msgs = [workload.random_bytes("test/service", i, (int(lens[i]),)).tobytes() for i in range(n)]
    # verify requests carry the oracle's signature, every fourth with one bit flipped
    sig_in, expect = [None] * n, [None] * n
    for i in range(n):
        pk, sk = host[int(level[i])]
        s, _ = oracle.sign(int(level[i]), sk[key[i]].tobytes(), msgs[i])
        if op[i] == sv.SIGN:
            expect[i] = s
        else:
            if i % 4 == 0:
                b = bytearray(s)
                b[i % len(b)] ^= 1
                s = bytes(b)
            sig_in[i] = s
            expect[i] = bool(oracle.verify(int(level[i]), pk[key[i]].tobytes(), msgs[i], s) == 1)
    svc = getattr(sv, front)(keysets, n_streams=3, max_batch=32, mem_budget=2 << 30, max_msg_bytes=1 << 20)
    tickets = [None] * n

    def client(part):
        for i in range(part, n, 3):
            tickets[i] = svc.submit(int(level[i]), int(op[i]), int(key[i]), msgs[i], sig_in[i])

    threads = [threading.Thread(target=client, args=(p,)) for p in range(3)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    got = [svc.wait(t, timeout=120) for t in tickets]
    assert got == expect
    assert svc.poll(tickets[0]) is None            # handed out once
    assert svc.batches > 1
    with pytest.raises(ValueError):
        svc.submit(2, sv.SIGN, 6, b"x")             # key row outside the table
    with pytest.raises(ValueError):
        svc.submit(65, sv.VERIFY, 0, b"x")          # verify without a signature
    with pytest.raises(ValueError):
        svc.submit(3, sv.SIGN, 0, b"x")             # no table for the level
    svc.close()
    with pytest.raises(RuntimeError):
        svc.submit(2, sv.SIGN, 0, b"x")
    for ks in keysets.values():
        ks.close()
    ctx.close()


@pytest.mark.parametrize("engine", ["python", "native"])
def test_serving_mldsa_tables(engine):
    """Both engines serve key tables of ML-DSA levels beside round-3 ones (a trace mixing levels
    2, 65 and 87): every signature and verdict equals the oracle's."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd import serving as sv
    ctx = dl.Context(0, mode=dl.MODE_PERSISTENT)
    keys = {2: 6, 65: 5, 87: 4}
    keysets, host = {}, {}
    for lv, nk in keys.items():
        pk, sk = oracle.keygen_batch(lv, workload.keygen_seeds(nk, seed=320 + lv))
        host[lv] = (pk, sk)
        keysets[lv] = dl.KeySet(ctx, lv, pk=torch.from_numpy(pk).cuda(), sk=torch.from_numpy(sk).cuda())
    reqs = sv.build_requests(240, lam=20000.0, keys_per_level={2: 6, 3: 5, 5: 4}, seed=11)
    reqs.level = np.where(reqs.level == 3, 65, np.where(reqs.level == 5, 87, reqs.level)).astype(np.int8)
    flipped = sv.attach_signatures(reqs, ctx, keysets, flip_rate=0.1, seed=11)
    cls = sv.Server if engine == "python" else sv.NativeServer
    server = cls(keysets, n_streams=3, max_batch=64, mem_budget=2 << 30, max_msg_bytes=1 << 20)
    res = server.serve(reqs)
    server.close()
    assert np.isfinite(res.t_done).all()
    _check_against_oracle(sv, host, reqs, flipped, res)
    for ks in keysets.values():
        ks.close()
    ctx.close()


def test_native_server_rejects_duplicate_levels(setup):
    dl, sv, ctx, keysets, host, reqs, flipped = setup
    import ctypes
    lib = dl.load()
    h = ctypes.c_void_p()
    tables = (ctypes.c_void_p * 2)(keysets[2].h.value, keysets[2].h.value)
    rc = lib.dil_server_create_tables(ctypes.byref(h), 0, ctypes.cast(tables, ctypes.c_void_p), 2, 2, 64,
                                      1 << 20, 2 << 30, dl.MODE_PERSISTENT)
    assert rc == dl.DIL_EINVAL and not h.value


def test_native_service_modes_and_errors():
    """The C entry points of the interactive mode directly: a trace replay is refused while the
    mode is on; poll reports an unfinished request and hands a result out once; wait with a
    zero timeout returns a finished result; unknown tickets, bad rows and a stopped mode are
    refused; stop finishes what was submitted, and the engine then replays a trace again."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import ctypes
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd import serving as sv
    ctx = dl.Context(0, mode=dl.MODE_PERSISTENT)
    pk, sk = oracle.keygen_batch(2, workload.keygen_seeds(3, seed=340))
    ks = dl.KeySet(ctx, 2, pk=torch.from_numpy(pk).cuda(), sk=torch.from_numpy(sk).cuda())
    server = sv.NativeServer({2: ks}, n_streams=2, max_batch=16, mem_budget=2 << 30, max_msg_bytes=1 << 16)
    lib, h = server.lib, server.h
    c = ctypes
    msgs = [workload.random_bytes("test/native-service", i, (17 * i,)).tobytes() for i in range(12)]
    assert lib.dil_server_start(h) == dl.DIL_OK
    assert lib.dil_server_start(h) == dl.DIL_EINVAL            # already on
    one = sv.Requests(np.zeros(1), np.array([sv.SIGN], np.int8), np.array([2], np.int8), np.array([0], np.int32),
                      np.frombuffer(msgs[1], np.uint8).copy(), np.array([0, len(msgs[1])], np.int64))
    with pytest.raises(dl.DilError):
        server.serve(one)                                      # replay refused while the mode is on
    t = c.c_uint64()
    tickets = []
    for i, m in enumerate(msgs):
        buf = c.create_string_buffer(m, max(len(m), 1))
        assert lib.dil_server_submit(h, sv.SIGN, 2, i % 3, c.cast(buf, c.c_void_p), len(m), None, c.byref(t)) == 0
        tickets.append(t.value)
    bad = c.create_string_buffer(b"x", 1)
    assert lib.dil_server_submit(h, sv.SIGN, 2, 3, c.cast(bad, c.c_void_p), 1, None, c.byref(t)) == dl.DIL_EINVAL
    assert lib.dil_server_submit(h, sv.VERIFY, 2, 0, c.cast(bad, c.c_void_p), 1, None, c.byref(t)) == dl.DIL_EINVAL
    assert lib.dil_server_submit(h, sv.SIGN, 3, 0, c.cast(bad, c.c_void_p), 1, None, c.byref(t)) == dl.DIL_EINVAL
    done, verdict = c.c_int(), c.c_int32()
    assert lib.dil_server_poll(h, 10 ** 9, c.byref(done), c.byref(verdict), None) == dl.DIL_EINVAL
    sbuf = c.create_string_buffer(dl.sizes(2)[2])
    got = {}
    for k, tk in enumerate(tickets):
        if k % 2:
            assert lib.dil_server_wait(h, tk, 60000, c.byref(verdict), c.cast(sbuf, c.c_void_p)) == dl.DIL_OK
        else:
            while True:
                assert lib.dil_server_poll(h, tk, c.byref(done), c.byref(verdict), c.cast(sbuf, c.c_void_p)) == 0
                if done.value:
                    break
        assert verdict.value == -1
        got[k] = sbuf.raw
        # handed out once
        assert lib.dil_server_poll(h, tk, c.byref(done), c.byref(verdict), None) == dl.DIL_EINVAL
    for k, m in enumerate(msgs):
        assert got[k] == oracle.sign(2, sk[k % 3].tobytes(), m)[0]
    # requests left to stop: it finishes them, and their results stay available
    last = []
    for i in range(5):
        buf = c.create_string_buffer(msgs[i], max(len(msgs[i]), 1))
        assert lib.dil_server_submit(h, sv.SIGN, 2, 1, c.cast(buf, c.c_void_p), len(msgs[i]), None, c.byref(t)) == 0
        last.append(t.value)
    assert lib.dil_server_stop(h) == dl.DIL_OK
    assert lib.dil_server_stop(h) == dl.DIL_EINVAL             # not on
    assert lib.dil_server_submit(h, sv.SIGN, 2, 0, c.cast(bad, c.c_void_p), 1, None, c.byref(t)) == dl.DIL_EINVAL
    for i, tk in enumerate(last):
        assert lib.dil_server_wait(h, tk, 0, c.byref(verdict), c.cast(sbuf, c.c_void_p)) == dl.DIL_OK
        assert sbuf.raw == oracle.sign(2, sk[1].tobytes(), msgs[i])[0]
    res = server.serve(one)                                    # replay works again
    assert bytes(res.sig[0]) == oracle.sign(2, sk[0].tobytes(), msgs[1])[0]
    server.close()
    ks.close()
    ctx.close()


@pytest.mark.parametrize("engine", ["native"])
def test_large_batches_match_oracle(setup, engine):
    """Batches of up to 2,048 requests, all arriving at once: the native engine stages a batch
    of several MB (messages and verify signatures in, signatures out) on several host threads,
    and every output still equals the oracle's."""
    dl, sv, ctx, keysets, host, reqs, flipped = setup
    keys = {lv: ks.n_keys for lv, ks in keysets.items()}
    big = sv.build_requests(1500, lam=0.0, keys_per_level=keys, seed=17)
    big_flipped = sv.attach_signatures(big, ctx, keysets, flip_rate=0.1, seed=17)
    server = sv.NativeServer(keysets, n_streams=2, max_batch=2048, mem_budget=16 << 30, max_msg_bytes=64 << 20)
    res = server.serve(big)
    server.close()
    assert res.batches <= 3
    _check_against_oracle(sv, host, big, big_flipped, res)


def test_native_engine_mldsa_internal_mode():
    """DIL_SERVER_MLDSA_INTERNAL: the native engine's ML-DSA groups take formatted messages M'
    (context strings here) while round-3 requests stay plain: every signature and verdict equals
    the oracle's internal (ML-DSA) or plain (level 2) output.  Unknown mode bits are refused."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import ctypes
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd import serving as sv
    ctx = dl.Context(0, mode=dl.MODE_PERSISTENT)
    keys = {2: 5, 65: 4, 87: 3}
    keysets, host = {}, {}
    for lv, nk in keys.items():
        pk, sk = oracle.keygen_batch(lv, workload.keygen_seeds(nk, seed=360 + lv))
        host[lv] = (pk, sk)
        keysets[lv] = dl.KeySet(ctx, lv, pk=torch.from_numpy(pk).cuda(), sk=torch.from_numpy(sk).cuda())
    lib = dl.load()
    h = ctypes.c_void_p()
    tables = (ctypes.c_void_p * 3)(*[keysets[lv].h.value for lv in sorted(keysets)])
    assert lib.dil_server_create_tables(ctypes.byref(h), 0, ctypes.cast(tables, ctypes.c_void_p), 3, 2, 64,
                                        1 << 20, 2 << 30, dl.MODE_PERSISTENT | 0x200) == dl.DIL_EINVAL
    rng = np.random.default_rng(41)
    n = 90
    level = rng.choice([2, 65, 87], size=n)
    op = (rng.random(n) < 0.5).astype(int)
    key = np.array([rng.integers(0, keys[int(lv)]) for lv in level])
    reqs, expect = [], []
    for i in range(n):
        lv = int(level[i])
        pk, sk = host[lv]
        m = workload.random_bytes("test/serve-internal", i, (int(rng.integers(0, 300)),)).tobytes()
        if lv != 2:
            m = oracle.mldsa_format(m, b"ctx-%d" % (i % 7))
            s = oracle.mldsa_sign_internal(lv, sk[key[i]].tobytes(), m)
        else:
            s = oracle.sign(lv, sk[key[i]].tobytes(), m)[0]
        if op[i] == sv.SIGN:
            reqs.append((lv, sv.SIGN, int(key[i]), m, None))
            expect.append(s)
        else:
            if i % 3 == 0:
                b = bytearray(s)
                b[i % len(b)] ^= 4
                s = bytes(b)
            reqs.append((lv, sv.VERIFY, int(key[i]), m, s))
            ok = oracle.mldsa_verify_internal(lv, pk[key[i]].tobytes(), m, s) if lv != 2 else \
                oracle.verify(lv, pk[key[i]].tobytes(), m, s)
            expect.append(bool(ok == 1))
    svc = sv.NativeService(keysets, n_streams=2, max_batch=32, mem_budget=2 << 30, max_msg_bytes=1 << 20,
                           mldsa_internal=True)
    tickets = [svc.submit(*r) for r in reqs]
    got = [svc.wait(t, timeout=120) for t in tickets]
    svc.close()
    assert got == expect
    for ks in keysets.values():
        ks.close()
    ctx.close()
