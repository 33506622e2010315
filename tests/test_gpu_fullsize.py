"""Full-size parity: 10,000-task batches in the launch configurations the benchmark times
(persistent Sign with the schedule the autotuner recorded for that workload, and with
automatic schedules of one and four wavefronts per workgroup): every key and every
signature of the batch equals the multi-threaded oracle's, plus properties that hold at
any size (every signature verifies on the GPU, every level-2 flipped signature is
rejected)."""
import functools

import numpy as np
import pytest

import oracle
from paper_2211_12265_amd import workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@functools.lru_cache(maxsize=4)
def _oracle_batch(level: int, n: int, lengths: str):
    """The oracle's keys and signatures for the whole batch (all host threads), shared by the
    parametrizations that run the same batch."""
    seeds = workload.keygen_seeds(n, seed=level)
    lens = workload.fixed_lengths(n, 32) if lengths == "fixed32" else workload.uniform_lengths(n, 32, 4096, seed=level)
    msg, off = workload.messages(lens, seed=level)
    opk, osk = oracle.keygen_batch(level, seeds)
    osig, _ = oracle.sign_batch(level, osk, msg, off)
    return seeds, lens, msg, off, opk, osk, osig


@pytest.mark.parametrize("level,lengths,waves", [(2, "fixed32", 1), (2, "fixed32", 4), (2, "fixed32", "recorded"),
                                                 (3, "uniform", 1), (3, "uniform", "recorded"),
                                                 (5, "uniform", 4), (5, "uniform", "recorded")])
def test_ten_thousand_tasks(level, lengths, waves):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import autotune
    from paper_2211_12265_amd import dilithium as dl
    n = 10000
    ctx = dl.Context(0, mode=dl.MODE_PERSISTENT)
    if waves == "recorded":
        sched = autotune.cached_schedule(level, n, lengths)
        assert sched is not None, "no recorded schedule for the benchmark workload"
        autotune.apply_schedule(ctx, sched)
        ctx.set_param("graph", 1)
    else:
        ctx.set_param("persist.waves", waves)
    pkl, skl, sgl = dl.sizes(level)
    seeds, lens, msg, off, opk, osk, osig = _oracle_batch(level, n, lengths)
    pk = torch.zeros((n, pkl), dtype=torch.uint8, device="cuda")
    sk = torch.zeros((n, skl), dtype=torch.uint8, device="cuda")
    ctx.keygen(level, torch.from_numpy(seeds).cuda(), pk, sk)
    gm, go = torch.from_numpy(msg).cuda(), torch.from_numpy(off.astype(np.int64)).cuda()
    sig = torch.zeros((n, sgl), dtype=torch.uint8, device="cuda")
    ctx.sign(level, sk, gm, go, sig)
    ver = torch.zeros(n, dtype=torch.int32, device="cuda")
    ctx.verify(level, pk, gm, go, sig, ver)
    torch.cuda.synchronize()
    assert int(ver.sum()) == n
    ev, seq = ctx.sign_stats()
    assert ev >= seq >= n
    pk_h, sk_h, sig_h = pk.cpu().numpy(), sk.cpu().numpy(), sig.cpu().numpy()
    assert np.array_equal(pk_h, opk) and np.array_equal(sk_h, osk)
    assert np.array_equal(sig_h, osig), f"{int((sig_h != osig).any(axis=1).sum())} of {n} signatures differ"
    if level == 2:
        bad = sig_h.copy()
        rows = np.arange(n)
        bit = np.random.default_rng(9).integers(0, sgl * 8, size=n)
        bad[rows, bit // 8] ^= (1 << (bit % 8)).astype(np.uint8)
        ctx.verify(level, pk, gm, go, torch.from_numpy(bad).cuda(), ver)
        torch.cuda.synchronize()
        assert int(ver.sum()) == 0
    ctx.close()


@pytest.mark.parametrize("level", [2, 5])
def test_ten_thousand_tasks_randomized(level):
    """Randomized Sign (caller-supplied rho' per task) at the benchmark's size and recorded
    schedule: all signatures equal the oracle's for the same rho', and every signature
    verifies on the GPU."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import autotune
    from paper_2211_12265_amd import dilithium as dl
    n = 10000
    lengths = "fixed32" if level == 2 else "uniform"
    ctx = dl.Context(0, mode=dl.MODE_PERSISTENT)
    autotune.apply_schedule(ctx, autotune.cached_schedule(level, n, lengths))
    pkl, skl, sgl = dl.sizes(level)
    seeds = workload.keygen_seeds(n, seed=300 + level)
    pk = torch.zeros((n, pkl), dtype=torch.uint8, device="cuda")
    sk = torch.zeros((n, skl), dtype=torch.uint8, device="cuda")
    ctx.keygen(level, torch.from_numpy(seeds).cuda(), pk, sk)
    lens = workload.fixed_lengths(n, 32) if lengths == "fixed32" else workload.uniform_lengths(n, 32, 4096, seed=301)
    msg, off = workload.messages(lens, seed=301)
    rnd = workload.random_bytes("test/rnd", 300 + level, (n, 64))
    gm, go = torch.from_numpy(msg).cuda(), torch.from_numpy(off.astype(np.int64)).cuda()
    sig = torch.zeros((n, sgl), dtype=torch.uint8, device="cuda")
    ctx.sign(level, sk, gm, go, sig, rnd=torch.from_numpy(rnd).cuda())
    ver = torch.zeros(n, dtype=torch.int32, device="cuda")
    ctx.verify(level, pk, gm, go, sig, ver)
    torch.cuda.synchronize()
    assert int(ver.sum()) == n
    osig, _ = oracle.sign_batch(level, sk.cpu().numpy(), msg, off, rnd=rnd)
    assert np.array_equal(sig.cpu().numpy(), osig)
    ctx.close()


@pytest.mark.parametrize("mode", ["staged", "persistent"])
@pytest.mark.parametrize("level", [2, 3, 5])
def test_single_task(mode, level):
    """count = 1 in every execution form (a persistent launch with one workgroup holding one task)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import dilithium as dl
    ctx = dl.Context(0, mode=dl.MODE_STAGED if mode == "staged" else dl.MODE_PERSISTENT)
    seeds = workload.keygen_seeds(1, seed=170 + level)
    opk, osk = oracle.keygen_batch(level, seeds)
    msg, off = workload.messages(workload.fixed_lengths(1, 77), seed=171)
    osig, _ = oracle.sign_batch(level, osk, msg, off)
    sig = torch.zeros((1, dl.sizes(level)[2]), dtype=torch.uint8, device="cuda")
    gm, go = torch.from_numpy(msg).cuda(), torch.from_numpy(off.astype(np.int64)).cuda()
    ctx.sign(level, torch.from_numpy(osk).cuda(), gm, go, sig)
    v = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.verify(level, torch.from_numpy(opk).cuda(), gm, go, sig, v)
    torch.cuda.synchronize()
    assert np.array_equal(sig.cpu().numpy(), osig) and int(v.item()) == 1
    ctx.close()


@pytest.mark.parametrize("level", [3, 44, 87])
def test_long_messages(level):
    """64 KiB messages (482 SHAKE256 blocks for mu) next to empty ones, at level 3 and at two
    ML-DSA levels (66-byte mu prefix)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import dilithium as dl
    ctx = dl.Context(0, mode=dl.MODE_PERSISTENT)
    seeds = workload.keygen_seeds(4, seed=180)
    opk, osk = oracle.keygen_batch(level, seeds)
    lens = np.array([65536, 0, 65535, 1], dtype=np.int64)
    msg, off = workload.messages(lens, seed=181)
    osig, _ = oracle.sign_batch(level, osk, msg, off)
    sig = torch.zeros((4, dl.sizes(level)[2]), dtype=torch.uint8, device="cuda")
    gm, go = torch.from_numpy(msg).cuda(), torch.from_numpy(off.astype(np.int64)).cuda()
    ctx.sign(level, torch.from_numpy(osk).cuda(), gm, go, sig)
    v = torch.zeros(4, dtype=torch.int32, device="cuda")
    ctx.verify(level, torch.from_numpy(opk).cuda(), gm, go, sig, v)
    torch.cuda.synchronize()
    assert np.array_equal(sig.cpu().numpy(), osig)
    assert v.cpu().tolist() == [1, 1, 1, 1]
    ctx.close()


def test_hundred_thousand_tasks():
    """A batch ten times the benchmark's (workspace growth, queue and grid limits): all keys
    and signatures equal the oracle's and every signature verifies."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import dilithium as dl
    level, n = 2, 100000
    ctx = dl.Context(0, mode=dl.MODE_PERSISTENT)
    pkl, skl, sgl = dl.sizes(level)
    seeds = workload.keygen_seeds(n, seed=190)
    pk = torch.zeros((n, pkl), dtype=torch.uint8, device="cuda")
    sk = torch.zeros((n, skl), dtype=torch.uint8, device="cuda")
    ctx.keygen(level, torch.from_numpy(seeds).cuda(), pk, sk)
    lens = workload.fixed_lengths(n, 32)
    msg, off = workload.messages(lens, seed=190)
    gm, go = torch.from_numpy(msg).cuda(), torch.from_numpy(off.astype(np.int64)).cuda()
    sig = torch.zeros((n, sgl), dtype=torch.uint8, device="cuda")
    ctx.sign(level, sk, gm, go, sig)
    v = torch.zeros(n, dtype=torch.int32, device="cuda")
    ctx.verify(level, pk, gm, go, sig, v)
    torch.cuda.synchronize()
    assert int(v.sum()) == n
    opk, osk = oracle.keygen_batch(level, seeds)
    assert np.array_equal(sk.cpu().numpy(), osk) and np.array_equal(pk.cpu().numpy(), opk)
    osig, _ = oracle.sign_batch(level, osk, msg, off)
    assert np.array_equal(sig.cpu().numpy(), osig)
    ctx.close()
