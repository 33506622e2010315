"""End-to-end host path (pinned host buffers, chunked over several streams):
its signatures and verdicts equal the oracle's and the device-resident batch path's."""
import numpy as np
import pytest

import oracle
from paper_2211_12265_amd import workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("level,n_streams,chunk,threads", [(2, 3, 17, False), (3, 1, 64, False), (5, 4, 9, False),
                                                           (2, 3, 17, True), (5, 4, 9, True)])
def test_host_pipeline_matches_oracle(level, n_streams, chunk, threads):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd.pipeline import HostPipeline, pinned
    n = 61   # ragged last chunk for every chunk size above
    seeds = workload.keygen_seeds(n, seed=140 + level)
    opk, osk = oracle.keygen_batch(level, seeds)
    lens = workload.uniform_lengths(n, 0, 700, seed=141)
    lens[5] = 0
    msg, off = workload.messages(lens, seed=141)
    osig, _ = oracle.sign_batch(level, osk, msg, off)
    pkl, skl, sgl = dl.sizes(level)
    h_sk, h_pk = pinned((n, skl)), pinned((n, pkl))
    h_sk.numpy()[:] = osk
    h_pk.numpy()[:] = opk
    h_msg = pinned((max(len(msg), 1),))
    h_msg.numpy()[:len(msg)] = msg
    h_sig = pinned((n, sgl))
    h_ver = pinned((n,), torch.int32)
    p = HostPipeline(level, n_streams=n_streams, chunk=chunk, host_threads=threads)
    p.sign(h_sk, h_msg, off, h_sig)
    torch.cuda.synchronize()
    p.check()
    assert np.array_equal(h_sig.numpy(), osig)
    bad = osig.copy()
    bad[7, 40] ^= 4
    h_bad = pinned((n, sgl))
    h_bad.numpy()[:] = bad
    p.verify(h_pk, h_msg, off, h_sig, h_ver)
    torch.cuda.synchronize()
    assert h_ver.numpy().tolist() == [1] * n
    p.verify(h_pk, h_msg, off, h_bad, h_ver)
    torch.cuda.synchronize()
    exp = [1] * n
    exp[7] = 0
    assert h_ver.numpy().tolist() == exp
    # second batch through the same pipeline (buffers and plans reused or rebuilt)
    p.sign(h_sk, h_msg, off, h_sig)
    torch.cuda.synchronize()
    assert np.array_equal(h_sig.numpy(), osig)
    p.close()
