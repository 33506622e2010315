"""The two primitive workloads at full size (2^20 polynomials each), in the launch
configuration `bench.py --micro` times: c = INTT(NTT(a) o b) and ExpandA from 34-byte
inputs.  Sampled rows are compared with the oracle's row by row; every row is checked to
be canonical; the ablation forms of the NTT primitive must return the production
kernel's words exactly, over the whole batch."""
import numpy as np
import pytest

import oracle
from paper_2211_12265_amd import workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FULL = 1 << 20


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12265_amd import dilithium as dl
    c = dl.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ntt_inputs(ctx):
    a = workload.uniform_polys(FULL, seed=0)
    b = workload.uniform_polys(FULL, seed=0, tag="dil/poly2")
    ga, gb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    prod = torch.empty((FULL, 256), dtype=torch.int32, device="cuda")
    ctx.set_param("ntt.variant", 0)
    ctx.ntt_mul(ga, gb, prod)
    torch.cuda.synchronize()
    return a, b, ga, gb, prod


def sample_rows(n, k, seed):
    idx = np.random.default_rng(seed).choice(n, size=k, replace=False)
    return np.unique(np.concatenate([idx, [0, n - 1]]))


def test_ntt_mul_full_size(ntt_inputs):
    a, b, _, _, prod = ntt_inputs
    q = oracle.Q
    assert bool(((prod >= 0) & (prod < q)).all().item())
    idx = sample_rows(FULL, 4096, 11)
    got = prod[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert np.array_equal(got, oracle.ntt_mul_batch(a[idx], b[idx]))


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_ntt_ablation_forms_full_size(ctx, ntt_inputs, variant):
    _, _, ga, gb, prod = ntt_inputs
    c = torch.full((FULL, 256), -1, dtype=torch.int32, device="cuda")
    ctx.set_param("ntt.variant", variant)
    try:
        ctx.ntt_mul(ga, gb, c)
        torch.cuda.synchronize()
    finally:
        ctx.set_param("ntt.variant", 0)
    assert torch.equal(c, prod)


def test_expand_a_full_size(ctx):
    seeds = workload.expand_a_inputs(FULL, seed=0)
    out = torch.full((FULL, 256), -1, dtype=torch.int32, device="cuda")
    ctx.expand_a(torch.from_numpy(seeds).cuda(), out)
    torch.cuda.synchronize()
    assert bool(((out >= 0) & (out < oracle.Q)).all().item())
    idx = sample_rows(FULL, 4096, 12)
    got = out[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert np.array_equal(got, oracle.expand_a_polys(seeds[idx]))
