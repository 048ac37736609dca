"""The entry point that allocates nothing (dabs_mlp_pool_features_noalloc)
against the allocating dabs_mlp_pool_features, bit for bit, on two calls in a
row on the same GPU (the second smaller, so stale counts of the first call
would show), and against the oracle's features."""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2207_03069_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2207_03069_amd as dabs  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def features(fn, p, pools):
    P, m, n = pools.shape
    feat = torch.zeros((P, m, n, 8), dtype=torch.int16, device=DEV)
    fn(p, dev(inputs.pack_bits(pools.reshape(P * m, n)).view(np.int64)), P, m, feat)
    torch.cuda.synchronize()
    return feat.cpu().numpy().view(np.uint16)


def test_noalloc_features_match_allocating_call_twice():
    rng = np.random.default_rng(5)
    cases = [(700, np.int16, 3, 6), (130, np.int32, 2, 4)]     # second call smaller
    for n, wt, P, m in cases:
        print("no-alloc features: n=%d %s P=%d m=%d" % (n, np.dtype(wt).name, P, m), flush=True)
        W = inputs.dense_qubo(n, -300, 300, 11 + n, dtype=wt)
        p = dabs.dabs_problem_create(dev(W))
        pools = rng.integers(0, 2, (P, m, n)).astype(np.uint8)
        got = features(dabs.dabs_mlp_pool_features_noalloc, p, pools)
        ref = features(dabs.dabs_mlp_pool_features, p, pools)
        assert np.array_equal(got, ref)
        for q in range(P):
            for r in (0, m - 1):
                assert np.array_equal(got[q, r], omlp.bf16_bits(omlp.features(W, pools[q, r], pools[q], r)))
        dabs.dabs_problem_destroy(p)


def test_noalloc_features_reject_oversize_shape():
    n = 4096
    W = inputs.dense_qubo(n, -10, 10, 3)
    p = dabs.dabs_problem_create(dev(W))
    P = dabs.DABS_NOALLOC_COUNTS // n + 1
    bits = torch.zeros((P, (n + 63) // 64), dtype=torch.int64, device=DEV)
    feat = torch.zeros((P, 1, n, 8), dtype=torch.int16, device=DEV)
    with pytest.raises(dabs.DabsError) as e:
        dabs.dabs_mlp_pool_features_noalloc(p, bits, P, 1, feat)
    assert e.value.status == dabs.DABS_E_INVALID
    dabs.dabs_problem_destroy(p)
