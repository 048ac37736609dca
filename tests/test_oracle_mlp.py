"""Pins of the learned-proposal oracle (oracle/mlp.py) against things other
than itself: torch's bfloat16 conversion, central finite differences of the
loss, torch's Adam, energies from scratch, and closed forms."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2207_03069_amd import inputs

torch = pytest.importorskip("torch")


def test_bf16_matches_torch_round_to_nearest_even():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(20000).astype(np.float32) * np.float32(10) ** rng.integers(-6, 6, 20000)
    # exact ties: low 16 bits = 0x8000, both parities of the kept LSB
    ties = (rng.integers(0, 1 << 15, 4000, dtype=np.uint32) << 17 | np.uint32(0x8000)
            | (rng.integers(0, 2, 4000, dtype=np.uint32) << 16)) & np.uint32(0x3FFFFFFF)
    x = np.concatenate([x, ties.view(np.float32), -ties.view(np.float32), [0.0, -0.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16(x).view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(mlp.from_bf16_bits(mlp.bf16_bits(x)).view(np.uint32), ref.view(np.uint32))


def _case(N=40, seed=1):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed) + rng.normal(0, 0.05, mlp.N_PARAMS).astype(np.float32)
    F = rng.normal(0, 1, (N, mlp.N_FEAT))
    y = rng.integers(0, 2, N).astype(np.float64)
    return p.astype(np.float64), F, y


def test_gradient_matches_central_differences():
    p, F, y = _case()
    g = mlp.grad(p, F, y, rounding=False)
    h = 1e-6
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 300, replace=False),
                          [mlp.OFF_B1, mlp.OFF_B2, mlp.OFF_W3, mlp.OFF_B3, mlp.OFF_W1 + 7, mlp.OFF_W2 + 4095]])
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        num = (mlp.loss(p + e, F, y, rounding=False) - mlp.loss(p - e, F, y, rounding=False)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * (1 + abs(g[i])), (i, num, g[i])


def test_loss_closed_forms():
    # zero network: z = b3 = 0 for every sample, loss = log 2, dL/db3 = mean(1/2 - y)
    p = np.zeros(mlp.N_PARAMS)
    F = np.random.default_rng(3).normal(size=(10, 8))
    y = np.array([1, 0, 1, 1, 0, 0, 0, 1, 1, 1], dtype=np.float64)
    assert mlp.loss(p, F, y, rounding=False) == pytest.approx(np.log(2.0))
    g = mlp.grad(p, F, y, rounding=False)
    assert g[mlp.OFF_B3] == pytest.approx(np.mean(0.5 - y))
    assert np.all(g[:mlp.OFF_B3] == 0)


def test_forward_routes_each_feature():
    """W1 picks feature i into hidden unit i, W2 passes unit i, W3 reads unit j:
    the logit is ReLU(f_j) for the routed feature (a transposed or shifted
    weight matrix would read another feature)."""
    for j in range(8):
        d = dict(W1=np.zeros((64, 8)), b1=np.zeros(64), W2=np.zeros((64, 64)), b2=np.zeros(64),
                 W3=np.zeros(64), b3=np.zeros(1))
        for i in range(8):
            d["W1"][i, i] = 1.0
            d["W2"][10 + i, i] = 1.0
        d["W3"][10 + j] = 1.0
        F = np.random.default_rng(j).normal(size=(30, 8))
        z = mlp.forward(mlp.pack(d), F, rounding=False)
        assert np.allclose(z, np.maximum(F[:, j], 0))


def test_rounded_gradient_close_to_exact():
    p, F, y = _case(200, 5)
    g0 = mlp.grad(p, F, y, rounding=False)
    g1 = mlp.grad(p, F, y, rounding=True)
    assert np.linalg.norm(g1 - g0) <= 0.02 * np.linalg.norm(g0)


def test_adam_matches_torch():
    rng = np.random.default_rng(7)
    p0 = rng.normal(size=mlp.N_PARAMS)
    t = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=3e-3, betas=(mlp.ADAM_B1, mlp.ADAM_B2), eps=mlp.ADAM_EPS)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for step in range(1, 6):
        g = rng.normal(size=mlp.N_PARAMS) * 10.0 ** (-step)
        opt.zero_grad()
        t.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = mlp.adam(p, g, m, v, step, 3e-3)
        assert np.allclose(p, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_features_by_definition():
    W = inputs.dense_qubo(40, -50, 50, 11)
    n = 40
    rng = np.random.default_rng(1)
    pool = rng.integers(0, 2, (7, n)).astype(np.uint8)
    X = pool[3]
    F = mlp.features(W, X, pool, 3)
    e0 = oracle.energy(W, X)
    B = oracle.delta_bound(W)
    assert mlp.row_abs(W).max() == B
    for k in range(n):
        Y = X.copy()
        Y[k] ^= 1
        d = oracle.energy(W, Y) - e0                      # Delta_k from scratch energies
        xk, bk, wkk = int(X[k]), int(pool[0, k]), int(W[k, k])
        rk = abs(wkk) + 2 * (int(np.abs(W[k].astype(np.int64)).sum()) - abs(wkk))
        pk = pool[:, k].astype(np.float64).mean()
        exp = [d / B, 2 * xk - 1, wkk / B, rk / B, 2 * pk - 1, (2 * xk - 1) * (2 * pk - 1), 2 * bk - 1, 3 / 7]
        # every feature within bfloat16 rounding (2^-8 relative) of its exact value
        assert np.allclose(F[k], exp, rtol=2 ** -8, atol=1e-12), (k, F[k], exp)
    assert F.dtype == np.float32 and np.array_equal(mlp.bf16(F), F)


def test_operations():
    rng = np.random.default_rng(4)
    n = 600
    parent = rng.integers(0, 2, n).astype(np.uint8)
    z = rng.normal(size=n).astype(np.float32)
    z[:5] = [0.0, -0.0, 1e-30, -1e-30, 3.0]
    t = mlp.mlp_seed(parent, z)
    assert np.array_equal(t ^ parent, (z > 0).astype(np.uint8))
    assert list((t ^ parent)[:5]) == [0, 0, 1, 0, 1]
    # q = -128 never flips; q = 0 flips at the Mutation rate 1/8; q = 127 at ~1/4
    for zval, rate in ((-100.0, 0.0), (0.0, 1 / 8), (100.0, (1 + 127 / 128) / 8)):
        flips = np.mean([np.mean(mlp.mlp_mutate(parent, np.full(n, zval, np.float32), 9, r, 3) ^ parent)
                         for r in range(8)])
        assert abs(flips - rate) < 0.02, (zval, flips, rate)
    assert list(mlp.mutate_level(np.array([0.03125, 0.09375, -0.03125, 8.1, -9.0], np.float32))) == [0, 2, 0, 127, -128]


def test_labels_symmetric_closed_forms():
    ref = np.array([1, 0, 1, 1, 0, 0, 1, 0], np.uint8)
    assert list(mlp.labels(ref, ref)) == [0] * 8
    assert list(mlp.labels(1 - ref, ref)) == [1] * 8
    assert list(mlp.labels(1 - ref, ref, symmetric=True)) == [0] * 8      # the complement is the same cut
    x = ref.copy(); x[:4] ^= 1                                            # distance 4 = n/2: ties keep ref
    assert list(mlp.labels(x, ref, symmetric=True)) == [1, 1, 1, 1, 0, 0, 0, 0]
    x[4] ^= 1                                                             # distance 5 > n/2: complement
    assert list(mlp.labels(x, ref, symmetric=True)) == [0, 0, 0, 0, 0, 1, 1, 1]
