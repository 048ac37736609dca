"""GPU parity of the learned proposal against oracle/mlp.py: features and
labels bit for bit, the MLP operations bit for bit on the same logits, the
forward pass and the gradient within float32-accumulation tolerance (the
bfloat16 roundings are at the same points on both sides), training steps,
and the solver with the learned operations attached (exact energies, pool
invariants; with the learned operations disabled, bit-exact with the
oracle)."""
import numpy as np
import pytest

import oracle
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


def packed(bits):
    return dev(inputs.pack_bits(bits).view(np.int64))


def bf16_feats(rng, N):
    return omlp.bf16(rng.normal(0, 1, (N, 8)).astype(np.float32))


def to_dev_bf16(F):
    return dev(omlp.bf16_bits(F).view(np.int16))


@pytest.mark.parametrize("n,wt,P,m", [(300, np.int16, 2, 5), (70, np.int32, 3, 4), (1, np.int16, 1, 3),
                                      (129, np.int16, 2, 7)])
def test_features_bit_exact(n, wt, P, m):
    W = inputs.dense_qubo(n, -300, 300, 40 + n, dtype=wt)
    p = dabs.dabs_problem_create(dev(W))
    rng = np.random.default_rng(n)
    pools = rng.integers(0, 2, (P, m, n)).astype(np.uint8)
    feat = torch.zeros((P, m, n, 8), dtype=torch.int16, device=DEV)
    dabs.dabs_mlp_pool_features(p, packed(pools.reshape(P * m, n)), P, m, feat)
    torch.cuda.synchronize()
    got = feat.cpu().numpy().view(np.uint16)
    for q in range(P):
        for r in range(m):
            exp = omlp.bf16_bits(omlp.features(W, pools[q, r], pools[q], r))
            assert np.array_equal(got[q, r], exp), (q, r)


@pytest.mark.parametrize("n", [130, 64, 1])
def test_labels_bit_exact(n):
    W = inputs.dense_qubo(n, -5, 5, 1)
    p = dabs.dabs_problem_create(dev(W))
    rng = np.random.default_rng(n)
    ref = rng.integers(0, 2, n).astype(np.uint8)
    X = rng.integers(0, 2, (9, n)).astype(np.uint8)
    X[0] = ref
    X[1] = 1 - ref                                  # the complement
    X[2, : n // 8] = 1 - ref[: n // 8]              # near the reference
    X[2, n // 8:] = ref[n // 8:]
    for sym in (False, True):
        lab = torch.zeros((9, n), dtype=torch.uint8, device=DEV)
        dabs.dabs_mlp_labels(p, packed(X), 9, packed(ref[None])[0], lab, sym)
        torch.cuda.synchronize()
        exp = np.stack([omlp.labels(x, ref, sym) for x in X])
        assert np.array_equal(lab.cpu().numpy(), exp), sym


@pytest.mark.parametrize("op", [dabs.DABS_OP_MLP_SEED, dabs.DABS_OP_MLP_MUTATE])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 300, 2048])
def test_operations_bit_exact(op, n):
    rng = np.random.default_rng(n + op)
    cnt = 5
    parents = rng.integers(0, 2, (cnt, n)).astype(np.uint8)
    z = (rng.normal(0, 3, (cnt, n))).astype(np.float32)
    special = np.array([0.0, -0.0, 1e-30, -1e-30, 0.03125, 0.09375, -0.03125, -0.09375, 7.96875, -8.0, 100.0,
                        -100.0], np.float32)
    z.ravel()[:min(special.size, z.size)] = special[:min(special.size, z.size)]
    out = torch.zeros((cnt, (n + 63) // 64), dtype=torch.int64, device=DEV)
    seed, rnd, inst0 = 12345, 7, 30
    dabs.dabs_mlp_apply_op(op, n, cnt, packed(parents), dev(z), seed, rnd, inst0, out)
    torch.cuda.synchronize()
    got = inputs.unpack_bits(out.cpu().numpy().view(np.uint64), n)
    for i in range(cnt):
        exp = omlp.mlp_seed(parents[i], z[i]) if op == dabs.DABS_OP_MLP_SEED else \
            omlp.mlp_mutate(parents[i], z[i], seed, rnd, inst0 + i)
        assert np.array_equal(got[i], exp), i


def params_case(seed):
    rng = np.random.default_rng(seed)
    return (omlp.init_params(seed) + rng.normal(0, 0.1, omlp.N_PARAMS).astype(np.float32)).astype(np.float32)


def test_forward_routing_exact():
    """Weights that route feature j through one hidden unit of each layer:
    every product is exact, so the logit is ReLU(f_j) exactly (a wrong
    matrix-core operand layout reads another feature or sample)."""
    rng = np.random.default_rng(1)
    F = bf16_feats(rng, 77)
    for j in range(8):
        d = dict(W1=np.zeros((64, 8)), b1=np.zeros(64), W2=np.zeros((64, 64)), b2=np.zeros(64),
                 W3=np.zeros(64), b3=np.zeros(1))
        for i in range(8):
            d["W1"][3 + 7 * i, i] = 1.0
            d["W2"][60 - 5 * i, 3 + 7 * i] = 1.0
        d["W3"][60 - 5 * j] = 1.0
        net = dabs.dabs_mlp_create(omlp.pack(d).astype(np.float32))
        z = torch.zeros(77, dtype=torch.float32, device=DEV)
        dabs.dabs_mlp_forward(net, 77, to_dev_bf16(F), z)
        torch.cuda.synchronize()
        assert np.array_equal(z.cpu().numpy(), np.maximum(F[:, j], 0)), j


# float32 accumulation on the matrix cores vs float64 in the oracle: a
# pre-activation may round to the neighbouring bfloat16 value (2^-8 relative)
# on one side only; logits agree to about 1e-5 and never by more than 2e-2.
@pytest.mark.parametrize("N", [1, 16, 1000, 40003])
def test_forward_parity(N):
    rng = np.random.default_rng(N)
    F = bf16_feats(rng, N)
    prm = params_case(3)
    net = dabs.dabs_mlp_create(prm)
    z = torch.zeros(N, dtype=torch.float32, device=DEV)
    dabs.dabs_mlp_forward(net, N, to_dev_bf16(F), z)
    torch.cuda.synchronize()
    got = z.cpu().numpy().astype(np.float64)
    exp = omlp.forward(prm, F, rounding=True)
    err = np.abs(got - exp) / (1 + np.abs(exp))
    assert err.max() < 2e-2
    assert np.mean(err < 1e-4) > 0.99


@pytest.mark.parametrize("N", [5, 1000, 30011])
def test_gradient_parity(N):
    rng = np.random.default_rng(100 + N)
    F = bf16_feats(rng, N)
    y = (rng.random(N) < 0.3).astype(np.uint8)
    prm = params_case(4)
    net = dabs.dabs_mlp_create(prm)
    g = torch.zeros(omlp.N_PARAMS, dtype=torch.float32, device=DEV)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    dabs.dabs_mlp_grad(net, N, to_dev_bf16(F), dev(y), g, loss)
    torch.cuda.synchronize()
    gg = g.cpu().numpy().astype(np.float64)
    ge = omlp.grad(prm, F, y.astype(np.float64), rounding=True)
    assert np.linalg.norm(gg - ge) <= 1e-2 * np.linalg.norm(ge) + 1e-7
    assert float(loss.item()) == pytest.approx(omlp.loss(prm, F, y, rounding=True), rel=1e-4)
    # every block of parameters individually
    for a, b in ((omlp.OFF_W1, omlp.OFF_B1), (omlp.OFF_B1, omlp.OFF_W2), (omlp.OFF_W2, omlp.OFF_B2),
                 (omlp.OFF_B2, omlp.OFF_W3), (omlp.OFF_W3, omlp.OFF_B3), (omlp.OFF_B3, omlp.N_PARAMS)):
        assert np.linalg.norm(gg[a:b] - ge[a:b]) <= 2e-2 * np.linalg.norm(ge[a:b]) + 1e-7, (a, b)


def test_training_steps_follow_oracle():
    """Five Adam steps on the same minibatch: the losses follow the oracle's
    (its own gradients and Adam) and decrease."""
    rng = np.random.default_rng(9)
    N = 4096
    F = bf16_feats(rng, N)
    y = (F[:, 0] + 0.5 * F[:, 3] > 0.2).astype(np.uint8)        # a learnable rule
    prm = params_case(5)
    net = dabs.dabs_mlp_create(prm)
    Fd, yd = to_dev_bf16(F), dev(y)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    p, m, v = prm.astype(np.float64), np.zeros(omlp.N_PARAMS), np.zeros(omlp.N_PARAMS)
    got, exp = [], []
    for step in range(1, 6):
        dabs.dabs_mlp_train_step(net, N, Fd, yd, 3e-3, loss)
        torch.cuda.synchronize()
        got.append(float(loss.item()))
        exp.append(omlp.loss(p, F, y, rounding=True))
        p, m, v = omlp.adam(p, omlp.grad(p, F, y.astype(np.float64), rounding=True), m, v, step, 3e-3)
    assert np.allclose(got, exp, rtol=2e-3), (got, exp)
    out = torch.zeros(omlp.N_PARAMS, dtype=torch.float32, device=DEV)
    dabs.dabs_mlp_params(net, out)
    torch.cuda.synchronize()
    # Adam moves each parameter by at most ~lr per step
    assert np.max(np.abs(out.cpu().numpy() - p)) < 5 * 3e-3 * 2
    assert got[-1] < got[0]


def solver_with_mlp(W, ops, rounds, inst=16, P=2, m=8, seed=3):
    n = W.shape[0]
    g = dabs.ga_params(T=max(1, n // 8), Bn=2 * n, tau=8, seed=seed, capacity=m, npools=P, ops=ops,
                       greedy_cap=100000)
    p = dabs.dabs_problem_create(dev(W))
    s = dabs.dabs_solver_create(p, g, inst)
    net = dabs.dabs_mlp_create(params_case(6))
    dabs.dabs_solver_set_mlp(s, net)
    for _ in range(rounds):
        dabs.dabs_solver_run(s, 1)
    nw = (n + 63) // 64
    bits = torch.zeros((P, m, nw), dtype=torch.int64, device=DEV)
    pe = torch.zeros((P, m), dtype=torch.int64, device=DEV)
    po = torch.zeros((P, m), dtype=torch.int32, device=DEV)
    x = torch.zeros((inst, nw), dtype=torch.int64, device=DEV)
    e = torch.zeros(inst, dtype=torch.int64, device=DEV)
    dabs.dabs_solver_pools(s, bits, pe, None, po)
    dabs.dabs_solver_state(s, x, e)
    torch.cuda.synchronize()
    return (inputs.unpack_bits(bits.cpu().numpy().view(np.uint64), n), pe.cpu().numpy(), po.cpu().numpy(),
            inputs.unpack_bits(x.cpu().numpy().view(np.uint64), n), e.cpu().numpy(), g)


def test_solver_with_learned_operations_exact_energies():
    n = 90
    W = inputs.dense_qubo(n, -100, 100, 8)
    ops = tuple(range(10))
    bits, pe, po, x, e, _ = solver_with_mlp(W, ops, 4)
    P, m = pe.shape
    for q in range(P):
        assert np.all(pe[q][1:] >= pe[q][:-1])              # sorted (no subtraction: +inf is INT64_MAX)
        fin = pe[q] < np.iinfo(np.int64).max
        for r in np.nonzero(fin)[0]:
            assert oracle.energy(W, bits[q, r]) == pe[q, r]
        rows = {bits[q, r].tobytes() for r in np.nonzero(fin)[0]}
        assert len(rows) == int(fin.sum())                   # no duplicates
        assert np.all((po[q] >= 0) & (po[q] <= 9))
    for i in range(x.shape[0]):
        assert oracle.energy(W, x[i]) == e[i]


def exact_ga_network():
    """A network whose every product and sum is exact in bfloat16 / float32
    on pools of capacity 8:  z = |f1 - f6| + f4/4 + 3 f7/4 - 5/4.  The logit
    is positive where the bit differs from the pool's best entry, and also
    where it agrees but most of the pool has the bit set in a low-ranked
    entry, so both learned operations draw non-trivial targets, and both
    sides compute the same logits to the last bit."""
    d = dict(W1=np.zeros((64, 8)), b1=np.zeros(64), W2=np.zeros((64, 64)), b2=np.zeros(64),
             W3=np.zeros(64), b3=np.array([-1.25]))
    d["W1"][0, 1], d["W1"][0, 6] = 1.0, -1.0       # relu(f1 - f6)
    d["W1"][1, 1], d["W1"][1, 6] = -1.0, 1.0       # relu(f6 - f1)
    d["W1"][2, 4] = 1.0                            # relu(f4)
    d["W1"][3, 4] = -1.0                           # relu(-f4)
    d["W1"][4, 7] = 1.0                            # f7 >= 0
    for u in range(5):
        d["W2"][u, u] = 1.0
    d["W3"][:5] = [1.0, 1.0, 0.25, -0.25, 0.75]
    return omlp.pack(d).astype(np.float32)


@pytest.mark.parametrize("n,wt,ops", [(90, np.int16, tuple(range(10))), (70, np.int32, (8, 9, 2)),
                                      (130, np.int16, (8, 9)), (70, "wide", (8, 9, 2))])
def test_learned_ga_bit_exact_with_oracle(n, wt, ops):
    """The learned operations inside device rounds (pool scoring, parent
    logits, MLP-seed / MLP-mutate targets) against the oracle's generational
    loop with the same network: pools, states and energies bit for bit (also
    on the wide-delta kernels, with a delta bound near 2^31)."""
    if wt == "wide":
        W = inputs.wide_qubo(n, (1 << 31) - 1, 21 + n)
    else:
        W = inputs.dense_qubo(n, -100, 100, 21 + n, dtype=wt)
    params = exact_ga_network()
    inst, P, m, rounds, seed = 16, 2, 8, 4, 5
    g = dabs.ga_params(T=max(1, n // 8), Bn=2 * n, tau=8, seed=seed, capacity=m, npools=P, ops=ops,
                       greedy_cap=100000)
    p = dabs.dabs_problem_create(dev(W))
    assert dabs.dabs_problem_wide(p) == (wt == "wide")
    s = dabs.dabs_solver_create(p, g, inst)
    net = dabs.dabs_mlp_create(params)
    dabs.dabs_solver_set_mlp(s, net)
    dabs.dabs_solver_run(s, rounds)
    nw = (n + 63) // 64
    bits = torch.zeros((P, m, nw), dtype=torch.int64, device=DEV)
    pe = torch.zeros((P, m), dtype=torch.int64, device=DEV)
    po = torch.zeros((P, m), dtype=torch.int32, device=DEV)
    x = torch.zeros((inst, nw), dtype=torch.int64, device=DEV)
    e = torch.zeros(inst, dtype=torch.int64, device=DEV)
    dabs.dabs_solver_pools(s, bits, pe, None, po)
    dabs.dabs_solver_state(s, x, e)
    torch.cuda.synchronize()
    used = []

    def score(rnd, pool_bits):
        used.append(rnd)
        return omlp.pool_logits(params, W, pool_bits)

    ref = oracle.solve(W, oracle.ga_params(T=g.T, Bn=g.Bn, tau=8, seed=seed, capacity=m, npools=P, ops=ops,
                                           greedy_cap=100000), inst, rounds, score=score)
    assert used == list(range(rounds))
    assert np.array_equal(pe.cpu().numpy(), ref["pool_e"])
    assert np.array_equal(inputs.unpack_bits(bits.cpu().numpy().view(np.uint64), n), ref["pool_bits"])
    assert np.array_equal(po.cpu().numpy(), ref["pool_op"])
    assert np.array_equal(inputs.unpack_bits(x.cpu().numpy().view(np.uint64), n), ref["x"])
    assert np.array_equal(e.cpu().numpy(), ref["e"])
    # the learned operations produced pooled entries (not only initial columns)
    fin = ref["pool_e"] < np.iinfo(np.int64).max
    assert np.isin(ref["pool_op"][fin], (8, 9)).any()
    dabs.dabs_solver_destroy(s)
    dabs.dabs_mlp_destroy(net)
    dabs.dabs_problem_destroy(p)


def test_solver_with_network_attached_but_plain_operations_is_exact():
    """Attaching a network changes nothing while the learned operations are
    disabled: bit-exact with the oracle."""
    n = 70
    W = inputs.dense_qubo(n, -100, 100, 2)
    bits, pe, po, x, e, g = solver_with_mlp(W, tuple(range(8)), 3)
    ref = oracle.solve(W, oracle.ga_params(T=g.T, Bn=g.Bn, tau=8, seed=3, capacity=8, npools=2,
                                           greedy_cap=100000), 16, 3)
    assert np.array_equal(pe, ref["pool_e"]) and np.array_equal(bits, ref["pool_bits"])
    assert np.array_equal(x, ref["x"]) and np.array_equal(e, ref["e"])


def test_learned_operations_need_a_network():
    W = inputs.dense_qubo(20, -5, 5, 1)
    p = dabs.dabs_problem_create(dev(W))
    s = dabs.dabs_solver_create(p, dabs.ga_params(T=2, Bn=40, ops=(dabs.DABS_OP_MLP_SEED,)), 4)
    with pytest.raises(dabs.DabsError):
        dabs.dabs_solver_run(s, 1)


def test_training_on_plain_search_solutions_generalises():
    """The network trained on pool solutions of plain runs on one max-cut
    graph predicts the flips of pool solutions on another graph of the
    family better than the untrained network (held-out loss)."""
    from paper_2207_03069_amd import train
    n = 256

    def data(seed):
        W, _, _ = inputs.maxcut_instance(n, 0.2, seed=seed)
        p = dabs.dabs_problem_create(dev(W))
        g = dabs.ga_params(T=26, Bn=n, tau=8, seed=seed, capacity=20, npools=2)
        return train.collect(p, g, instances=64, rounds=40, every=2, symmetric=True)[:2]
    f_tr, y_tr = data(1)
    f_te, y_te = data(2)
    untrained = dabs.dabs_mlp_create(train.init_params(0))
    net, hist = train.fit(f_tr, y_tr, epochs=3, batch=1 << 14, lr=3e-3, seed=0)
    loss = torch.zeros(2, dtype=torch.float32, device=DEV)
    dabs.dabs_mlp_grad(untrained, f_te.shape[0], f_te, y_te, None, loss[0:1])
    dabs.dabs_mlp_grad(net, f_te.shape[0], f_te, y_te, None, loss[1:2])
    torch.cuda.synchronize()
    before, after = loss.cpu().numpy()
    assert hist[-1] < hist[0]
    assert after < before and after < np.log(2.0), (before, after)
