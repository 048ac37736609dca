"""Pins of the oracle parts whose only earlier check was agreement with the
device: RandomMin's candidate probability q(t), IntervalZero's segment, the
uniform pick of MaxMin / PositiveMin, the learned operations inside the
genetic algorithm, and the restart of merged pools.

Each check compares the oracle with something other than its own code: the
real-valued schedule of Section III-A.5, statistics of the choices it makes
(geometric ranks, chi-square uniformity), equivalences with the plain
Mutation operation at hand-derived thresholds, and exact energies.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_2207_03069_amd import inputs

scipy_stats = pytest.importorskip("scipy.stats")


def E(W, x):
    x = x.astype(np.int64)
    return int(x @ W.astype(np.int64) @ x)


# ------------------------------------------------------------- RandomMin q(t)
@pytest.mark.parametrize("n", [1, 24, 100, 800, 1024, 4096])
@pytest.mark.parametrize("T", [1, 7, 80, 205])
def test_randommin_threshold_follows_the_real_schedule(n, T):
    """Section III-A.5: bit k is a candidate with probability
    p(t) = max((t/T)^3, 32/n) (at most 1); the threshold in 1/256 units is
    within one unit of 256 p(t) and equals 256 at t = T."""
    for t in range(1, T + 1):
        q = oracle.randmin_q(t, T, n)
        p = min(1.0, max((t / T) ** 3, 32.0 / n))
        assert abs(q - 256 * p) <= 1.0, (t, q, p)
    assert oracle.randmin_q(T, T, n) == 256


def test_randommin_candidate_rate_statistics():
    """With W diagonal (Delta_k = W_kk = k + 1 from X = 0, and a flip changes
    only the flipped bit's own delta) and tau >= T, the domain at iteration t
    is the set of bits not flipped yet, ordered by index.  RandomMin flips the
    least-delta candidate, so the rank of the flipped bit inside the domain is
    geometric with parameter p(t): mean (1 - p)/p.  The estimate of p(t) from
    300 instances matches max((t/T)^3, 32/n) -- a linear schedule, a missing
    32/n floor or a biased byte stream would all miss it by far."""
    n, T = 1024, 64
    W = np.zeros((n, n), np.int32)
    np.fill_diagonal(W, np.arange(1, n + 1))
    x0 = np.zeros(n, np.uint8)
    ranks = {t: [] for t in (8, 24, 32, 48, 56)}
    for inst in range(300):
        r = oracle.search(W, oracle.RANDOMMIN, x0, T=T, tau=T, seed=2024, inst=inst, ph=1, trace_cap=T)
        flipped = np.zeros(n, bool)
        for t in range(1, T + 1):
            i = int(r["trace"][t - 1])
            if t in ranks:
                ranks[t].append(int((~flipped[:i]).sum()))
            flipped[i] = True
    for t, rk in ranks.items():
        mean = float(np.mean(rk))
        p_hat = 1.0 / (1.0 + mean)
        p = max((t / T) ** 3, 32.0 / n)
        assert abs(p_hat - p) < 0.12 * p + 0.01, (t, p_hat, p)


# ------------------------------------------------------------- IntervalZero
@pytest.mark.parametrize("n", [10, 40, 64, 100, 1000])
def test_intervalzero_clears_one_cyclic_segment(n):
    """Section IV-A IntervalZero on an all-ones parent: the cleared bits form
    exactly one cyclic run of length L in [min(32, n), max(min(32, n),
    floor(n/2))]; over many draws L and the start cover their ranges
    uniformly."""
    m = 3
    g = oracle.ga_params(T=10, Bn=20, seed=11, capacity=m, npools=1, ops=(oracle.OP_INTERVALZERO,),
                         p_explore=2**32 - 1)
    pools = np.ones((1, m, n), np.uint8)
    lo = min(32, n)
    hi = max(lo, n // 2)
    lengths, starts = [], []
    draws = 1500
    for inst in range(draws):
        t, _, op = oracle.target_from_pools(g, pools, inst, rnd=3)
        assert op == oracle.OP_INTERVALZERO
        z = np.flatnonzero(t == 0)
        L = len(z)
        assert lo <= L <= hi, (inst, L)
        if L == n:
            continue
        # one cyclic run: exactly one 1 -> 0 edge going around the ring
        edges = int(np.sum((t == 1) & (np.roll(t, -1) == 0)))
        assert edges == 1, inst
        start = int((np.flatnonzero((np.roll(t, 1) == 1) & (t == 0)))[0])
        assert all(t[(start + o) % n] == 0 for o in range(L))
        lengths.append(L)
        starts.append(start)
    if hi > lo:
        counts = np.bincount(np.asarray(lengths) - lo, minlength=hi - lo + 1)
        if hi - lo + 1 <= 40:
            assert scipy_stats.chisquare(counts).pvalue > 1e-4
        else:
            assert min(lengths) < lo + (hi - lo) // 10 and max(lengths) > hi - (hi - lo) // 10
            assert abs(np.mean(lengths) - (lo + hi) / 2) < 0.06 * (hi - lo)
    if starts:
        bins = np.bincount(np.asarray(starts) * 10 // n, minlength=10)
        assert scipy_stats.chisquare(bins).pvalue > 1e-4


# ------------------------------------------------------------- uniform pick
def _first_choices(W, rule, count, T=1):
    n = W.shape[0]
    x0 = np.zeros(n, np.uint8)
    out = np.empty(count, np.int64)
    for inst in range(count):
        r = oracle.search(W, rule, x0, T=T, tau=0, seed=77, inst=inst, ph=2, trace_cap=1)
        out[inst] = r["trace"][0]
    return out


@pytest.mark.parametrize("rule", [oracle.MAXMIN, oracle.POSITIVEMIN])
def test_uniform_pick_over_equal_candidates(rule):
    """Sections III-A.3 / III-A.6 pick uniformly among the candidates.  With
    every delta equal (diagonal W = 5, X = 0) all 40 bits are candidates:
    the first choice over 4000 instances passes a chi-square test."""
    n = 40
    W = np.zeros((n, n), np.int32)
    np.fill_diagonal(W, 5)
    ch = _first_choices(W, rule, 4000)
    assert scipy_stats.chisquare(np.bincount(ch, minlength=n)).pvalue > 1e-4


@pytest.mark.parametrize("rule", [oracle.MAXMIN, oracle.POSITIVEMIN])
def test_uniform_pick_over_a_candidate_subset(rule):
    """Deltas 1 on even bits and 100 on odd bits: PositiveMin's candidates are
    the bits at or below the least positive delta and MaxMin's at t = T the
    bits at the minimum -- the even bits in both cases; the choice is always
    even and uniform over them."""
    n = 40
    W = np.zeros((n, n), np.int32)
    np.fill_diagonal(W, np.where(np.arange(n) % 2 == 0, 1, 100))
    ch = _first_choices(W, rule, 3000)
    assert np.all(ch % 2 == 0)
    assert scipy_stats.chisquare(np.bincount(ch // 2, minlength=n // 2)).pvalue > 1e-4


# ------------------------------------------------------------- learned operations
def _const_score(z):
    return lambda rnd, pools: np.full(pools.shape, z, np.float32)


# logit z -> the Mutation threshold MLP-mutate must reproduce, derived by hand
# from clamp(round-half-even(16 z), -128, 127): 2^29 + q 2^22
MUTATE_EQUIV = [(0.0, 536870912), (1 / 32, 536870912), (3 / 32, 545259520), (0.5, 570425344),
                (8.0, 1069547520), (100.0, 1069547520), (-8.0, 0), (-0.25, 520093696)]


@pytest.mark.parametrize("z,thr", MUTATE_EQUIV)
def test_mlp_mutate_with_constant_logits_is_mutation(z, thr):
    """The learned MLP-mutate with every logit equal to z flips each bit with
    the same per-bit draw as Mutation at the threshold 2^29 + q 2^22: the two
    whole generational runs agree bit for bit (pools, states), only the
    operation column differs."""
    n = 60
    W = inputs.dense_qubo(n, -50, 50, 3, dtype=np.int32)
    kw = dict(T=6, Bn=120, tau=8, seed=9, capacity=8, npools=2, p_explore=2**32 - 1)
    a = oracle.solve(W, oracle.ga_params(ops=(oracle.OP_MLP_MUTATE,), **kw), 10, 3, score=_const_score(z))
    b = oracle.solve(W, oracle.ga_params(ops=(oracle.OP_MUTATION,), p_mutation=thr, **kw), 10, 3)
    for k in ("pool_bits", "pool_e", "pool_algo", "x", "e", "ph"):
        assert np.array_equal(a[k], b[k]), k
    assert np.all(a["pool_op"] == oracle.OP_MLP_MUTATE) and np.all(b["pool_op"] == oracle.OP_MUTATION)


@pytest.mark.parametrize("z", [-1.0, 0.0, 2.0])
def test_mlp_seed_with_constant_logits(z):
    """MLP-seed flips exactly the bits of positive logit: with z <= 0 it
    copies the rank-selected parent (Mutation at rate 0), with z > 0 it
    takes the parent's complement."""
    n = 50
    W = inputs.dense_qubo(n, -50, 50, 4, dtype=np.int32)
    kw = dict(T=5, Bn=100, tau=8, seed=5, capacity=6, npools=1, p_explore=2**32 - 1)
    a = oracle.solve(W, oracle.ga_params(ops=(oracle.OP_MLP_SEED,), **kw), 8, 2, score=_const_score(z))
    if z <= 0:
        b = oracle.solve(W, oracle.ga_params(ops=(oracle.OP_MUTATION,), p_mutation=0, **kw), 8, 2)
        for k in ("pool_bits", "pool_e", "x", "e", "ph"):
            assert np.array_equal(a[k], b[k]), k
    g = oracle.ga_params(ops=(oracle.OP_MLP_SEED,), **kw)
    pools = inputs.random_bits(6, n, 1)[None]
    for inst in range(6):
        plain, _, _ = oracle.target_from_pools(g, pools, inst, rnd=1)
        t, _, _ = oracle.target_from_pools(g, pools, inst, rnd=1, logits=np.full((1, 6, n), z, np.float32))
        assert np.array_equal(t, plain ^ np.uint8(z > 0))


def test_learned_operations_use_their_parents_logits():
    """Per-bit logits: MLP-seed flips the parent's bits whose own logit is
    positive (logits of other pool entries do not matter)."""
    n, m = 70, 5
    g = oracle.ga_params(T=5, Bn=100, seed=3, capacity=m, npools=1, ops=(oracle.OP_MLP_SEED,),
                         p_explore=2**32 - 1)
    pools = inputs.random_bits(m, n, 2)[None]
    rng = np.random.default_rng(0)
    for inst in range(12):
        plain, _, _ = oracle.target_from_pools(g, pools, inst)        # the rank-selected parent
        r = [k for k in range(m) if np.array_equal(pools[0, k], plain)][0]
        z = rng.normal(0, 1, (1, m, n)).astype(np.float32)
        t, _, _ = oracle.target_from_pools(g, pools, inst, logits=z)
        assert np.array_equal(t, plain ^ (z[0, r] > 0).astype(np.uint8))


def test_solve_scores_the_pools_with_the_network():
    """The scoring hook receives the pools as they stand at the start of the
    round; with oracle/mlp.py's network the learned run keeps exact pooled
    energies, sorted and duplicate-free pools."""
    n = 40
    W = inputs.dense_qubo(n, -60, 60, 8, dtype=np.int32)
    params = omlp.init_params(1)
    seen = []

    def score(rnd, pools):
        seen.append((rnd, pools.copy()))
        return omlp.pool_logits(params, W, pools)
    g = oracle.ga_params(T=5, Bn=80, tau=8, seed=1, capacity=6, npools=2, ops=tuple(range(10)))
    s = oracle.solve(W, g, 8, 3, score=score, verify=True)
    assert [r for r, _ in seen] == [0, 1, 2]
    first = oracle.solve(W, g, 8, 1, score=lambda rnd, p: omlp.pool_logits(params, W, p))
    assert np.array_equal(seen[1][1], first["pool_bits"])
    for q in range(2):
        pe = s["pool_e"][q]
        assert np.all(pe[:-1] <= pe[1:])
        assert len({s["pool_bits"][q, r].tobytes() for r in range(6)}) == 6
        for r in range(6):
            if pe[r] != np.iinfo(np.int64).max:
                assert E(W, s["pool_bits"][q, r]) == pe[r]


# ------------------------------------------------------------- restart on merge
def test_restart_on_merge():
    """Section IV-B: merged pools are refilled with fresh random vectors.
    Reading: merged = every entry evaluated and within Hamming distance h of
    the best pooled vector.  h = 0 never merges (pool entries are distinct);
    h = n merges in the first round after which no entry is unevaluated, and
    the refill is a new draw (energies +inf, other bits than the first fill);
    the run's best vector survives the restart with its exact energy."""
    n, I = 40, 32
    W = inputs.dense_qubo(n, -60, 60, 12, dtype=np.int32)
    base = dict(T=3, Bn=2 * n, tau=4, seed=7, capacity=3, npools=2)
    R = 5
    plain = [oracle.solve(W, oracle.ga_params(**base), I, r) for r in range(R + 1)]
    full = [r for r in range(1, R + 1) if np.all(plain[r]["pool_e"] < np.iinfo(np.int64).max)]
    assert full, "the pools never fill"
    r0 = full[0]
    never = oracle.solve(W, oracle.ga_params(flags=oracle.GA_RESTART, merge_hamming=0, **base), I, R)
    assert never["restarts"] == 0 and np.array_equal(never["pool_bits"], plain[R]["pool_bits"])
    g = oracle.ga_params(flags=oracle.GA_RESTART, merge_hamming=n, **base)
    before = oracle.solve(W, g, I, r0 - 1)
    assert before["restarts"] == 0 and np.array_equal(before["pool_bits"], plain[r0 - 1]["pool_bits"])
    at = oracle.solve(W, g, I, r0)
    assert at["restarts"] == 1
    assert np.all(at["pool_e"] == np.iinfo(np.int64).max)
    assert not np.array_equal(at["pool_bits"], plain[0]["pool_bits"])
    assert at["best_e"] == int(plain[r0]["pool_e"].min())
    assert E(W, at["best_bits"]) == at["best_e"]
    prev = at["best_e"]
    for r in range(r0 + 1, R + 1):
        s = oracle.solve(W, g, I, r)
        assert s["best_e"] <= prev and E(W, s["best_bits"]) == s["best_e"]
        prev = s["best_e"]


# ------------------------------------------------------------- bookkeeping
def test_operation_and_algorithm_counters():
    """The counters behind the tables of Section VI-D: every instance chooses
    one operation and one main algorithm per round; a packet that enters a
    pool counts once for its operation and once for its algorithm; the
    record's columns are those of the pooled entry holding it."""
    W = inputs.dense_qubo(60, -40, 40, 3)
    I, R = 12, 4
    r = oracle.solve(W, oracle.ga_params(T=6, Bn=60, tau=4, seed=2, capacity=5, npools=2), I, R)
    st = r["stats"]
    use_op, use_al, ins_op, ins_al = st[0:16], st[16:24], st[24:40], st[40:48]
    assert use_op.sum() == I * R and use_al.sum() == I * R
    n_ins = int((r["inserts"] >= 0).sum())
    assert ins_op.sum() == n_ins and ins_al.sum() == n_ins
    assert np.all(ins_op <= use_op) and np.all(ins_al <= use_al)
    assert np.all(use_op[8:] == 0) and np.all(use_al[:2] == 0)       # only the enabled ones
    q, k = np.argwhere(r["pool_e"] == r["best_e"])[0]
    assert st[48] == r["pool_op"][q, k] and st[49] == r["pool_algo"][q, k]
