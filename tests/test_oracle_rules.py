"""Pins of the oracle's search rules, batch search and genetic algorithm.

Trajectories are replayed with numpy energies computed from scratch, so every
check below is independent of the oracle's incremental bookkeeping.  Where the
paper fixes a fact (TwoNeighbor's flip order, the batch-search schedule, the
local-minimum property of Greedy, Straight's Hamming distance, the rank
selection probability) the test states it.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2207_03069_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def E(W, x):
    x = x.astype(np.int64)
    return int(x @ W.astype(np.int64) @ x)


def D(W, x):
    """Delta by definition: E(f_k X) - E(X)."""
    e0 = E(W, x)
    out = np.zeros(len(x), np.int64)
    for k in range(len(x)):
        y = x.copy()
        y[k] ^= 1
        out[k] = E(W, y) - e0
    return out


def replay(W, x0, trace):
    """States X_0 .. X_f and their deltas."""
    xs, ds = [x0.copy()], [D(W, x0)]
    x = x0.copy()
    for i in trace:
        x[i] ^= 1
        xs.append(x.copy())
        ds.append(D(W, x))
    return xs, ds


def check_best(W, res, xs, ds):
    """Step 1 at every visited state: E(BEST) is the least energy over all
    visited states and their 1-bit neighbours, and BEST attains it."""
    lo = min(min(E(W, x), E(W, x) + int(d.min())) for x, d in zip(xs, ds))
    assert res["ebest"] == lo
    assert E(W, res["best"]) == lo


def first_argmin(vals, dom):
    idx = [k for k in range(len(vals)) if dom[k]]
    m = min(vals[k] for k in idx)
    return next(k for k in idx if vals[k] == m)


def make(n=40, seed=0, lo=-100, hi=100):
    W = inputs.dense_qubo(n, lo, hi, seed, dtype=np.int32)
    x0 = inputs.random_bits(1, n, seed + 100)[0]
    return W, x0


def test_twoneighbor_trace_golden():
    """Section III-A.7: n = 6 from 000000 flips 0,1,0,2,1,3,2,4,3,5,4 and
    visits the printed states."""
    g = _gold("twoneighbor_n6.json")
    n = g["n"]
    W = inputs.dense_qubo(n, -5, 5, 1, dtype=np.int32)
    r = oracle.search(W, oracle.TWONEIGHBOR, np.zeros(n, np.uint8), trace_cap=64, verify=True)
    assert r["flips"] == 2 * n - 1 == len(g["flips"])
    assert list(r["trace"]) == g["flips"]
    xs, ds = replay(W, np.zeros(n, np.uint8), r["trace"])
    assert ["".join(str(int(b)) for b in x) for x in xs] == g["states"]


def test_twoneighbor_covers_two_bit_neighbours():
    """Step 1 along TwoNeighbor sees every 2-bit neighbour of the start."""
    W, x0 = make(24, 3)
    r = oracle.search(W, oracle.TWONEIGHBOR, x0, trace_cap=64)
    lo = E(W, x0)
    n = len(x0)
    for i in range(n):
        for j in range(i, n):
            y = x0.copy()
            y[i] ^= 1
            if j != i:
                y[j] ^= 1
            lo = min(lo, E(W, y))
    assert r["ebest"] <= lo


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_greedy_reaches_local_minimum(seed):
    """Section III-A.1: Greedy flips the argmin Delta while a Delta is
    negative and stops at a local minimum (all Delta >= 0)."""
    W, x0 = make(48, seed)
    r = oracle.search(W, oracle.GREEDY, x0, trace_cap=4096, verify=True)
    xs, ds = replay(W, x0, r["trace"])
    for t, i in enumerate(r["trace"]):
        assert ds[t].min() < 0 and i == first_argmin(ds[t], np.ones(len(x0), bool))
        assert E(W, xs[t + 1]) < E(W, xs[t])
    assert ds[-1].min() >= 0
    assert np.array_equal(r["delta"], ds[-1]) and r["e"] == E(W, xs[-1])
    check_best(W, r, xs, ds)


@pytest.mark.parametrize("seed", [0, 1])
def test_straight_reaches_target(seed):
    """Section III-A.2: Straight makes exactly Hamming(X, D) flips, each the
    argmin Delta over differing bits, and ends at X = D."""
    W, x0 = make(40, seed)
    tgt = inputs.random_bits(1, 40, seed + 7)[0]
    r = oracle.search(W, oracle.STRAIGHT, x0, target=tgt, trace_cap=4096, verify=True)
    assert r["flips"] == int((x0 != tgt).sum())
    assert np.array_equal(r["x"], tgt)
    xs, ds = replay(W, x0, r["trace"])
    for t, i in enumerate(r["trace"]):
        assert i == first_argmin(ds[t], xs[t] != tgt)
    check_best(W, r, xs, ds)


def tabu_dom(trace, t, tau, n):
    """Non-tabu domain at iteration t (1-based): bits flipped at t-tau .. t-1
    are excluded; all bits when that excludes everything."""
    dom = np.ones(n, bool)
    for s in range(max(1, t - tau), t):
        dom[trace[s - 1]] = False
    return dom if dom.any() else np.ones(n, bool)


@pytest.mark.parametrize("tau", [0, 4, 8])
def test_tabu_greedy(tau):
    """Tabu greedy: each of the T flips is the non-tabu argmin Delta."""
    W, x0 = make(24, 5, -128, 127)
    T = 80
    r = oracle.search(W, oracle.TABU_GREEDY, x0, T=T, tau=tau, trace_cap=T, verify=True)
    assert r["flips"] == T
    xs, ds = replay(W, x0, r["trace"])
    for t in range(1, T + 1):
        assert r["trace"][t - 1] == first_argmin(ds[t - 1], tabu_dom(r["trace"], t, tau, 24))
    check_best(W, r, xs, ds)


def test_tabu_greedy_tiny_n_all_tabu():
    """With n <= tau every bit becomes tabu; the rule then ignores tabu."""
    W, x0 = make(3, 9)
    r = oracle.search(W, oracle.TABU_GREEDY, x0, T=20, tau=8, trace_cap=20, verify=True)
    xs, ds = replay(W, x0, r["trace"])
    for t in range(1, 21):
        assert r["trace"][t - 1] == first_argmin(ds[t - 1], tabu_dom(r["trace"], t, 8, 3))


def cyclic_windows(n, T):
    """Window starts and widths of CyclicMin from the integer reading, with
    the real-valued width max((t/T)^3 n, c) alongside."""
    pos, out = 0, []
    for t in range(1, T + 1):
        if t == T:
            w = n
        else:
            h = (t << 32) // T
            h3 = (((h * h) >> 32) * h) >> 32
            w = min(n, max(min(32, n), (n * h3) >> 32))
        real = max((t / T) ** 3 * n, min(32, n))
        out.append((pos, w, real))
        pos = (pos + w) % n
    return out


@pytest.mark.parametrize("n,T,tau", [(100, 150, 8), (20, 30, 4), (300, 64, 0)])
def test_cyclicmin(n, T, tau):
    """Section III-A.4: the flip is the (non-tabu) argmin inside a cyclic
    window of width w(t) = max((t/T)^3 n, c) that slides by its width;
    w(T) = n.  The integer width stays within one of the real formula."""
    W, x0 = make(n, 11)
    r = oracle.search(W, oracle.CYCLICMIN, x0, T=T, tau=tau, trace_cap=T, verify=n <= 100)
    wins = cyclic_windows(n, T)
    assert wins[-1][1] == n
    for pos, w, real in wins:
        assert abs(w - min(real, n)) <= 1
    xs, ds = replay(W, x0, r["trace"])
    for t in range(1, T + 1):
        pos, w, _ = wins[t - 1]
        win = np.zeros(n, bool)
        for o in range(w):
            win[(pos + o) % n] = True
        dom = win & tabu_dom(r["trace"], t, tau, n)
        if not dom.any():
            dom = win
        assert r["trace"][t - 1] == first_argmin(ds[t - 1], dom)
    check_best(W, r, xs, ds)


@pytest.mark.parametrize("tau", [0, 8])
def test_maxmin(tau):
    """Section III-A.3: the flipped bit has Delta in [minD, D(t)] over the
    non-tabu bits (D(t) real-valued, +1 for the integer reading), and at
    t = T the threshold equals minD."""
    n, T = 50, 120
    W, x0 = make(n, 12)
    r = oracle.search(W, oracle.MAXMIN, x0, T=T, tau=tau, seed=77, inst=3, ph=5,
                      trace_cap=T, verify=True)
    xs, ds = replay(W, x0, r["trace"])
    for t in range(1, T + 1):
        dom = tabu_dom(r["trace"], t, tau, n)
        d = ds[t - 1]
        mn, mx = d[dom].min(), d[dom].max()
        f = ((T - t) / T) ** 3
        Dt = (1 - f) * mn + f * mx
        i = r["trace"][t - 1]
        assert dom[i] and mn <= d[i] <= Dt + 1
        if t == T:
            assert d[i] == mn
    check_best(W, r, xs, ds)


def test_maxmin_uses_randomness():
    """Different instances (generator counters) give different trajectories."""
    W, x0 = make(50, 13)
    a = oracle.search(W, oracle.MAXMIN, x0, T=100, tau=8, seed=1, inst=0, trace_cap=100)
    b = oracle.search(W, oracle.MAXMIN, x0, T=100, tau=8, seed=1, inst=1, trace_cap=100)
    c = oracle.search(W, oracle.MAXMIN, x0, T=100, tau=8, seed=1, inst=0, trace_cap=100)
    assert not np.array_equal(a["trace"], b["trace"])
    assert np.array_equal(a["trace"], c["trace"])


@pytest.mark.parametrize("tau", [0, 8])
def test_positivemin(tau):
    """Section III-A.6: the flipped bit's Delta is at most the least positive
    non-tabu Delta (any non-tabu bit when none is positive)."""
    n, T = 45, 100
    W, x0 = make(n, 14)
    r = oracle.search(W, oracle.POSITIVEMIN, x0, T=T, tau=tau, seed=5, inst=2,
                      trace_cap=T, verify=True)
    xs, ds = replay(W, x0, r["trace"])
    for t in range(1, T + 1):
        dom = tabu_dom(r["trace"], t, tau, n)
        d = ds[t - 1]
        i = r["trace"][t - 1]
        assert dom[i]
        pos = d[dom & (d > 0)]
        if len(pos):
            assert d[i] <= pos.min()
    check_best(W, r, xs, ds)


@pytest.mark.parametrize("tau", [0, 8])
def test_randommin(tau):
    """Section III-A.5: the flipped bit is non-tabu with Delta at or above
    the non-tabu minimum, and at t = T (p = 1) it is the non-tabu argmin."""
    n, T = 70, 90
    W, x0 = make(n, 15)
    r = oracle.search(W, oracle.RANDOMMIN, x0, T=T, tau=tau, seed=9, inst=4,
                      trace_cap=T, verify=True)
    xs, ds = replay(W, x0, r["trace"])
    sizes = []
    for t in range(1, T + 1):
        dom = tabu_dom(r["trace"], t, tau, n)
        d = ds[t - 1]
        i = r["trace"][t - 1]
        assert dom[i] and d[i] >= d[dom].min()
        if t == T:
            assert i == first_argmin(d, dom)
        sizes.append(int((d[dom] < d[i]).sum()))
    check_best(W, r, xs, ds)
    # early iterations pick among few candidates: often not the global argmin
    assert sum(1 for s in sizes[: T // 3] if s > 0) > T // 10


def test_batch_schedule_golden():
    """Section III-B example: n = 1000, s = 0.6, b = 2.0 give 600 main flips
    and a 2000-flip batch budget; the main search then runs three times.
    With W = 0 every Greedy phase makes 0 flips and Straight makes
    Hamming(X, D) = 300, so the phases are 300, 0, 600, 0, 600, 0, 600, 0."""
    g = _gold("batch_example.json")
    n = g["n"]
    T, Bn = round(g["s"] * n), round(g["b"] * n)
    assert (T, Bn) == (g["main_flips"], g["batch_flips"])
    W = np.zeros((n, n), np.int32)
    x0 = np.zeros(n, np.uint8)
    tgt = np.zeros(n, np.uint8)
    tgt[: g["straight"]] = 1
    r = oracle.batch_search(W, oracle.CYCLICMIN, x0, tgt, T=T, Bn=Bn, tau=8)
    pf = list(r["phase_flips"])
    assert pf == [300, 0, 600, 0, 600, 0, 600, 0]
    assert len(pf[2::2]) == g["mains"] and r["ph"] == g["mains"]
    # with the printed 50-flip Greedy phases the same rule gives the printed total
    tot, mains = g["straight"] + g["greedy"], 0
    while tot < g["batch_flips"]:
        tot += g["main_flips"] + g["greedy"]
        mains += 1
    assert (tot, mains) == (g["total"], g["mains"])


@pytest.mark.parametrize("rule", [oracle.MAXMIN, oracle.CYCLICMIN, oracle.RANDOMMIN,
                                  oracle.POSITIVEMIN, oracle.TWONEIGHBOR])
def test_batch_search_structure(rule):
    """Straight to the target, Greedy, then {main, Greedy} until the flips of
    the batch search reach Bn (TwoNeighbor once); every Greedy ends at a local
    minimum; BEST covers the whole batch search."""
    n, T, Bn = 36, 20, 150
    W, x0 = make(n, 20 + rule)
    tgt = inputs.random_bits(1, n, 21)[0]
    r = oracle.batch_search(W, rule, x0, tgt, T=T, Bn=Bn, tau=8, seed=3, inst=1, ph=10,
                            trace_cap=100000, verify=True)
    pf = list(r["phase_flips"])
    assert pf[0] == int((x0 != tgt).sum())
    mains = pf[2::2]
    if rule == oracle.TWONEIGHBOR:
        assert mains == [2 * n - 1]
    else:
        assert all(m == T for m in mains)
        cum = pf[0] + pf[1]
        for k in range(len(mains)):
            assert cum < Bn
            cum += pf[2 + 2 * k] + pf[3 + 2 * k]
        assert cum >= Bn
    assert r["ph"] == 10 + len(mains)
    assert r["flips"] == sum(pf) == len(r["trace"])
    xs, ds = replay(W, x0, r["trace"])
    # end of each Greedy phase is a local minimum
    c = 0
    for k, f in enumerate(pf):
        c += f
        if k % 2 == 1:
            assert ds[c].min() >= 0
    check_best(W, r, xs, ds)


def test_rank_selection_probability():
    """Section IV-A: the (floor(r^3 m)+1)-th entry; the first is chosen with
    probability m^(-1/3) and P(rank <= k) = ((k+1)/m)^(1/3)."""
    m = 100
    u = np.random.default_rng(0).integers(0, 2**32, 200000, dtype=np.uint64)
    ranks = np.array([oracle.rank_index(int(v), m) for v in u[:200000]])
    assert ranks.min() >= 0 and ranks.max() < m
    p0 = (ranks == 0).mean()
    assert abs(p0 - m ** (-1 / 3)) < 0.005
    for k in (4, 19, 49):
        assert abs((ranks <= k).mean() - ((k + 1) / m) ** (1 / 3)) < 0.005


def _initial_pool(n, g):
    g0 = oracle.ga_params(T=g.T, Bn=g.Bn, seed=g.seed, capacity=g.capacity, npools=g.npools,
                          algos=tuple(g.algos[: g.n_algos]), ops=tuple(g.ops[: g.n_ops]),
                          crossover_kind=g.crossover_kind, p_mutation=g.p_mutation)
    s = oracle.solve(np.zeros((n, n), np.int32), g0, 1, 0)
    return s["pool_bits"]


@pytest.mark.parametrize("op", range(8))
def test_genetic_operations(op):
    """Section IV-A/B operation semantics on targets drawn from the initial
    pools: Zero only clears (~1/8), One only sets (~1/8), IntervalZero clears
    one cyclic segment of length in [32, n/2], Best copies entry 0, Mutation
    flips ~1/8, (X)rossover takes every bit from one of two entries (the
    second from the next pool for Xrossover), Random is unrelated to the pool."""
    n, P, m = 256, 3, 12
    g = oracle.ga_params(T=10, Bn=20, seed=4, capacity=m, npools=P, ops=(op,), p_explore=2**32 - 1)
    pools = _initial_pool(n, g)
    for inst in range(24):
        t, algo, o = oracle.first_target(n, g, inst)
        assert o == op and algo in oracle.MAIN_ALGOS
        q = inst % P
        own = pools[q]
        if op == oracle.OP_BEST:
            assert np.array_equal(t, own[0])
        elif op == oracle.OP_ZERO:
            ok = [a for a in own if np.all(t <= a)]
            assert ok and 0.03 < (ok[0] - t).sum() / max(ok[0].sum(), 1) < 0.3
        elif op == oracle.OP_ONE:
            ok = [a for a in own if np.all(t >= a)]
            assert ok and 0.03 < (t - ok[0]).sum() / max((1 - ok[0]).sum(), 1) < 0.3
        elif op == oracle.OP_INTERVALZERO:
            found = False
            for a in own:
                diff = np.flatnonzero(a != t)
                if np.all(t <= a):
                    found = True
                    break
            assert found
        elif op == oracle.OP_MUTATION:
            hd = min(int((a != t).sum()) for a in own)
            assert 0.05 * n < hd < 0.22 * n
        elif op in (oracle.OP_CROSSOVER, oracle.OP_XROSSOVER):
            other = pools[(q + 1) % P] if op == oracle.OP_XROSSOVER else own
            assert any(np.all((t == a) | (t == b)) and 0 < (t != a).sum()
                       for a in own for b in other)
        elif op == oracle.OP_RANDOM:
            assert min(int((a != t).sum()) for a in own) > n // 4


def test_two_point_crossover():
    """Two-point crossover: the target is the first parent outside one
    contiguous index range and the second parent inside it."""
    n, m = 200, 8
    g = oracle.ga_params(T=10, Bn=20, seed=6, capacity=m, npools=1, ops=(oracle.OP_CROSSOVER,),
                         p_explore=2**32 - 1, crossover_kind=1)
    pools = _initial_pool(n, g)[0]
    for inst in range(16):
        t, _, _ = oracle.first_target(n, g, inst)
        ok = False
        for a in pools:
            for b in pools:
                d = np.flatnonzero(t != a)
                if len(d) == 0:
                    ok = True
                elif np.all(t[d[0]: d[-1] + 1] == b[d[0]: d[-1] + 1]):
                    ok = True
        assert ok


def test_adaptive_choice_frequency():
    """Section IV-A: with probability 5% the operation is uniform over all
    operations, else copied from a uniform pool row."""
    n, m = 64, 10
    g = oracle.ga_params(T=10, Bn=20, seed=8, capacity=m, npools=1)
    s = oracle.solve(np.zeros((n, n), np.int32), g, 1, 0)
    col = s["pool_op"][0]
    hits = 0
    N = 3000
    for inst in range(N):
        _, _, o = oracle.first_target(n, g, inst)
        hits += o in set(col.tolist())
    # P(op in column) = 0.95 + 0.05 * |set(col)| / 8
    pin = 0.95 + 0.05 * len(set(col.tolist())) / 8
    assert abs(hits / N - pin) < 0.02


def test_solve_pool_invariants():
    """Generational loop: pools stay sorted ascending, hold no duplicate
    vectors, their energies are exact, and the best entry only improves."""
    n = 48
    W = inputs.dense_qubo(n, -100, 100, 31, dtype=np.int32)
    prev = None
    for rounds in (1, 2, 4):
        g = oracle.ga_params(T=10, Bn=60, tau=8, seed=2, capacity=10, npools=2)
        s = oracle.solve(W, g, 12, rounds, verify=True)
        for q in range(2):
            pe = s["pool_e"][q]
            assert np.all(pe[:-1] <= pe[1:])
            seen = set()
            for r in range(10):
                key = s["pool_bits"][q, r].tobytes()
                assert key not in seen
                seen.add(key)
                if pe[r] != np.iinfo(np.int64).max:
                    assert E(W, s["pool_bits"][q, r]) == pe[r]
        best = int(s["pool_e"].min())
        if prev is not None:
            assert best <= prev
        prev = best
        for i in range(12):
            assert E(W, s["x"][i]) == s["e"][i]


def test_c1_tabu_greedy_finds_certified_optimum():
    """The 24-bit correctness workload: 64 tabu-greedy instances (tau = 4) of
    2000 flips; the best energy found equals the Gray-code optimum."""
    W = inputs.dense_qubo(24, -128, 127, 0, dtype=np.int32)
    opt, _ = oracle.bruteforce(W)
    X0 = inputs.random_bits(64, 24, 1)
    best = min(oracle.search(W, oracle.TABU_GREEDY, x, T=2000, tau=4)["ebest"] for x in X0)
    assert best == opt
