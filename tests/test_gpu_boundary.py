"""GPU tests of the boundary features: the Ising front-end against the
oracle's map (Section I, Eq. (1) -> (2)); delta bounds per size class with a
QAP QUBO whose penalty needs more than 2^23 (Section II-B, Table III shape);
the restart of merged pools (Section IV-B) and the run's record against the
oracle's generational loop; cancellation through a pinned host flag
(Section III-B: the host's termination request), with every kernel ending
normally; and checkpoints restored into fresh solvers and batches."""
import time

import numpy as np
import pytest

import oracle
from paper_2207_03069_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2207_03069_amd as dabs  # noqa: E402

DEV = torch.device("cuda:0")
I64MAX = np.iinfo(np.int64).max


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def unpack(t, n):
    return inputs.unpack_bits(t.cpu().numpy().view(np.uint64), n)


# ---------------------------------------------------------------- Ising
@pytest.mark.parametrize("n,m,r,seed", [(300, 2100, 16, 0), (1, 0, 1, 1), (77, 500, 2, 2)])
def test_ising_to_qubo_matches_oracle(n, m, r, seed):
    edges = inputs.sparse_graph(n, m, 15, seed) if m else np.zeros((0, 2), np.int64)
    J, h = inputs.ising_instance(n, edges, r, seed)
    # a repeated edge adds; a self loop and an out-of-range index are skipped
    good_edges, good_J = edges, J
    if m:
        good_edges, good_J = np.concatenate([edges, edges[:1]]), np.concatenate([J, J[:1]])
        edges = np.concatenate([good_edges, [[3 % n, 3 % n], [0, n]]])
        J = np.concatenate([good_J, [5, 6]])
    print("ising n=%d edges=%d" % (n, len(edges)), flush=True)
    ref_W, ref_c, ref_skip = oracle.ising_qubo(n, edges, J, h)
    ld = n + 3
    Wd = torch.full((n, ld), 77, dtype=torch.int32, device=DEV)
    off = torch.zeros(2, dtype=torch.int64, device=DEV)
    dabs.dabs_ising_to_qubo(n, dev(edges.astype(np.int32)) if len(edges) else None,
                            dev(J.astype(np.int32)) if len(edges) else None, dev(h.astype(np.int32)), Wd, off)
    torch.cuda.synchronize()
    got = Wd.cpu().numpy()
    assert np.array_equal(got[:, :n].astype(np.int64), ref_W)
    assert np.all(got[:, n:] == 77)                       # the padding columns are left alone
    assert off.cpu().numpy().tolist() == [ref_c, ref_skip]
    # the energies of the loaded QUBO are the Hamiltonian plus c
    p = dabs.dabs_problem_create(Wd[:, :n].contiguous())
    X = inputs.random_bits(5, n, seed)
    e = torch.zeros(5, dtype=torch.int64, device=DEV)
    dabs.dabs_energy(p, dev(inputs.pack_bits(X).view(np.int64)), e)
    for c in range(5):
        assert int(e[c]) == oracle.ising_hamiltonian(good_edges, good_J, h, 2 * X[c].astype(np.int64) - 1) + ref_c
    dabs.dabs_problem_destroy(p)


# ---------------------------------------------------------------- bounds
@pytest.mark.parametrize("wt,n", [(np.int32, 200), (np.int32, 400), (np.int32, 1000), (np.int32, 2048),
                                  (np.int16, 4096), (np.int16, 2048)])
def test_delta_bound_edges(wt, n):
    wtype = dabs.DABS_W_I16 if wt == np.int16 else dabs.DABS_W_I32
    mb = dabs.dabs_fast_bound(wtype, n)
    assert dabs.dabs_max_bound(wtype, n) == (1 << 31) - 1
    # key shift: log2 of the elements a lane holds (V per 16-byte piece times
    # the power-of-two slot count), at least log2 V
    V = 8 if wt == np.int16 else 4
    slots = 1
    while slots * 64 * V < n:
        slots *= 2
    K = max(int(np.log2(V)), int(np.ceil(np.log2(V * slots))))
    assert mb == (1 << (29 - K)) - 2
    # at the packed kernels' bound they serve the problem; one above it the
    # wide-delta kernels do
    for B, wide in ((mb, 0), (mb + 1, 1)):
        W = np.zeros((n, n), np.int64)
        if wt == np.int32:
            W[0, 0] = B
        else:
            # row 0 reaches B through off-diagonal weights (int16 diagonal is too small)
            k, rem = divmod(B, 2 * 32767)
            assert k + 1 <= n - 1
            W[0, 1:k + 1] = W[1:k + 1, 0] = 32767
            W[0, 0] = rem
        p = dabs.dabs_problem_create(dev(W.astype(wt)))
        assert dabs.dabs_problem_info(p)[2] == B
        assert dabs.dabs_problem_wide(p) == wide
        if wide:
            with pytest.raises(dabs.DabsError) as e:
                dabs.dabs_problem_set_wide(p, 0)
            assert e.value.status == dabs.DABS_E_RANGE
        dabs.dabs_problem_destroy(p)


def test_int32_offdiagonal_range():
    """Off-diagonal int32 weights within the packed update's 24-bit operands
    load for the packed kernels, larger ones for the wide-delta kernels, and
    a delta bound of 2^31 is refused."""
    W = np.zeros((10, 10), np.int64)
    for w, wide in (((1 << 23) - 1, 0), (1 << 23, 1), ((1 << 30) - 1, 1)):
        W[1, 2] = W[2, 1] = w
        p = dabs.dabs_problem_create(dev(W.astype(np.int32)))
        assert dabs.dabs_problem_wide(p) == wide
        dabs.dabs_problem_destroy(p)
    W[1, 1] = 2                          # row 1: 2 + 2 (2^30 - 1) = 2^31
    with pytest.raises(dabs.DabsError) as e:
        dabs.dabs_problem_create(dev(W.astype(np.int32)))
    assert e.value.status == dabs.DABS_E_RANGE


RULES = [oracle.MAXMIN, oracle.POSITIVEMIN, oracle.RANDOMMIN, oracle.CYCLICMIN, oracle.TABU_GREEDY]


@pytest.mark.parametrize("rule", RULES)
def test_search_parity_near_the_bound(rule):
    """n = 200 int32 (key shift 2): weights large enough that B is close to
    2^27 - 2, every rule's trajectory bit-exact with the oracle."""
    n = 200
    rng = np.random.default_rng(rule)
    U = rng.integers(-(1 << 19), 1 << 19, size=(n, n))
    W = np.triu(U, 1)
    W = W + W.T
    np.fill_diagonal(W, rng.integers(-(1 << 22), 1 << 22, size=n))
    B = oracle.delta_bound(W)
    assert (1 << 23) < B <= dabs.dabs_fast_bound(dabs.DABS_W_I32, n)
    p = dabs.dabs_problem_create(dev(W.astype(np.int32)))
    assert dabs.dabs_problem_wide(p) == 0
    X0 = inputs.random_bits(8, n, 3)
    x = dev(inputs.pack_bits(X0).view(np.int64))
    best = torch.zeros_like(x)
    be = torch.zeros(8, dtype=torch.int64, device=DEV)
    e = torch.zeros(8, dtype=torch.int64, device=DEV)
    delta = torch.zeros((8, n), dtype=torch.int32, device=DEV)
    trace = torch.zeros((8, 300), dtype=torch.int32, device=DEV)
    sp = dabs.dabs_search_params(rule=rule, T=300, tau=5, greedy_cap=100000, seed=9, phase=2, inst0=0)
    dabs.dabs_search(p, sp, x, None, best, be, e, delta, trace, None)
    torch.cuda.synchronize()
    for c in range(8):
        r = oracle.search(W, rule, X0[c], T=300, tau=5, seed=9, inst=c, ph=2, greedy_cap=100000, trace_cap=300)
        assert np.array_equal(trace[c].cpu().numpy()[:r["flips"]], r["trace"][:r["flips"]])
        assert int(e[c]) == r["e"] and int(be[c]) == r["ebest"]
        assert np.array_equal(delta[c].cpu().numpy().astype(np.int64), r["delta"])
    dabs.dabs_problem_destroy(p)


def solver_state(s, n, inst, P, m):
    nw = (n + 63) // 64
    bits = torch.zeros((P, m, nw), dtype=torch.int64, device=DEV)
    pe = torch.zeros((P, m), dtype=torch.int64, device=DEV)
    pa = torch.zeros((P, m), dtype=torch.int32, device=DEV)
    po = torch.zeros((P, m), dtype=torch.int32, device=DEV)
    x = torch.zeros((inst, nw), dtype=torch.int64, device=DEV)
    e = torch.zeros(inst, dtype=torch.int64, device=DEV)
    rb = torch.zeros(nw, dtype=torch.int64, device=DEV)
    ro = torch.zeros(3, dtype=torch.int64, device=DEV)
    dabs.dabs_solver_pools(s, bits, pe, pa, po)
    dabs.dabs_solver_state(s, x, e)
    dabs.dabs_solver_record(s, rb, ro)
    torch.cuda.synchronize()
    return dict(pool_bits=unpack(bits, n), pool_e=pe.cpu().numpy(), pool_algo=pa.cpu().numpy(),
                pool_op=po.cpu().numpy(), x=unpack(x, n), e=e.cpu().numpy(), best_bits=unpack(rb, n),
                best_e=int(ro[0]), restarts=int(ro[1]), rounds=int(ro[2]))


def test_qap_large_penalty_solver_parity():
    """A tai20a-shaped QAP QUBO (20 facilities -> n = 400 int32, p = 200,000,
    delta bound above 2^23): device rounds bit-exact with the oracle."""
    F, D = inputs.qap_instance(20, 0)
    W = inputs.qap_qubo(F, D, 200000)
    n = W.shape[0]
    p = dabs.dabs_problem_create(dev(W))
    assert dabs.dabs_problem_info(p)[2] == oracle.delta_bound(W) > (1 << 23)
    kw = dict(T=40, Bn=400, tau=8, seed=4, capacity=8, npools=2, greedy_cap=100000)
    inst, rounds = 16, 3
    s = dabs.dabs_solver_create(p, dabs.ga_params(**kw), inst)
    dabs.dabs_solver_run(s, rounds)
    got = solver_state(s, n, inst, 2, 8)
    ref = oracle.solve(W, oracle.ga_params(**kw), inst, rounds)
    for k in ("pool_e", "pool_bits", "pool_algo", "pool_op", "x", "e"):
        assert np.array_equal(got[k], ref[k]), k
    assert got["best_e"] == ref["best_e"] and np.array_equal(got["best_bits"], ref["best_bits"])
    assert got["rounds"] == rounds and got["restarts"] == 0


# ---------------------------------------------------------------- restart
# (60, 14): 5 restarts in 10 rounds; (60, 20): one every round; (120, 14):
# 7 in 8; (90, 0): none (pool entries are distinct, so never merged)
@pytest.mark.parametrize("n,h,rounds", [(60, 14, 10), (60, 20, 10), (120, 14, 8), (90, 0, 3)])
def test_restart_of_merged_pools_matches_oracle(n, h, rounds):
    W = inputs.dense_qubo(n, -50, 50, 13 + n)
    kw = dict(T=max(1, n // 10), Bn=n, tau=4, seed=6, capacity=4, npools=2, greedy_cap=100000,
              flags=dabs.DABS_GA_RESTART, merge_hamming=h)
    inst = 32
    p = dabs.dabs_problem_create(dev(W))
    s = dabs.dabs_solver_create(p, dabs.ga_params(**kw), inst)
    for _ in range(rounds):
        dabs.dabs_solver_run(s, 1)
    got = solver_state(s, n, inst, 2, 4)
    ref = oracle.solve(W, oracle.ga_params(**kw), inst, rounds)
    for k in ("pool_e", "pool_bits", "pool_algo", "pool_op", "x", "e"):
        assert np.array_equal(got[k], ref[k]), k
    assert got["restarts"] == ref["restarts"]
    assert got["best_e"] == ref["best_e"] and np.array_equal(got["best_bits"], ref["best_bits"])
    assert oracle.energy(W, got["best_bits"]) == got["best_e"]
    if h > 0:
        assert got["restarts"] >= 1
    if h == 0:
        assert got["restarts"] == 0
    prog = torch.zeros(2, dtype=torch.int64, device=DEV)
    dabs.dabs_solver_progress(s, prog)
    assert int(prog[1]) == got["best_e"]


# ---------------------------------------------------------------- cancel
def test_cancel_flag_stops_rounds_and_resume_is_exact():
    n, inst, P, m = 512, 64, 2, 8
    W = inputs.dense_qubo(n, -100, 100, 3)
    kw = dict(T=51, Bn=8 * n, tau=8, seed=2, capacity=m, npools=P, greedy_cap=100000)
    p = dabs.dabs_problem_create(dev(W))
    s = dabs.dabs_solver_create(p, dabs.ga_params(**kw), inst)
    flag = torch.zeros(1, dtype=torch.int32, pin_memory=True)
    dabs.dabs_solver_set_cancel(s, flag)
    dabs.dabs_solver_run(s, 1)                          # one round before anything else
    torch.cuda.synchronize()
    t0 = time.time()
    dabs.dabs_solver_run(s, 400)                        # enqueued; the flag is set while they run
    time.sleep(0.05)
    flag[0] = 1
    torch.cuda.synchronize()
    waited = time.time() - t0
    st = solver_state(s, n, inst, P, m)
    done = st["rounds"]
    print("rounds completed before the flag: %d of 401 (%.3f s)" % (done, waited), flush=True)
    assert 1 <= done < 401
    with pytest.raises(dabs.DabsError) as e:
        dabs.dabs_solver_run(s, 1)
    assert e.value.status == dabs.DABS_E_CANCELLED
    # partial pools are valid: sorted, exact energies, no duplicates
    for q in range(P):
        assert np.all(st["pool_e"][q][1:] >= st["pool_e"][q][:-1])
        fin = st["pool_e"][q] < I64MAX
        for r in np.nonzero(fin)[0]:
            assert oracle.energy(W, st["pool_bits"][q, r]) == st["pool_e"][q, r]
    # resume: after clearing the flag the run continues as if the cancelled
    # rounds had never been enqueued
    flag[0] = 0
    dabs.dabs_solver_run(s, 2)
    got = solver_state(s, n, inst, P, m)
    ref_s = dabs.dabs_solver_create(p, dabs.ga_params(**kw), inst)
    dabs.dabs_solver_run(ref_s, done + 2)
    ref = solver_state(ref_s, n, inst, P, m)
    for k in ("pool_e", "pool_bits", "x", "e", "best_e", "rounds"):
        assert np.array_equal(got[k], ref[k]), k
    dabs.dabs_solver_set_cancel(s, None)
    dabs.dabs_solver_destroy(s)
    dabs.dabs_solver_destroy(ref_s)


def test_cancel_flag_stops_graph_replayed_batch_rounds():
    """The flag is read by the device inside replays of the captured round:
    a batch of two problems enqueues 300 graph replays, the flag stops them,
    and after clearing it the batch continues exactly as an uninterrupted
    one that ran the same number of rounds."""
    Ws = [inputs.dense_qubo(400, -80, 80, 7), inputs.dense_qubo(300, -80, 80, 8, dtype=np.int32)]
    params = [dabs.ga_params(T=40, Bn=8 * 400, seed=5, capacity=8, npools=2, greedy_cap=100000),
              dabs.ga_params(T=30, Bn=8 * 300, seed=6, capacity=6, npools=1, greedy_cap=100000)]
    inst = [48, 32]
    probs = [dabs.dabs_problem_create(dev(W)) for W in Ws]
    b = dabs.dabs_batched_create(probs, params, inst)
    flag = torch.zeros(1, dtype=torch.int32, pin_memory=True)
    dabs.dabs_batched_set_cancel(b, flag)
    dabs.dabs_batched_run(b, 1, None, use_graph=True)
    torch.cuda.synchronize()
    dabs.dabs_batched_run(b, 300, None, use_graph=True)
    time.sleep(0.05)
    flag[0] = 1
    torch.cuda.synchronize()
    rec = torch.zeros(3, dtype=torch.int64, device=DEV)
    dabs.dabs_batched_record(b, 0, None, rec)
    torch.cuda.synchronize()
    done = int(rec[2])
    print("rounds completed before the flag: %d of 301" % done, flush=True)
    assert 1 <= done < 301
    with pytest.raises(dabs.DabsError) as e:
        dabs.dabs_batched_run(b, 1, None, use_graph=True)
    assert e.value.status == dabs.DABS_E_CANCELLED
    flag[0] = 0
    dabs.dabs_batched_run(b, 2, None, use_graph=True)
    ref = dabs.dabs_batched_create(probs, params, inst)
    dabs.dabs_batched_run(ref, done + 2, None, use_graph=True)
    for q, W in enumerate(Ws):
        n = W.shape[0]
        nw = (n + 63) // 64
        g = params[q]
        out = []
        for s in (b, ref):
            bits = torch.zeros((g.npools, g.capacity, nw), dtype=torch.int64, device=DEV)
            pe = torch.zeros((g.npools, g.capacity), dtype=torch.int64, device=DEV)
            x = torch.zeros((inst[q], nw), dtype=torch.int64, device=DEV)
            dabs.dabs_batched_pools(s, q, bits, pe)
            dabs.dabs_batched_state(s, q, x)
            torch.cuda.synchronize()
            out.append((bits.cpu().numpy(), pe.cpu().numpy(), x.cpu().numpy()))
        for u, v in zip(*out):
            assert np.array_equal(u, v), q
    dabs.dabs_batched_set_cancel(b, None)


def test_cancel_flag_must_be_pinned():
    W = inputs.dense_qubo(30, -5, 5, 1)
    p = dabs.dabs_problem_create(dev(W))
    s = dabs.dabs_solver_create(p, dabs.ga_params(T=3, Bn=30), 4)
    with pytest.raises(ValueError):
        dabs.dabs_solver_set_cancel(s, torch.zeros(1, dtype=torch.int32))


# ---------------------------------------------------------------- checkpoint
def test_checkpoint_restore_continues_exactly():
    """A checkpoint after 3 rounds, restored into a fresh solver, continues
    exactly as the saved solver does and as the oracle's uninterrupted loop
    (restarts of merged pools, the record and the choice counters included)."""
    n, inst, P, m = 60, 32, 2, 4
    W = inputs.dense_qubo(n, -50, 50, 13 + n)
    kw = dict(T=6, Bn=n, tau=4, seed=6, capacity=m, npools=P, greedy_cap=100000, flags=dabs.DABS_GA_RESTART,
              merge_hamming=14)
    p = dabs.dabs_problem_create(dev(W))
    a = dabs.dabs_solver_create(p, dabs.ga_params(**kw), inst)
    dabs.dabs_solver_run(a, 3)
    nbytes = dabs.dabs_solver_checkpoint(a)
    assert nbytes > 0
    blob = torch.zeros(nbytes + 8, dtype=torch.uint8, device=DEV)
    assert dabs.dabs_solver_checkpoint(a, blob) == nbytes
    dabs.dabs_solver_run(a, 4)
    b = dabs.dabs_solver_create(p, dabs.ga_params(**kw), inst)
    dabs.dabs_solver_run(b, 1)                          # state to be overwritten
    dabs.dabs_solver_restore(b, blob)
    dabs.dabs_solver_run(b, 4)
    ga, gb = solver_state(a, n, inst, P, m), solver_state(b, n, inst, P, m)
    ref = oracle.solve(W, oracle.ga_params(**kw), inst, 7)
    for k in ("pool_e", "pool_bits", "pool_algo", "pool_op", "x", "e"):
        assert np.array_equal(ga[k], gb[k]), k
        assert np.array_equal(gb[k], ref[k]), k
    for k in ("best_e", "restarts", "rounds"):
        assert ga[k] == gb[k], k
    assert gb["rounds"] == 7 and gb["restarts"] == ref["restarts"] and gb["best_e"] == ref["best_e"]
    st = torch.zeros((2, dabs.DABS_STATS), dtype=torch.int64, device=DEV)
    dabs.dabs_solver_stats(a, st[0])
    dabs.dabs_solver_stats(b, st[1])
    fa = torch.zeros(2, dtype=torch.int64, device=DEV)
    dabs.dabs_solver_state(a, total_flips=fa[0:1])
    dabs.dabs_solver_state(b, total_flips=fa[1:2])
    torch.cuda.synchronize()
    assert np.array_equal(st[0].cpu().numpy(), st[1].cpu().numpy())
    assert np.array_equal(st[1].cpu().numpy(), ref["stats"])
    assert int(fa[0]) == int(fa[1]) == ref["flips"]


def test_checkpoint_restore_batched_with_graph():
    """Two problems of both weight types, graph-replayed rounds on either side
    of the checkpoint."""
    Ws = [inputs.dense_qubo(90, -60, 60, 1), inputs.dense_qubo(300, -60, 60, 2, dtype=np.int32)]
    params = [dabs.ga_params(T=9, Bn=90, seed=3, capacity=5, npools=2, greedy_cap=100000),
              dabs.ga_params(T=30, Bn=300, seed=4, capacity=6, npools=1, greedy_cap=100000)]
    inst = [12, 7]
    probs = [dabs.dabs_problem_create(dev(W)) for W in Ws]
    a = dabs.dabs_batched_create(probs, params, inst)
    dabs.dabs_batched_run(a, 2, None, use_graph=True)
    blob = torch.zeros(dabs.dabs_batched_checkpoint(a), dtype=torch.uint8, device=DEV)
    dabs.dabs_batched_checkpoint(a, blob)
    dabs.dabs_batched_run(a, 3, None, use_graph=True)
    b = dabs.dabs_batched_create(probs, params, inst)
    dabs.dabs_batched_run(b, 1, None, use_graph=True)   # a captured round before the restore
    dabs.dabs_batched_restore(b, blob)
    dabs.dabs_batched_run(b, 3, None, use_graph=True)
    for q, W in enumerate(Ws):
        n = W.shape[0]
        nw = (n + 63) // 64
        g = params[q]
        out = []
        for s in (a, b):
            bits = torch.zeros((g.npools, g.capacity, nw), dtype=torch.int64, device=DEV)
            pe = torch.zeros((g.npools, g.capacity), dtype=torch.int64, device=DEV)
            x = torch.zeros((inst[q], nw), dtype=torch.int64, device=DEV)
            ph = torch.zeros(inst[q], dtype=torch.int32, device=DEV)
            dabs.dabs_batched_pools(s, q, bits, pe)
            dabs.dabs_batched_state(s, q, x, None, ph)
            torch.cuda.synchronize()
            out.append((bits.cpu().numpy(), pe.cpu().numpy(), x.cpu().numpy(), ph.cpu().numpy()))
        for u, v in zip(*out):
            assert np.array_equal(u, v), q


def test_checkpoint_shape_mismatch_and_size():
    W = inputs.dense_qubo(50, -9, 9, 5)
    p = dabs.dabs_problem_create(dev(W))
    a = dabs.dabs_solver_create(p, dabs.ga_params(T=5, Bn=50, seed=1, capacity=4, npools=2), 8)
    dabs.dabs_solver_run(a, 1)
    nbytes = dabs.dabs_solver_checkpoint(a)
    small = torch.zeros(nbytes - 8, dtype=torch.uint8, device=DEV)
    with pytest.raises(dabs.DabsError):
        dabs.dabs_solver_checkpoint(a, small)
    blob = torch.zeros(nbytes, dtype=torch.uint8, device=DEV)
    dabs.dabs_solver_checkpoint(a, blob)
    for kw, inst in ((dict(T=5, Bn=50, seed=1, capacity=4, npools=2), 9),      # other instance count
                     (dict(T=5, Bn=50, seed=2, capacity=4, npools=2), 8),      # other seed
                     (dict(T=5, Bn=50, seed=1, capacity=5, npools=2), 8)):     # other capacity
        c = dabs.dabs_solver_create(p, dabs.ga_params(**kw), inst)
        with pytest.raises(dabs.DabsError):
            dabs.dabs_solver_restore(c, blob)
    with pytest.raises(dabs.DabsError):
        dabs.dabs_solver_restore(a, torch.zeros(nbytes, dtype=torch.uint8, device=DEV))   # no header


def test_item_trace_of_a_round():
    """The per-item trace of a round: one record per item of the packed,
    wide-delta and sparse kernels, with the class's launch stamp before the
    item's end, its problem, main rule and flips (summing to the round's
    flips), the wave's SIMD ids; tracing changes no result and stops when
    switched off."""
    Ws = [inputs.dense_qubo(300, -60, 60, 1), inputs.wide_qubo(200, (1 << 31) - 1, 2),
          inputs.maxcut_instance(500, 0.02, seed=3)[0]]
    mk = [lambda W: dabs.dabs_problem_create(dev(W))] * 2 + \
         [lambda W: dabs.dabs_problem_create_csr(*[dev(a) for a in inputs.csr_from_dense(W)], W.shape[0])]
    params = [dabs.ga_params(T=W.shape[0] // 10, Bn=W.shape[0], seed=7 + k, capacity=5, npools=2, greedy_cap=100000)
              for k, W in enumerate(Ws)]
    inst = [9, 6, 5]
    probs = [f(W) for f, W in zip(mk, Ws)]
    a = dabs.dabs_batched_create(probs, params, inst)
    b = dabs.dabs_batched_create(probs, params, inst)
    items = dabs.dabs_batched_trace_items(a)
    assert items == sum(inst)
    buf = torch.zeros(4 * items, dtype=torch.int64, device=DEV)
    with pytest.raises(dabs.DabsError):
        dabs.dabs_batched_trace_items(a, buf[:-1])
    dabs.dabs_batched_trace_items(a, buf)
    tot = torch.zeros(1, dtype=torch.int64, device=DEV)
    dabs.dabs_batched_run(a, 1, None, use_graph=True)
    dabs.dabs_batched_flips(a, tot)
    f1 = int(tot.item())
    dabs.dabs_batched_run(a, 1, None, use_graph=True)
    dabs.dabs_batched_flips(a, tot)
    torch.cuda.synchronize()
    r = buf.view(items, 4).cpu().numpy().view(np.uint64).astype(np.int64)
    start, end, hw, w3 = r[:, 0], r[:, 1], r[:, 2], r[:, 3]
    assert np.all(start > 0) and np.all(end >= start)
    flips, rule, prob = w3 & 0xFFFFFFFF, (w3 >> 32) & 0xFF, w3 >> 40
    assert int(flips.sum()) == int(tot.item()) - f1
    assert np.array_equal(np.bincount(prob, minlength=3), inst)
    assert set(rule.tolist()) <= {dabs.DABS_MAXMIN, dabs.DABS_CYCLICMIN, dabs.DABS_RANDOMMIN, dabs.DABS_POSITIVEMIN,
                                  dabs.DABS_TWONEIGHBOR}
    assert np.all((hw >> 32) < 8) and np.all(((hw >> 4) & 3) < 4)
    for c in np.unique(prob):                       # one launch stamp per size class (one class per problem here)
        assert len(np.unique(start[prob == c])) == 1
    dabs.dabs_batched_trace_items(a, None)
    before = buf.clone()
    dabs.dabs_batched_run(a, 1, None, use_graph=True)
    dabs.dabs_batched_run(b, 3, None, use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(buf, before)
    for q, W in enumerate(Ws):
        nw = (W.shape[0] + 63) // 64
        got = []
        for bb in (a, b):
            pe = torch.zeros((2, 5), dtype=torch.int64, device=DEV)
            bits = torch.zeros((2, 5, nw), dtype=torch.int64, device=DEV)
            dabs.dabs_batched_pools(bb, q, bits, pe)
            torch.cuda.synchronize()
            got.append((pe.cpu().numpy(), bits.cpu().numpy()))
        assert np.array_equal(got[0][0], got[1][0]) and np.array_equal(got[0][1], got[1][1]), q


def test_item_trace_lds_variant():
    """The LDS variant lays a class out in groups of four items of one
    problem (dummies pad each problem): the real items are recorded once
    each, the dummies get the launch stamp only."""
    Ws = [inputs.dense_qubo(100, -60, 60, 4), inputs.dense_qubo(60, -60, 60, 5)]
    params = [dabs.ga_params(T=10, Bn=100, seed=3, capacity=5, npools=1, greedy_cap=100000),
              dabs.ga_params(T=6, Bn=60, seed=4, capacity=5, npools=1, greedy_cap=100000)]
    inst = [6, 5]
    probs = [dabs.dabs_problem_create(dev(W)) for W in Ws]
    b = dabs.dabs_batched_create(probs, params, inst)
    classes = dabs.dabs_batched_classes(b)
    assert len(classes) == 1 and classes[0][3] == 2          # one class, W in LDS
    items = dabs.dabs_batched_trace_items(b)
    assert items == 8 + 8                                    # each problem padded to a multiple of four
    buf = torch.zeros(4 * items, dtype=torch.int64, device=DEV)
    dabs.dabs_batched_trace_items(b, buf)
    tot = torch.zeros(1, dtype=torch.int64, device=DEV)
    dabs.dabs_batched_run(b, 2, None, use_graph=True)
    dabs.dabs_batched_flips(b, tot)
    torch.cuda.synchronize()
    r = buf.view(items, 4).cpu().numpy().view(np.uint64).astype(np.int64)
    assert np.all(r[:, 0] > 0)
    real = r[:, 1] > 0
    assert int(real.sum()) == sum(inst)
    assert np.all(r[~real, 2:] == 0)
    prob = r[real, 3] >> 40
    assert np.array_equal(np.bincount(prob, minlength=2), inst)
    assert np.all(r[real, 1] >= r[real, 0])
