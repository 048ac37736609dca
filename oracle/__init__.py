"""CPU oracle of the Diverse Adaptive Bulk Search hot path (arXiv 2207.03069).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; the product package never
imports it.  The C source (``dabs_oracle.c``) is compiled with gcc into
``liboracle.so`` next to this file; this module only marshals numpy arrays.

Vectors are numpy uint8 arrays of 0/1 (one byte per bit); W is any integer
array, converted to int32 here.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dabs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GREEDY, STRAIGHT, MAXMIN, CYCLICMIN, RANDOMMIN, POSITIVEMIN, TWONEIGHBOR, TABU_GREEDY = range(8)
(OP_RANDOM, OP_BEST, OP_MUTATION, OP_CROSSOVER, OP_XROSSOVER, OP_ZERO, OP_ONE, OP_INTERVALZERO,
 OP_MLP_SEED, OP_MLP_MUTATE) = range(10)
GA_RESTART = 2                      # flag: restart the pools when they have merged
MAIN_ALGOS = (MAXMIN, CYCLICMIN, RANDOMMIN, POSITIVEMIN, TWONEIGHBOR)
ALL_OPS = tuple(range(8))
P_EXPLORE_5PCT = 214748365          # ceil(0.05 * 2^32)
P_EIGHTH = 1 << 29                  # 1/8
P_ONE_PERCENT = 42949673            # ceil(0.01 * 2^32)
GREEDY_CAP_DEFAULT = 1 << 40


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class GAParams(C.Structure):
    _fields_ = [("n_algos", C.c_int32), ("algos", C.c_int32 * 8),
                ("n_ops", C.c_int32), ("ops", C.c_int32 * 16),
                ("p_explore", C.c_uint32), ("p_mutation", C.c_uint32),
                ("p_zero", C.c_uint32), ("p_one", C.c_uint32),
                ("crossover_kind", C.c_int32), ("capacity", C.c_int32),
                ("npools", C.c_int32), ("tau", C.c_int32),
                ("T", C.c_int64), ("Bn", C.c_int64), ("greedy_cap", C.c_int64),
                ("seed", C.c_uint64), ("flags", C.c_uint32), ("merge_hamming", C.c_int32)]


def ga_params(*, T, Bn, tau=8, seed=0, capacity=100, npools=1, algos=MAIN_ALGOS, ops=ALL_OPS,
              p_explore=P_EXPLORE_5PCT, p_mutation=P_EIGHTH, p_zero=P_EIGHTH, p_one=P_EIGHTH,
              crossover_kind=0, greedy_cap=GREEDY_CAP_DEFAULT, flags=0, merge_hamming=0) -> GAParams:
    g = GAParams()
    g.n_algos = len(algos)
    for i, a in enumerate(algos):
        g.algos[i] = a
    g.n_ops = len(ops)
    for i, o in enumerate(ops):
        g.ops[i] = o
    g.p_explore, g.p_mutation, g.p_zero, g.p_one = p_explore, p_mutation, p_zero, p_one
    g.crossover_kind, g.capacity, g.npools, g.tau = crossover_kind, capacity, npools, tau
    g.T, g.Bn, g.greedy_cap, g.seed = T, Bn, greedy_cap, seed
    g.flags, g.merge_hamming = flags, merge_hamming
    return g


SCORE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.POINTER(C.c_uint8), C.POINTER(C.c_float))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i32, i64, u32, u64 = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
        L.orc_philox.argtypes = [P, u64, P]
        L.orc_energy.argtypes = [P, i32, P]
        L.orc_energy.restype = i64
        L.orc_delta_scratch.argtypes = [P, i32, P, P]
        L.orc_delta_closed.argtypes = [P, i32, P, P]
        L.orc_delta_bound.argtypes = [P, i32]
        L.orc_delta_bound.restype = i64
        L.orc_is_symmetric.argtypes = [P, i32]
        L.orc_is_symmetric.restype = i32
        L.orc_rank_index.argtypes = [u32, u32]
        L.orc_rank_index.restype = u32
        L.orc_search.argtypes = [P, i32, i32, i64, i32, u64, u32, u32, i64,
                                 P, P, P, P, P, P, P, i64, i32]
        L.orc_search.restype = i64
        L.orc_batch_search.argtypes = [P, i32, i32, i64, i64, i32, u64, u32, P, i64,
                                       P, P, P, P, P, P, P, i64, P, i32, P, i32]
        L.orc_batch_search.restype = i64
        L.orc_solve.argtypes = [P, i32, P, i32, i32, P, P, P, P, P, P, P, P, P, P, i32]
        L.orc_solve.restype = i64
        L.orc_solve_ex.argtypes = [P, i32, P, i32, i32, P, P, P, P, P, P, P, P, P, P, i32,
                                   SCORE_FN, P, P, P, P, P, P]
        L.orc_solve_ex.restype = i64
        L.orc_target_from_pools.argtypes = [i32, P, P, P, P, P, P, u32, u32, P, P, P]
        L.orc_randmin_q.argtypes = [i64, i64, i32]
        L.orc_randmin_q.restype = i32
        L.orc_first_target.argtypes = [i32, P, u32, P, P, P]
        L.orc_first_target.restype = i32
        L.orc_all_energies.argtypes = [P, i32, P]
        L.orc_bruteforce.argtypes = [P, i32, P]
        L.orc_bruteforce.restype = i64
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _w(W):
    W = np.ascontiguousarray(np.asarray(W, dtype=np.int32))
    assert W.ndim == 2 and W.shape[0] == W.shape[1]
    return W


def _bits(x, n):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.uint8))
    assert x.shape == (n,)
    return x.copy()


def philox(ctr, seed):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_p(c), C.c_uint64(seed), _p(out))
    return out


def energy(W, x) -> int:
    W = _w(W)
    return int(lib().orc_energy(_p(W), W.shape[0], _p(_bits(x, W.shape[0]))))


def delta_scratch(W, x):
    W = _w(W)
    out = np.zeros(W.shape[0], dtype=np.int64)
    lib().orc_delta_scratch(_p(W), W.shape[0], _p(_bits(x, W.shape[0])), _p(out))
    return out


def delta_closed(W, x):
    W = _w(W)
    out = np.zeros(W.shape[0], dtype=np.int64)
    lib().orc_delta_closed(_p(W), W.shape[0], _p(_bits(x, W.shape[0])), _p(out))
    return out


def delta_bound(W) -> int:
    W = _w(W)
    return int(lib().orc_delta_bound(_p(W), W.shape[0]))


def is_symmetric(W) -> bool:
    W = _w(W)
    return bool(lib().orc_is_symmetric(_p(W), W.shape[0]))


def ising_hamiltonian(edges, J, h, s) -> int:
    """Eq. (1): H(S) = sum over edges of J_ij s_i s_j + sum_i h_i s_i
    (s_i in {-1, +1}), summed edge by edge as written."""
    s = np.asarray(s, dtype=np.int64)
    H = 0
    for (i, j), v in zip(np.asarray(edges).tolist(), np.asarray(J).tolist()):
        H += int(v) * int(s[i]) * int(s[j])
    return H + int(np.asarray(h, dtype=np.int64) @ s)


def ising_qubo(n: int, edges, J, h):
    """The QUBO of an Ising model under x_i = (s_i + 1) / 2 and the energy of
    Eq. (2) summed over all ordered pairs: substituting s_i = 2 x_i - 1 into
    Eq. (1), an edge term J s_i s_j = 4J x_i x_j - 2J x_i - 2J x_j + J and a
    bias term h s_i = 2h x_i - h.  The quadratic part 4J x_i x_j is split
    over the two ordered pairs (W_ij = W_ji = 2J), the linear parts go to the
    diagonal (x_i^2 = x_i) and the constants to c, so that E(X) = H(S) + c
    with c = sum h - sum J.  Edges with i == j or an index outside [0, n)
    are skipped (returned as the count `skipped`).  Returns (W int64, c,
    skipped)."""
    W = np.zeros((n, n), dtype=np.int64)
    c = 0
    skipped = 0
    for (i, j), v in zip(np.asarray(edges).reshape(-1, 2).tolist(), np.asarray(J).tolist()):
        if i == j or not (0 <= i < n and 0 <= j < n):
            skipped += 1
            continue
        W[i, j] += 2 * v
        W[j, i] += 2 * v
        W[i, i] -= 2 * v
        W[j, j] -= 2 * v
        c -= v
    for i, v in enumerate(np.asarray(h).tolist()):
        W[i, i] += 2 * v
        c += v
    return W, c, skipped


def rank_index(u: int, m: int) -> int:
    return int(lib().orc_rank_index(u, m))


def search(W, rule, x0, *, T=0, tau=0, seed=0, inst=0, ph=0, target=None,
           greedy_cap=GREEDY_CAP_DEFAULT, trace_cap=0, verify=False):
    """One search call (one phase of `rule`) from x0.  Returns a dict."""
    W = _w(W)
    n = W.shape[0]
    x = _bits(x0, n)
    tg = _bits(target, n) if target is not None else None
    best = np.zeros(n, dtype=np.uint8)
    eb, e = C.c_int64(), C.c_int64()
    delta = np.zeros(n, dtype=np.int64)
    trace = np.full(max(trace_cap, 1), -1, dtype=np.int32)
    f = lib().orc_search(_p(W), n, rule, T, tau, C.c_uint64(seed), inst, ph, greedy_cap,
                         _p(x), _p(tg), _p(best), C.byref(eb), C.byref(e), _p(delta),
                         _p(trace) if trace_cap else None, trace_cap, int(verify))
    if f < 0:
        raise RuntimeError("oracle search failed (%d)" % f)
    return dict(flips=int(f), x=x, e=int(e.value), best=best, ebest=int(eb.value), delta=delta,
                trace=trace[:min(f, trace_cap)] if trace_cap else None)


def batch_search(W, rule, x0, target, *, T, Bn, tau=0, seed=0, inst=0, ph=0,
                 greedy_cap=GREEDY_CAP_DEFAULT, trace_cap=0, phase_cap=256, verify=False):
    W = _w(W)
    n = W.shape[0]
    x = _bits(x0, n)
    tg = _bits(target, n)
    best = np.zeros(n, dtype=np.uint8)
    eb, e = C.c_int64(), C.c_int64()
    phc = C.c_uint32(ph)
    delta = np.zeros(n, dtype=np.int64)
    trace = np.full(max(trace_cap, 1), -1, dtype=np.int32)
    pf = np.zeros(phase_cap, dtype=np.int64)
    npf = C.c_int32()
    f = lib().orc_batch_search(_p(W), n, rule, T, Bn, tau, C.c_uint64(seed), inst, C.byref(phc),
                               greedy_cap, _p(x), _p(tg), _p(best), C.byref(eb), C.byref(e),
                               _p(delta), _p(trace) if trace_cap else None, trace_cap,
                               _p(pf), phase_cap, C.byref(npf), int(verify))
    if f < 0:
        raise RuntimeError("oracle batch search failed (%d)" % f)
    return dict(flips=int(f), x=x, e=int(e.value), best=best, ebest=int(eb.value), delta=delta,
                ph=int(phc.value), phase_flips=pf[:min(npf.value, phase_cap)].copy(),
                trace=trace[:min(f, trace_cap)] if trace_cap else None)


def solve(W, g: GAParams, instances: int, rounds: int, verify=False, score=None, tick=None):
    """Generational DABS loop; returns pools, per-instance state, insert log,
    the best pooled vector over the run (kept across restarts) and the number
    of restarts.  score(round, pool_bits [P][m][n] uint8) -> float32 logits
    [P][m][n] gives the learned scores of every pooled bit at the start of a
    round (the MLP operations copy their parent without it); tick(round),
    optional, is called at the start of every round; round_best holds the
    record's energy after each round."""
    W = _w(W)
    n = W.shape[0]
    P, m = g.npools, g.capacity
    cb = SCORE_FN()
    if score is not None:
        def _cb(ctx, rnd, bits, out):
            if tick is not None:
                tick(int(rnd))
            pb = np.ctypeslib.as_array(bits, shape=(P, m, n)).copy()
            z = np.ascontiguousarray(np.asarray(score(int(rnd), pb), dtype=np.float32).reshape(P * m * n))
            np.ctypeslib.as_array(out, shape=(P * m * n,))[:] = z
        cb = SCORE_FN(_cb)
    elif tick is not None:
        if any(o in (OP_MLP_SEED, OP_MLP_MUTATE) for o in g.ops[:g.n_ops]):
            raise ValueError("tick without score: the learned operations need scores")

        def _tick(ctx, rnd, bits, out):   # the scores are left unset: no learned operation is enabled
            tick(int(rnd))
        cb = SCORE_FN(_tick)
    rb = np.zeros(max(rounds, 1), dtype=np.int64)
    st = np.zeros(50, dtype=np.int64)
    pb = np.zeros((P, m, n), dtype=np.uint8)
    pe = np.zeros((P, m), dtype=np.int64)
    pa = np.zeros((P, m), dtype=np.int32)
    po = np.zeros((P, m), dtype=np.int32)
    x = np.zeros((instances, n), dtype=np.uint8)
    e = np.zeros(instances, dtype=np.int64)
    ph = np.zeros(instances, dtype=np.uint32)
    ins = np.zeros((max(rounds, 1), instances), dtype=np.int32)
    tg = np.zeros((instances, n), dtype=np.uint8)
    pk = np.zeros(instances, dtype=np.int64)
    bb = np.zeros(n, dtype=np.uint8)
    be = C.c_int64()
    nr = C.c_int32()
    f = lib().orc_solve_ex(_p(W), n, C.byref(g), instances, rounds, _p(pb), _p(pe), _p(pa), _p(po),
                           _p(x), _p(e), _p(ph), _p(ins), _p(tg), _p(pk), int(verify), cb, None,
                           _p(bb), C.byref(be), C.byref(nr), _p(rb), _p(st))
    if f < 0:
        raise RuntimeError("oracle solve failed (%d)" % f)
    return dict(flips=int(f), pool_bits=pb, pool_e=pe, pool_algo=pa, pool_op=po, x=x, e=e, ph=ph,
                inserts=ins[:rounds], targets=tg, packets=pk, best_bits=bb, best_e=int(be.value),
                restarts=int(nr.value), round_best=rb[:rounds], stats=st)


def target_from_pools(g: GAParams, pool_bits, inst, rnd=0, pool_e=None, pool_algo=None, pool_op=None,
                      logits=None):
    """The target (and algorithm, operation) that instance `inst` draws in
    round `rnd` from the given pools ([P][m][n] 0/1)."""
    pb = np.ascontiguousarray(np.asarray(pool_bits, dtype=np.uint8))
    P, m, n = pb.shape
    assert (P, m) == (g.npools, g.capacity)
    pe = np.ascontiguousarray(pool_e if pool_e is not None else np.zeros((P, m)), dtype=np.int64)
    pa = np.ascontiguousarray(pool_algo if pool_algo is not None else np.full((P, m), MAXMIN), dtype=np.int32)
    po = np.ascontiguousarray(pool_op if pool_op is not None else np.zeros((P, m)), dtype=np.int32)
    lg = None if logits is None else np.ascontiguousarray(np.asarray(logits, dtype=np.float32).reshape(P, m, n))
    t = np.zeros(n, dtype=np.uint8)
    a, o = C.c_int32(), C.c_int32()
    lib().orc_target_from_pools(n, C.byref(g), _p(pb), _p(pe), _p(pa), _p(po), _p(lg), rnd, inst, _p(t),
                                C.byref(a), C.byref(o))
    return t, int(a.value), int(o.value)


def randmin_q(t: int, T: int, n: int) -> int:
    """RandomMin's candidate threshold at iteration t (in 1/256 units)."""
    return int(lib().orc_randmin_q(t, T, n))


def first_target(n, g: GAParams, inst):
    t = np.zeros(n, dtype=np.uint8)
    a, o = C.c_int32(), C.c_int32()
    lib().orc_first_target(n, C.byref(g), inst, _p(t), C.byref(a), C.byref(o))
    return t, int(a.value), int(o.value)


def all_energies(W):
    W = _w(W)
    n = W.shape[0]
    assert n <= 20
    out = np.zeros(1 << n, dtype=np.int64)
    lib().orc_all_energies(_p(W), n, _p(out))
    return out


def bruteforce(W):
    W = _w(W)
    n = W.shape[0]
    assert n <= 40
    am = np.zeros(n, dtype=np.uint8)
    e = lib().orc_bruteforce(_p(W), n, _p(am))
    return int(e), am
