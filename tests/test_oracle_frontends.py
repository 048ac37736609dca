"""Pins of the problem front-ends the oracle checks the device against:
the Ising -> QUBO map of Section I (Eq. (1) -> Eq. (2)) by brute force over
every spin vector, and the one-hot QAP QUBO of Section II-B (E = C(g) - n p
on every permutation, E >= -(n-1) p on infeasible vectors)."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from paper_2207_03069_amd import inputs

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _bits(v, n):
    return np.array([(v >> k) & 1 for k in range(n)], np.uint8)


@pytest.mark.parametrize("n,m,r,seed", [(1, 0, 1, 0), (6, 9, 1, 1), (10, 20, 2, 2), (12, 30, 16, 3)])
def test_ising_qubo_brute_force(n, m, r, seed):
    """E(X) = H(S) + c for all 2^n pairs x = (s + 1) / 2 (the definition of
    Eq. (1) evaluated edge by edge against the oracle's energy of Eq. (2))."""
    edges = inputs.sparse_graph(n, m, n, seed) if m else np.zeros((0, 2), np.int64)
    J, h = inputs.ising_instance(n, edges, r, seed)
    W, c, skipped = oracle.ising_qubo(n, edges, J, h)
    assert skipped == 0 and oracle.is_symmetric(W)
    for v in range(1 << n):
        x = _bits(v, n)
        assert oracle.energy(W, x) == oracle.ising_hamiltonian(edges, J, h, 2 * x.astype(np.int64) - 1) + c


def test_ising_qubo_worked_example_stand_in():
    """The stand-in for the example of Section I-A: c = 6 and the QUBO optimum
    X = [1,0,0,0,1], E = -8 (H = -14)."""
    g = json.load(open(os.path.join(GOLD, "worked_example.json")))
    edges = np.array([[i, j] for i, j, _ in g["J"]])
    J = np.array([v for _, _, v in g["J"]])
    W, c, _ = oracle.ising_qubo(g["n"], edges, J, g["h"])
    assert c == g["printed"]["offset"]
    e, am = oracle.bruteforce(W)
    assert e == g["printed"]["E_opt"] and list(am) == g["printed"]["X_opt"]
    assert oracle.ising_hamiltonian(edges, J, g["h"], g["printed"]["S_opt"]) == g["printed"]["H_opt"]


def test_ising_qubo_skips_bad_edges_and_adds_repeats():
    edges = np.array([[0, 1], [1, 1], [0, 1], [2, 5]])
    J = np.array([3, 7, -1, 4])
    W, c, skipped = oracle.ising_qubo(3, edges, J, [1, 0, -2])
    assert skipped == 2
    W2, c2, _ = oracle.ising_qubo(3, np.array([[0, 1]]), np.array([2]), [1, 0, -2])
    assert np.array_equal(W, W2) and c == c2


def test_qap_qubo_identity_on_every_permutation():
    """Section II-B: a feasible X (a permutation g) has E(X) = C(g) - n p."""
    n, p = 5, 10000
    F, D = inputs.qap_instance(n, 4)
    W = inputs.qap_qubo(F, D, p, dtype=np.int64)
    assert oracle.is_symmetric(W)
    for g in itertools.permutations(range(n)):
        x = np.zeros(n * n, np.uint8)
        x[np.arange(n) * n + np.array(g)] = 1
        assert oracle.energy(W, x) == inputs.qap_cost(F, D, g) - n * p


def test_qap_qubo_infeasible_vectors_lie_above():
    """Section II-B: with nonnegative flows and distances an infeasible X has
    E(X) >= -(n - 1) p (all vectors of weight <= 3 and random ones)."""
    n, p = 4, 10000
    F, D = inputs.qap_instance(n, 5)
    W = inputs.qap_qubo(F, D, p, dtype=np.int64)
    N = n * n
    rng = np.random.default_rng(0)
    cands = [np.zeros(N, np.uint8)]
    for k in (1, 2, 3):
        for idx in itertools.combinations(range(N), k):
            x = np.zeros(N, np.uint8)
            x[list(idx)] = 1
            cands.append(x)
    cands += list(rng.integers(0, 2, (3000, N)).astype(np.uint8))
    for x in cands:
        M = x.reshape(n, n)
        if (M.sum(0) == 1).all() and (M.sum(1) == 1).all():
            continue
        assert oracle.energy(W, x) >= -(n - 1) * p


def test_qap_table3_shape_fits_the_device_bound():
    """A tai20a-shaped QUBO (20 facilities, p = 200,000, flows and distances
    in [0, 99]) has a delta bound above 2^23 (the flat bound of the largest
    slot class) but below 2^26 - 2, the device bound at n = 400 int32."""
    F, D = inputs.qap_instance(20, 0)
    W = inputs.qap_qubo(F, D, 200000)
    B = oracle.delta_bound(W)
    assert (1 << 23) < B < (1 << 26) - 2


def test_batched_targets_file_reproduces():
    """The stored time-to-target energies of the many-problem workload are
    what the committed script computes with the oracle (three of the
    smallest problems recomputed)."""
    import importlib.util
    path = os.path.join(GOLD, "make_batched_targets.py")
    spec = importlib.util.spec_from_file_location("make_batched_targets", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    stored = json.load(open(os.path.join(GOLD, "batched_targets.json")))["targets"]
    sizes = inputs.batched_sizes(256, seed=0)
    for p in np.argsort(sizes)[:3]:
        assert mod.target(int(p)) == stored[int(p)], p
