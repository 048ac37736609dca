"""Pins of the oracle's energy, flip deltas, problem encodings and generator.

Each check ties the oracle to something other than itself: a numpy quadratic
form, the definition of Delta by two energies, exhaustive enumeration, numbers
printed in the paper, or an independent library routine (rocrand's Philox).
"""
import itertools
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2207_03069_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _rand_sym(n, lo, hi, seed):
    return inputs.dense_qubo(n, lo, hi, seed, dtype=np.int32)


@pytest.mark.parametrize("n,seed", [(1, 0), (5, 1), (24, 2), (65, 3), (130, 4)])
def test_energy_is_quadratic_form(n, seed):
    """Eq. (2) over all ordered pairs equals x^T W x (numpy int64 matmul)."""
    W = _rand_sym(n, -1000, 1000, seed)
    X = inputs.random_bits(8, n, seed + 10)
    for x in X:
        ref = int(x.astype(np.int64) @ W.astype(np.int64) @ x.astype(np.int64))
        assert oracle.energy(W, x) == ref


def test_zero_vector_state():
    """Section III-A: X = 0 gives E = 0 and Delta_k = W_kk."""
    W = _rand_sym(40, -128, 127, 5)
    z = np.zeros(40, np.uint8)
    assert oracle.energy(W, z) == 0
    assert np.array_equal(oracle.delta_closed(W, z), np.diag(W).astype(np.int64))
    assert np.array_equal(oracle.delta_scratch(W, z), np.diag(W).astype(np.int64))


@pytest.mark.parametrize("n,seed", [(2, 0), (17, 1), (64, 2), (97, 3)])
def test_closed_form_delta_equals_definition(n, seed):
    """Eq. (3) in closed form equals E(f_k X) - E(X) from two scratch energies."""
    W = _rand_sym(n, -30000, 30000, seed)
    for x in inputs.random_bits(4, n, seed):
        assert np.array_equal(oracle.delta_closed(W, x), oracle.delta_scratch(W, x))


def test_flip_negates_own_delta():
    """Eq. (5): Delta_i(f_i X) = -Delta_i(X)."""
    n = 33
    W = _rand_sym(n, -500, 500, 9)
    x = inputs.random_bits(1, n, 9)[0]
    d = oracle.delta_scratch(W, x)
    for i in range(n):
        y = x.copy()
        y[i] ^= 1
        assert oracle.delta_scratch(W, y)[i] == -d[i]


def test_delta_bound_is_attained_bound():
    """|Delta_k(X)| never exceeds the load-time bound, and the bound is the
    largest |Delta| over all X for a small n (exhaustive)."""
    n = 10
    W = _rand_sym(n, -50, 50, 11)
    B = oracle.delta_bound(W)
    worst = 0
    for v in range(1 << n):
        x = np.array([(v >> k) & 1 for k in range(n)], np.uint8)
        worst = max(worst, int(np.abs(oracle.delta_closed(W, x)).max()))
    assert worst <= B
    # the bound is attained when the signs of x line up with the row (exhaustive max
    # over X reaches max_k |W_kk| + 2 sum |W_kj| only if signs allow; check it is tight
    # for a row of one sign)
    W2 = np.abs(W)
    assert max(int(np.abs(oracle.delta_closed(W2, np.ones(n, np.uint8))).max()),
               int(np.abs(oracle.delta_closed(W2, np.zeros(n, np.uint8))).max())) <= oracle.delta_bound(W2)
    k = int(np.argmax(np.abs(np.diag(W2)) + 2 * (W2.sum(1) - np.diag(W2))))
    x = np.ones(n, np.uint8)
    x[k] = 0
    assert abs(int(oracle.delta_closed(W2, x)[k])) == oracle.delta_bound(W2)


def test_symmetry_check():
    W = _rand_sym(12, -9, 9, 3)
    assert oracle.is_symmetric(W)
    W[2, 7] += 1
    assert not oracle.is_symmetric(W)


def test_worked_example_stand_in():
    """Section I-A: E(X) = H(S) + 6 for all corresponding S, X; optimum
    S = [+1,-1,-1,-1,+1], H = -14; X = [1,0,0,0,1], E = -8.  The J, h values
    are a constructed stand-in (Fig. 1's numbers are not in the text)."""
    g = _gold("worked_example.json")
    n = g["n"]
    J = np.zeros((n, n), np.int64)
    for i, j, v in g["J"]:
        J[i, j] = v
    h = np.array(g["h"], np.int64)
    # Ising -> QUBO under the spin map s = 2x - 1 and the full ordered-pair sum
    W = np.zeros((n, n), np.int64)
    for i, j, v in g["J"]:
        W[i, j] = W[j, i] = 2 * v
    Jsym = J + J.T
    for i in range(n):
        W[i, i] = 2 * h[i] - 2 * Jsym[i].sum()
    pr = g["printed"]
    best_h, best_s = None, None
    for v in range(1 << n):
        x = np.array([(v >> k) & 1 for k in range(n)], np.uint8)
        s = 2 * x.astype(np.int64) - 1
        H = int(sum(J[i, j] * s[i] * s[j] for i in range(n) for j in range(n)) + h @ s)
        assert oracle.energy(W, x) == H + pr["offset"]
        if best_h is None or H < best_h:
            best_h, best_s = H, s
    assert best_h == pr["H_opt"] and list(best_s) == pr["S_opt"]
    e, am = oracle.bruteforce(W)
    assert e == pr["E_opt"] and list(am) == pr["X_opt"]


@pytest.mark.parametrize("n,seed", [(1, 0), (6, 1), (11, 2), (14, 3)])
def test_bruteforce_matches_enumeration(n, seed):
    """Gray-code enumeration minimum equals the minimum of scratch energies,
    and its argmin attains it."""
    W = _rand_sym(n, -128, 127, seed)
    allE = oracle.all_energies(W)
    e, am = oracle.bruteforce(W)
    assert e == int(allE.min())
    assert oracle.energy(W, am) == e
    if n <= 10:
        ref = min(int(x @ W.astype(np.int64) @ x) for x in
                  (np.array([(v >> k) & 1 for k in range(n)], np.int64) for v in range(1 << n)))
        assert ref == e


def test_qap_energy_identity():
    """Section II-B: for the one-hot QAP QUBO, E(X) = C(g) - n p for every
    feasible X (all permutations, n = 5) and E(X) >= -(n-1) p otherwise."""
    n, p = 5, 1000
    rng = np.random.default_rng(7)
    L = rng.integers(0, 20, (n, n)); L = np.triu(L, 1); L = L + L.T
    Dm = rng.integers(0, 20, (n, n)); Dm = np.triu(Dm, 1); Dm = Dm + Dm.T
    N = n * n
    W = np.zeros((N, N), np.int64)
    for i, j, i2, j2 in itertools.product(range(n), repeat=4):
        a, b = i * n + j, i2 * n + j2
        if i != i2 and j != j2:
            W[a, b] = L[i, i2] * Dm[j, j2]
        elif i == i2 and j == j2:
            W[a, b] = -p
        else:
            W[a, b] = p
    for g in itertools.permutations(range(n)):
        x = np.zeros(N, np.uint8)
        for i in range(n):
            x[i * n + g[i]] = 1
        C = sum(L[i, j] * Dm[g[i], g[j]] for i in range(n) for j in range(n))
        assert oracle.energy(W, x) == C - n * p
    for x in inputs.random_bits(300, N, 8):
        feasible = all(x.reshape(n, n).sum(0) == 1) and all(x.reshape(n, n).sum(1) == 1)
        if not feasible:
            assert oracle.energy(W, x) >= -(n - 1) * p


def test_qap_table3_arithmetic():
    """Table III's QUBO optima are C - n p (the full-sum convention; the
    once-per-pair sum would give C/2 - n p)."""
    for r in _gold("qap_table3.json")["rows"]:
        assert r["C"] - r["n"] * r["p"] == r["qubo"]
        assert r["C"] // 2 - r["n"] * r["p"] != r["qubo"]


def test_maxcut_energy_is_minus_cut():
    """Section II-A: -E(X) is the cut value of the node split X."""
    n = 120
    W, edges, w = inputs.maxcut_instance(n, 0.08, seed=3, dtype=np.int32)
    for x in inputs.random_bits(10, n, 4):
        cut = int(sum(wt for (i, j), wt in zip(edges, w) if x[i] != x[j]))
        assert -oracle.energy(W, x) == cut


def test_maxcut_generator_shape():
    """The 800-node workload: about 0.06 * C(800,2) edges, weights +-1."""
    W, edges, w = inputs.maxcut_instance(800, 0.06, seed=0)
    m = len(edges)
    exp = 0.06 * 800 * 799 / 2
    assert abs(m - exp) < 5 * np.sqrt(exp)
    assert set(np.unique(w)) == {-1, 1}
    assert oracle.is_symmetric(W)
    assert np.array_equal(np.diag(W).astype(np.int64), -(W.astype(np.int64).sum(1) - np.diag(W)))


def test_tsp_encoding_small():
    """TSP as a one-hot QUBO: every tour of 6 cities has E = 2 L - 2 N A and
    is a local minimum (no single flip lowers E)."""
    N = 6
    xy, D = inputs.tsp_cities(N, seed=5)
    A = 2 * int(D.max())
    W = inputs.tsp_qubo(D, A)
    for perm in itertools.permutations(range(N)):
        x = np.zeros(N * N, np.uint8)
        for t, c in enumerate(perm):
            x[c * N + t] = 1
        Ltour = sum(D[perm[t], perm[(t + 1) % N]] for t in range(N))
        assert oracle.energy(W, x) == 2 * Ltour - 2 * N * A
        if perm[0] == 0 and perm[1] < perm[-1]:
            assert oracle.delta_closed(W, x).min() >= 0


def test_tsp_generator_c3():
    """32 cities, n = 1024, random tours satisfy E = 2 L - 2 N A."""
    W, D, A = inputs.tsp_instance(32, seed=0)
    assert W.shape == (1024, 1024) and W.dtype == np.int32
    assert A == 2 * int(D.max())
    rng = np.random.default_rng(1)
    for _ in range(3):
        perm = rng.permutation(32)
        x = np.zeros(1024, np.uint8)
        for t, c in enumerate(perm):
            x[c * 32 + t] = 1
        Ltour = int(sum(D[perm[t], perm[(t + 1) % 32]] for t in range(32)))
        assert oracle.energy(W, x) == 2 * Ltour - 2 * 32 * A


def test_rounded_distance():
    for dx in range(0, 60):
        for dy in range(0, 60):
            assert inputs.rounded_distance(dx, dy) == int(np.floor(np.hypot(dx, dy) + 0.5))


def test_pack_roundtrip():
    for n in (1, 63, 64, 65, 800):
        b = inputs.random_bits(3, n, n)
        assert np.array_equal(inputs.unpack_bits(inputs.pack_bits(b), n), b)
    b = np.zeros(70, np.uint8)
    b[65] = 1
    assert inputs.pack_bits(b)[1] == 2


_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct P : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};
int main() {
    P e; unsigned a, b, c, d, k0, k1;
    while (scanf("%u %u %u %u %u %u", &a, &b, &c, &d, &k0, &k1) == 6) {
        uint4 r = e.ten_rounds(uint4{a, b, c, d}, uint2{k0, k1});
        printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
}
"""


def test_philox_matches_rocrand(tmp_path):
    """The oracle's Philox4x32-10 equals rocrand's host implementation of the
    same generator on random (counter, key) tuples."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "probe.cpp"
    src.write_text(_PROBE)
    exe = tmp_path / "probe"
    subprocess.check_call([hipcc, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           "-O1", str(src), "-o", str(exe)])
    rng = np.random.default_rng(0)
    tup = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
    tup[0] = 0
    tup[1] = 2**32 - 1
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in tup)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    got = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], np.uint64)
    for row, ref in zip(tup, got):
        seed = int(row[4]) | (int(row[5]) << 32)
        assert np.array_equal(oracle.philox(row[:4].astype(np.uint32), seed).astype(np.uint64), ref)


def test_philox_uniform_bytes():
    cnt = np.zeros(256, np.int64)
    for i in range(4096):
        w = oracle.philox([i, 7, 0, 1 << 24], 12345)
        cnt += np.bincount(w.view(np.uint8), minlength=256)
    exp = cnt.sum() / 256
    chi2 = float(((cnt - exp) ** 2 / exp).sum())
    assert chi2 < 400  # 255 dof; p ~ 1e-8 tail
