"""Seeded synthetic inputs for the bulk-search workloads.

This module only draws problems and bit vectors; it holds none of the search
arithmetic and is shared by the tests, the benchmark and the oracle checks.
Every generator uses ``numpy.random.default_rng(seed)`` with the draw order
stated in its docstring.  Bit vectors are numpy uint8 arrays of 0/1.

Workload shapes follow the paper's problem families (Section II and VI):
dense random QUBOs, max-cut graphs mapped to QUBO (Section II-A) and TSP as a
one-hot QUBO (the circular-flow special case of Section II-B).  The benchmark
instances of the paper (K2000, G-set, QAPLIB, the D-Wave QASP graph) are not
available; these generators stand in for them with the same shapes.
"""
from __future__ import annotations

import math

import numpy as np


def dense_qubo(n: int, lo: int, hi: int, seed: int, dtype=np.int16) -> np.ndarray:
    """Symmetric W: the upper triangle including the diagonal is drawn uniform
    in [lo, hi] (one n x n draw, row-major, upper part kept) and mirrored."""
    rng = np.random.default_rng(seed)
    U = rng.integers(lo, hi + 1, size=(n, n), dtype=np.int64)
    W = np.triu(U)
    W = W + np.triu(W, 1).T
    return W.astype(dtype)


def wide_qubo(n: int, bound: int, seed: int, dtype=np.int32) -> np.ndarray:
    """Symmetric int32 W whose delta bound max_k(|W_kk| + 2 sum_{j!=k} |W_kj|)
    is at most `bound` and close to it: off-diagonal entries uniform in
    [-a, a] with a = bound // (4 max(n - 1, 1)), the diagonal uniform in
    [-bound // 2, bound // 2] (one n x n draw, upper part kept, mirrored)."""
    rng = np.random.default_rng(seed)
    a = bound // (4 * max(n - 1, 1))
    U = rng.integers(-a, a + 1, size=(n, n), dtype=np.int64)
    W = np.triu(U, 1)
    W = W + W.T
    np.fill_diagonal(W, rng.integers(-(bound // 2), bound // 2 + 1, size=n, dtype=np.int64))
    return W.astype(dtype)


def extreme_qubo(n: int, seed: int) -> np.ndarray:
    """int32 W (n >= 3) with delta bound exactly 2^31 - 1, whose deltas reach
    +-(2^31 - 1): W_00 = 2^30 - 1, W_11 = -(2^30 - 1), W_01 = 2^29 (rows 0
    and 1 otherwise zero, so Delta_0 = +-(2^31 - 1) when x_1 = 1), the other
    rows a wide_qubo block of bound 2^31 - 1."""
    W = np.zeros((n, n), np.int64)
    W[0, 0], W[1, 1] = (1 << 30) - 1, -((1 << 30) - 1)
    W[0, 1] = W[1, 0] = 1 << 29
    W[2:, 2:] = wide_qubo(n - 2, (1 << 31) - 1, seed).astype(np.int64)
    return W.astype(np.int32)


def maxcut_graph(n: int, p: float, seed: int):
    """Erdos-Renyi G(n, p) with +-1 edge weights of equal probability.
    Draw order: an n x n uniform matrix (edge i<j present iff U_ij < p), then
    an n x n sign matrix (weight of edge i<j is +1 iff S_ij = 1).
    Returns (edges int64 [m,2] with i<j, weights int64 [m])."""
    rng = np.random.default_rng(seed)
    U = rng.random((n, n))
    S = rng.integers(0, 2, size=(n, n))
    iu, ju = np.triu_indices(n, 1)
    keep = U[iu, ju] < p
    edges = np.stack([iu[keep], ju[keep]], axis=1).astype(np.int64)
    w = np.where(S[iu[keep], ju[keep]] == 1, 1, -1).astype(np.int64)
    return edges, w


def maxcut_qubo(n: int, edges: np.ndarray, w: np.ndarray, dtype=np.int16) -> np.ndarray:
    """Section II-A: each edge contributes w (2 x_i x_j - x_i^2 - x_j^2).  With
    the energy summed over all ordered pairs this is W_ij = W_ji = w_ij and
    W_ii = -sum_j w_ij, so E(X) = -cut(X)."""
    W = np.zeros((n, n), dtype=np.int64)
    W[edges[:, 0], edges[:, 1]] = w
    W[edges[:, 1], edges[:, 0]] = w
    np.fill_diagonal(W, -W.sum(axis=1))
    return W.astype(dtype)


def maxcut_instance(n: int = 800, p: float = 0.06, seed: int = 0, dtype=np.int16):
    edges, w = maxcut_graph(n, p, seed)
    return maxcut_qubo(n, edges, w, dtype), edges, w


def rounded_distance(dx: int, dy: int) -> int:
    """round(sqrt(dx^2 + dy^2)) in exact integer arithmetic (half rounds up)."""
    s = dx * dx + dy * dy
    r = math.isqrt(s)
    return r + (1 if s > r * r + r else 0)


def tsp_cities(ncity: int = 32, grid: int = 1000, seed: int = 0):
    """City coordinates uniform integers in [0, grid-1]^2; returns (xy, D)."""
    rng = np.random.default_rng(seed)
    xy = rng.integers(0, grid, size=(ncity, 2), dtype=np.int64)
    D = np.zeros((ncity, ncity), dtype=np.int64)
    for a in range(ncity):
        for b in range(ncity):
            D[a, b] = rounded_distance(int(xy[a, 0] - xy[b, 0]), int(xy[a, 1] - xy[b, 1]))
    return xy, D


def tsp_qubo(D: np.ndarray, A: int | None = None, dtype=np.int32) -> np.ndarray:
    """TSP as a one-hot QUBO, bit (c, t) = city c at tour position t at index
    c * N + t (the indexing of Section II-B).  W_aa = -2A; W_ab = A when a, b
    share exactly one of {city, position}; W_ab = d(c, c') when c != c' and
    t' = t +- 1 (mod N); else 0.  A feasible tour of length L has
    E = 2 L - 2 N A.  Default A = 2 max d."""
    N = D.shape[0]
    if A is None:
        A = 2 * int(D.max())
    n = N * N
    W = np.zeros((n, n), dtype=np.int64)
    for c in range(N):
        for t in range(N):
            a = c * N + t
            for c2 in range(N):
                for t2 in range(N):
                    b = c2 * N + t2
                    if a == b:
                        W[a, b] = -2 * A
                    elif (c == c2) != (t == t2):
                        W[a, b] = A
                    elif c != c2 and ((t2 - t) % N in (1, N - 1)):
                        W[a, b] = D[c, c2]
    return W.astype(dtype)


def tsp_instance(ncity: int = 32, seed: int = 0):
    xy, D = tsp_cities(ncity, seed=seed)
    A = 2 * int(D.max())
    return tsp_qubo(D, A), D, A


def qap_instance(nfac: int, seed: int, lo: int = 0, hi: int = 99):
    """A symmetric QAP of nfac facilities (Section II-B): flows l(i, j) and
    distances d(i, j) uniform integers in [lo, hi] for i < j, mirrored, zero
    diagonals (the uniform random shape of Taillard's tai*a instances).  Draw
    order: one nfac x nfac flow matrix, then one distance matrix, upper parts
    kept.  Returns (flow, dist) int64."""
    rng = np.random.default_rng(seed)
    F = np.triu(rng.integers(lo, hi + 1, size=(nfac, nfac), dtype=np.int64), 1)
    D = np.triu(rng.integers(lo, hi + 1, size=(nfac, nfac), dtype=np.int64), 1)
    return F + F.T, D + D.T


def qap_qubo(flow: np.ndarray, dist: np.ndarray, p: int, dtype=np.int32) -> np.ndarray:
    """The one-hot QUBO of Section II-B: bit <i, j> = i * n + j (facility i at
    location j); W = l(i, i') d(j, j') for i != i' and j != j', -p on the
    diagonal, p for two bits sharing exactly one of facility and location.
    A feasible X has E(X) = C(g_X) - n p."""
    n = flow.shape[0]
    N = n * n
    W = np.einsum("ac,bd->abcd", flow.astype(np.int64), dist.astype(np.int64)).reshape(N, N)
    fi = np.repeat(np.arange(n), n)
    lj = np.tile(np.arange(n), n)
    same_f = fi[:, None] == fi[None, :]
    same_l = lj[:, None] == lj[None, :]
    W[same_f != same_l] = p
    W[same_f & same_l] = -p
    return W.astype(dtype)


def qap_cost(flow: np.ndarray, dist: np.ndarray, g) -> int:
    """C(g) = sum_{i, j} l(i, j) d(g(i), g(j))."""
    g = np.asarray(g)
    return int((flow * dist[np.ix_(g, g)]).sum())


def sparse_graph(n: int, m: int, max_degree: int, seed: int):
    """m distinct undirected edges on n nodes, every degree <= max_degree:
    candidate pairs (i, j), i != j, drawn uniformly in batches of 4m; a pair
    is kept when new and both ends are below the cap.  Returns edges int64
    [m, 2] with i < j.  Stands in for a quantum annealer's sparse hardware
    graph (Section II-C: 5,627 nodes, 40,279 edges; degree at most 15)."""
    rng = np.random.default_rng(seed)
    deg = np.zeros(n, dtype=np.int64)
    seen = set()
    out = []
    while len(out) < m:
        cand = rng.integers(0, n, size=(4 * m, 2))
        for i, j in cand.tolist():
            if len(out) == m:
                break
            if i == j:
                continue
            a, b = (i, j) if i < j else (j, i)
            if (a, b) in seen or deg[a] >= max_degree or deg[b] >= max_degree:
                continue
            seen.add((a, b))
            deg[a] += 1
            deg[b] += 1
            out.append((a, b))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def ising_instance(n: int, edges: np.ndarray, r: int, seed: int):
    """A random Ising model of resolution r (Section II-C): every J_ij uniform
    over the nonzero integers in [-r, r] and every h_i over the nonzero
    integers in [-4r, 4r].  Draw order: J (one per edge), then h.  Returns
    (J int64 [m], h int64 [n])."""
    rng = np.random.default_rng(seed)

    def nonzero(k, size):
        v = rng.integers(1, k + 1, size=size)
        return np.where(rng.integers(0, 2, size=size) == 1, v, -v).astype(np.int64)

    J = nonzero(r, len(edges))
    h = nonzero(4 * r, n)
    return J, h


def csr_from_dense(W: np.ndarray):
    """CSR rows (row_ptr, col, val as int32) of the nonzeros of W, columns
    increasing within a row."""
    W = np.asarray(W)
    rows, cols = np.nonzero(W)
    rp = np.zeros(W.shape[0] + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp).astype(np.int32), cols.astype(np.int32), W[rows, cols].astype(np.int32)


def batched_sizes(count: int = 256, lo: int = 256, ratio: int = 16, seed: int = 0) -> np.ndarray:
    """Problem sizes n = floor(lo * ratio^U), U ~ U[0,1), for the many-problem
    workload (log-uniform in [256, 4096))."""
    rng = np.random.default_rng(seed)
    U = rng.random(count)
    return np.floor(lo * np.power(float(ratio), U)).astype(np.int64)


def batched_problems(count: int = 256, seed: int = 0, lo: int = -1000, hi: int = 1000):
    """Sizes from batched_sizes(seed), then problem p drawn by
    dense_qubo(n_p, lo, hi, seed * 100003 + p + 1)."""
    sizes = batched_sizes(count, seed=seed)
    return [dense_qubo(int(n), lo, hi, seed * 100003 + p + 1) for p, n in enumerate(sizes)]


def random_bits(count: int, n: int, seed: int) -> np.ndarray:
    """[count, n] uint8 uniform 0/1."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=(count, n), dtype=np.uint8)


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """[..., n] 0/1 -> [..., ceil(n/64)] uint64, bit k in word k//64 at k%64."""
    bits = np.asarray(bits, dtype=np.uint8)
    n = bits.shape[-1]
    words = (n + 63) // 64
    pad = np.zeros(bits.shape[:-1] + (words * 64,), dtype=np.uint8)
    pad[..., :n] = bits
    by = np.packbits(pad.reshape(bits.shape[:-1] + (words * 8, 8)), axis=-1, bitorder="little")
    return np.ascontiguousarray(by.reshape(bits.shape[:-1] + (words * 8,))).view(np.uint64)


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    """Inverse of pack_bits."""
    words = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
    by = words.view(np.uint8)
    bits = np.unpackbits(by.reshape(words.shape[:-1] + (words.shape[-1] * 8, 1)), axis=-1,
                         bitorder="little")
    return bits.reshape(words.shape[:-1] + (words.shape[-1] * 64,))[..., :n].copy()
