"""Training the learned proposal on solutions the plain search produces.

Host-side orchestration only: every step (the plain DABS rounds, features,
labels, forward, backward, Adam) is a C-ABI call into libdabs.so; this module
loops over them.

Data: a plain solver runs `rounds` generational rounds; every `every` rounds
its pools are snapshotted on the device.  After the run, every snapshotted
entry's bits are labelled against the best vector of the whole run
(label 1 = the bit differs), so the network learns which bits of a pooled
vector the search later ended up flipping.  For problems invariant under
complementing every bit (max-cut) the label is taken against the best vector
or its complement, whichever is nearer.
"""
from __future__ import annotations

import numpy as np

from . import (DABS_MLP_PARAMS, dabs_mlp_create, dabs_mlp_labels, dabs_mlp_pool_features,
               dabs_mlp_train_step, dabs_solver_create, dabs_solver_pools, dabs_solver_run)


def init_params(seed: int) -> np.ndarray:
    """He-style uniform initial parameters (float32, host)."""
    rng = np.random.default_rng(seed)
    a1, a2, a3 = np.sqrt(6.0 / 8), np.sqrt(6.0 / 64), np.sqrt(3.0 / 64)
    p = np.concatenate([rng.uniform(-a1, a1, 512), np.zeros(64), rng.uniform(-a2, a2, 4096), np.zeros(64),
                        rng.uniform(-a3, a3, 64), np.zeros(1)])
    assert p.size == DABS_MLP_PARAMS
    return p.astype(np.float32)


def collect(problem, params, instances: int, rounds: int, every: int, symmetric: bool = False):
    """Runs the plain solver and returns (features [S][8] bf16 as int16,
    labels [S] u8) on the device for all snapshotted pool entries."""
    import torch
    dev = torch.device("cuda:0")
    n, nw = problem.n, problem.nwords
    P, m = params.npools, params.capacity
    s = dabs_solver_create(problem, params, instances)
    snaps = []
    e = torch.zeros((P, m), dtype=torch.int64, device=dev)
    best_e, best_bits = None, None
    for r in range(rounds):
        dabs_solver_run(s, 1)
        if (r + 1) % every == 0 or r == rounds - 1:
            bits = torch.zeros((P, m, nw), dtype=torch.int64, device=dev)
            dabs_solver_pools(s, bits, e)
            snaps.append(bits)
            q = int(torch.argmin(e[:, 0]).item())
            if best_e is None or int(e[q, 0].item()) < best_e:
                best_e, best_bits = int(e[q, 0].item()), bits[q, 0].clone()
    cnt = len(snaps) * P * m
    feats = torch.zeros((cnt, n, 8), dtype=torch.int16, device=dev)
    labels = torch.zeros((cnt, n), dtype=torch.uint8, device=dev)
    for i, b in enumerate(snaps):
        sl = slice(i * P * m, (i + 1) * P * m)
        dabs_mlp_pool_features(problem, b, P, m, feats[sl])
        dabs_mlp_labels(problem, b, P * m, best_bits, labels[sl], symmetric)
    return feats.reshape(-1, 8), labels.reshape(-1), best_e


def fit(feats, labels, *, epochs: int, batch: int, lr: float, seed: int = 0, net=None):
    """Adam on minibatches of consecutive samples, minibatch order shuffled
    per epoch on the host.  Returns (network, mean loss of each epoch)."""
    import torch
    dev = feats.device
    net = net if net is not None else dabs_mlp_create(init_params(seed))
    N = feats.shape[0]
    nb = max(1, N // batch)
    loss = torch.zeros(nb, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    hist = []
    for _ in range(epochs):
        for j, b in enumerate(rng.permutation(nb)):
            lo = int(b) * batch
            hi = N if b == nb - 1 else lo + batch
            dabs_mlp_train_step(net, hi - lo, feats[lo:hi], labels[lo:hi], lr, loss[j:j + 1])
        hist.append(float(loss.mean().item()))
    return net, hist
