"""Oracle of the learned proposal: per-bit features, a 3-layer MLP
(8 -> 64 -> 64 -> 1, ReLU) that turns them into flip-priority logits, its
binary cross-entropy loss, gradients and Adam step, and the two genetic
operations that consume the logits (MLP-seed, MLP-mutate).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/`` and ``__graft_entry__``'s
smoke check; the product package never imports it.

Arithmetic is numpy float64.  The device stores weights, activations and the
gradients fed to its matrix cores in bfloat16 (round to nearest even) with
float32 accumulation; ``rounding=True`` rounds at exactly those points
(weights, layer outputs after ReLU, the back-propagated deltas), so the two
agree up to float32 accumulation order.  ``rounding=False`` is the plain
float64 network, used to pin the gradient formulas by finite differences.

Parameter vector layout (float32 master copy, 4801 values):
W1[64][8] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3.

Features of bit k of a pooled vector X (pool q, rank r, m entries), each a
float32 expression rounded to bfloat16:
  f0 = Delta_k(X) / B          (Delta by the closed form of Eq. (3), B the
                                problem's Delta bound)
  f1 = 2 x_k - 1
  f2 = W_kk / B
  f3 = R_k / B,  R_k = |W_kk| + 2 sum_{j != k} |W_kj|
  f4 = 2 (c_k / m) - 1,  c_k = entries of pool q with bit k set
  f5 = f1 * f4                 (agreement with the pool majority)
  f6 = 2 b_k - 1,  b = the pool's best entry (rank 0)
  f7 = r / m
"""
from __future__ import annotations

import numpy as np

from . import delta_closed, philox

N_FEAT, HID = 8, 64
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 512, 576, 4672, 4736, 4800
N_PARAMS = 4801
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8
TAG_GA, KIND_BITS = 4, 2


# ------------------------------------------------------------------ bfloat16
def bf16(x):
    """float32 -> bfloat16 round-to-nearest-even, returned as float32 values."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u << 16).astype(np.uint32).view(np.float32).reshape(x.shape)


def bf16_bits(x):
    """The 16-bit patterns of bf16(x)."""
    return (bf16(x).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b):
    return (np.asarray(b, dtype=np.uint32) << 16).astype(np.uint32).view(np.float32)


# ------------------------------------------------------------------ params
def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return dict(W1=p[OFF_W1:OFF_B1].reshape(HID, N_FEAT), b1=p[OFF_B1:OFF_W2],
                W2=p[OFF_W2:OFF_B2].reshape(HID, HID), b2=p[OFF_B2:OFF_W3],
                W3=p[OFF_W3:OFF_B3], b3=p[OFF_B3:N_PARAMS])


def pack(d):
    return np.concatenate([d["W1"].ravel(), d["b1"], d["W2"].ravel(), d["b2"], d["W3"], np.atleast_1d(d["b3"])])


def init_params(seed):
    """He-style uniform initialisation (float32), drawn by numpy on the host."""
    rng = np.random.default_rng(seed)
    a1, a2, a3 = np.sqrt(6.0 / N_FEAT), np.sqrt(6.0 / HID), np.sqrt(3.0 / HID)
    d = dict(W1=rng.uniform(-a1, a1, (HID, N_FEAT)), b1=np.zeros(HID), W2=rng.uniform(-a2, a2, (HID, HID)),
             b2=np.zeros(HID), W3=rng.uniform(-a3, a3, HID), b3=np.zeros(1))
    return pack(d).astype(np.float32)


# ------------------------------------------------------------------ features
def row_abs(W):
    """R_k = |W_kk| + 2 sum_{j != k} |W_kj| (int64)."""
    A = np.abs(np.asarray(W, dtype=np.int64))
    return 2 * A.sum(axis=1) - np.diag(A)


def features(W, X, pool_bits, rank):
    """Features (bfloat16 values as float32, shape [n][8]) of vector X (0/1
    uint8, length n) that sits at rank `rank` of a pool whose entries are the
    rows of pool_bits ([m][n] 0/1)."""
    W = np.asarray(W)
    n = W.shape[0]
    X = np.asarray(X, dtype=np.uint8)
    pool_bits = np.asarray(pool_bits, dtype=np.uint8)
    m = pool_bits.shape[0]
    R = row_abs(W)
    B = int(R.max())
    f32 = np.float32
    D = np.asarray(delta_closed(W, X), dtype=np.int64)
    fB = f32(B)
    f = np.zeros((n, N_FEAT), dtype=np.float32)
    f[:, 0] = D.astype(f32) / fB
    f[:, 1] = (2 * X.astype(np.int64) - 1).astype(f32)
    f[:, 2] = np.diag(W).astype(np.int64).astype(f32) / fB
    f[:, 3] = R.astype(f32) / fB
    cnt = pool_bits.astype(np.int64).sum(axis=0)
    f[:, 4] = f32(2) * (cnt.astype(f32) / f32(m)) - f32(1)
    f[:, 5] = f[:, 1] * f[:, 4]
    f[:, 6] = (2 * pool_bits[0].astype(np.int64) - 1).astype(f32)
    f[:, 7] = f32(rank) / f32(m)
    return bf16(f)


def labels(X, ref, symmetric=False):
    """1 where bit k of X differs from the reference; with symmetric, from the
    reference or its complement, whichever is nearer (ties: the reference)."""
    X = np.asarray(X, dtype=np.uint8)
    ref = np.asarray(ref, dtype=np.uint8)
    d = X ^ ref
    if symmetric and 2 * int(d.sum()) > X.shape[0]:
        d = 1 - d
    return d.astype(np.uint8)


# ------------------------------------------------------------------ network
def _r(x, rounding):
    return bf16(x.astype(np.float32)).astype(np.float64) if rounding else x


def forward(params, F, rounding=True, keep=False):
    """Logits (float64) of the samples F ([N][8]).  With rounding, the layer
    outputs are float32 values rounded to bfloat16 after ReLU, as on the
    device, and the logit is a float32 value."""
    P = unpack(params)
    W1, W2, W3 = (_r(P[k], rounding) for k in ("W1", "W2", "W3"))
    F = np.asarray(F, dtype=np.float64)
    z1 = F @ W1.T + P["b1"]
    if rounding:
        z1 = z1.astype(np.float32).astype(np.float64)
    a1 = _r(np.maximum(z1, 0.0), rounding)
    z2 = a1 @ W2.T + P["b2"]
    if rounding:
        z2 = z2.astype(np.float32).astype(np.float64)
    a2 = _r(np.maximum(z2, 0.0), rounding)
    z = a2 @ W3 + P["b3"][0]
    if rounding:
        z = z.astype(np.float32).astype(np.float64)
    if keep:
        return z, dict(F=F, z1=z1, a1=a1, z2=z2, a2=a2, W1=W1, W2=W2, W3=W3)
    return z


def loss(params, F, y, rounding=True):
    """Mean binary cross-entropy with logits: mean(softplus(z) - y z)."""
    z = forward(params, F, rounding)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(np.logaddexp(0.0, z) - y * z))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * np.asarray(z, dtype=np.float64)))


def grad(params, F, y, rounding=True):
    """Gradient of loss() w.r.t. the 4801 parameters (chain rule through the
    three layers; with rounding, the deltas fed to bfloat16 products are
    rounded as on the device)."""
    z, c = forward(params, F, rounding, keep=True)
    y = np.asarray(y, dtype=np.float64)
    N = z.shape[0]
    dz = (sigmoid(z) - y) / N                                  # dL/dz
    if rounding:
        dz = dz.astype(np.float32).astype(np.float64)
    dW3 = c["a2"].T @ dz
    db3 = dz.sum()
    dA2 = np.outer(dz, c["W3"]) * (c["z2"] > 0)                # [N][64]
    db2 = dA2.sum(axis=0)
    dA2r = _r(dA2, rounding)
    dW2 = dA2r.T @ c["a1"]
    dH1 = dA2r @ c["W2"]
    dA1 = dH1 * (c["z1"] > 0)
    db1 = dA1.sum(axis=0)
    dA1r = _r(dA1, rounding)
    dW1 = dA1r.T @ c["F"]
    return pack(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=np.array([db3])))


def adam(params, g, m, v, t, lr):
    """One Adam step (Kingma & Ba), t = 1 for the first step.  Returns new
    (params, m, v)."""
    p = np.asarray(params, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = ADAM_B1 * np.asarray(m, dtype=np.float64) + (1 - ADAM_B1) * g
    v = ADAM_B2 * np.asarray(v, dtype=np.float64) + (1 - ADAM_B2) * g * g
    mh = m / (1 - ADAM_B1 ** t)
    vh = v / (1 - ADAM_B2 ** t)
    return p - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v


# ------------------------------------------------------------------ operations
def ga_bit_u32(seed, rnd, inst, k):
    """Per-bit u32 of the genetic operations' threshold stream (the draw
    (round, instance, k/4, TAG_GA<<24 | KIND_BITS), word k mod 4)."""
    return int(philox([rnd, inst, k // 4, (TAG_GA << 24) | KIND_BITS], seed)[k % 4])


def mlp_seed(parent, logits):
    """MLP-seed: flip every bit whose logit is positive (a float32 compare)."""
    parent = np.asarray(parent, dtype=np.uint8)
    z = np.asarray(logits, dtype=np.float32)
    return parent ^ (z > np.float32(0)).astype(np.uint8)


def mutate_level(logits):
    """q_k = clamp(round-half-even(16 z_k), -128, 127) in float32."""
    z = np.asarray(logits, dtype=np.float32)
    return np.clip(np.rint(z * np.float32(16)), -128, 127).astype(np.int64)


def mlp_mutate(parent, logits, seed, rnd, inst):
    """MLP-mutate: flip bit k when its u32 draw is below 2^29 + q_k 2^22, i.e.
    with probability (1 + q_k/128)/8: the Mutation rate 1/8 tilted by the
    logit."""
    parent = np.asarray(parent, dtype=np.uint8)
    q = mutate_level(logits)
    out = parent.copy()
    for k in range(parent.shape[0]):
        if ga_bit_u32(seed, rnd, inst, k) < (1 << 29) + q[k] * (1 << 22):
            out[k] ^= 1
    return out


def pool_logits(params, W, pool_bits):
    """Logits of every bit of every pooled vector ([P][m][n] 0/1 ->
    float32 [P][m][n]): the features of entry r of pool q (rank r within
    pool q) through the network, as a round with a network attached scores
    its pools before target generation."""
    pool_bits = np.asarray(pool_bits, dtype=np.uint8)
    P, m, n = pool_bits.shape
    out = np.zeros((P, m, n), dtype=np.float32)
    for q in range(P):
        for r in range(m):
            out[q, r] = forward(params, features(W, pool_bits[q, r], pool_bits[q], r)).astype(np.float32)
    return out
