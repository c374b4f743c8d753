"""CPU oracle of the learned cluster assigner (embedding bag + two-layer MLP,
one argmax per hash configuration) and of its embedding-bag training step.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the GPU
library or its binding.

The paper has no learned assigner; this model is the library's own, defined
as follows and computed here in float64 from that definition:

    e_u = bf16( mean_{i in P_u} E[i] )
    h_u = bf16( ReLU(W1 e_u + b1) )
    z_u = W2 h_u + b2
    key_j(u) = argmax_{c < b} z_u[j*b + c]  (lowest c on ties)
    gap_j(u) = top-1 minus top-2 value of z_u over head j

bf16() rounds to the nearest bfloat16 value, ties to even (8 significant
bits).  Weights are given as float64 arrays holding bf16 values.
"""

from __future__ import annotations

import numpy as np

DIM, HIDDEN = 64, 256


def bf16_round(x) -> np.ndarray:
    """Nearest bfloat16 (8-bit significand), ties to even, for finite x
    in the normal range; computed directly from float64 (no float32 step)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                 # x = m * 2^e, 0.5 <= |m| < 1
    scale = np.ldexp(1.0, e - 8)       # spacing of 8-bit significands at x
    return np.round(x / scale) * scale  # np.round: half to even


def bf16_bits(x) -> np.ndarray:
    """uint16 patterns of values that are exactly bf16."""
    f = np.asarray(x, dtype=np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(
        np.float64)


def embag(indptr, indices, E, rows=None) -> np.ndarray:
    """mean of E rows over the items of each listed user (float64)."""
    ip = np.asarray(indptr, dtype=np.int64)
    ix = np.asarray(indices, dtype=np.int64)
    rows = np.arange(len(ip) - 1) if rows is None else np.asarray(rows, dtype=np.int64)
    out = np.zeros((len(rows), E.shape[1]))
    for r, u in enumerate(rows):
        items = ix[ip[u]:ip[u + 1]]
        if len(items):
            out[r] = E[items].sum(axis=0) / len(items)
    return out


def embag_backward(indptr, indices, m, grad, rows=None) -> np.ndarray:
    """dE of sum_r <grad[r], embag(r)>: item i of row r receives grad[r]/|P_u|."""
    ip = np.asarray(indptr, dtype=np.int64)
    ix = np.asarray(indices, dtype=np.int64)
    rows = np.arange(len(grad)) if rows is None else np.asarray(rows, dtype=np.int64)
    dE = np.zeros((m, grad.shape[1]))
    for r, u in enumerate(rows):
        items = ix[ip[u]:ip[u + 1]]
        if len(items):
            dE[items] += grad[r] / len(items)
    return dE


def hidden(indptr, indices, E, W1, b1):
    """(e, h): the rounded bag means and the rounded hidden layer."""
    e = bf16_round(embag(indptr, indices, E))
    pre = e @ W1.T + b1
    return e, bf16_round(np.maximum(pre, 0.0))


def logits(h, W2, b2) -> np.ndarray:
    return h @ W2.T + b2


def keys(h, W2, b2, t, b):
    """(key[t][n], gap[t][n], z) from the definition."""
    z = logits(h, W2, b2)
    n = h.shape[0]
    key = np.empty((t, n), dtype=np.uint32)
    gap = np.empty((t, n))
    for j in range(t):
        zj = z[:, j * b:(j + 1) * b]
        key[j] = np.argmax(zj, axis=1)            # first maximum: lowest index
        top2 = np.partition(zj, b - 2, axis=1)[:, b - 2:]
        gap[j] = top2[:, 1] - top2[:, 0]
    return key, gap, z
