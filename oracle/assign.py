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


# ------------------------------------------------------------------ training
#
# The training objective of the assigner (the library's own; the paper has
# none).  A batch is R = 2B profile rows: rows 0..B-1 are users u_i, rows
# B..2B-1 their exact neighbours v_i, and w_i = v_{i-1 mod B} serves as u_i's
# non-neighbour.  With p_r = softmax over head j of z_r (the logits of row r,
# the forward above with e and h rounded to bf16 at the same points):
#
#   s_ij  = <p_{u_i,j}, p_{v_i,j}>,   n_ij = <p_{u_i,j}, p_{w_i,j}>
#   q_j   = mean_r p_{r,j}
#   L = - mean_{i,j} log max(s_ij, 1e-12)
#       - w_neg mean_{i,j} log(1 - clip(n_ij, 0, 1 - 1e-6))
#       + w_bal mean_j sum_c q_jc log(q_jc b + 1e-12)
#       + w_ent mean_{r,j} H(p_{r,j})
#
# The gradients are those of L in float64, with the two bf16 roundings taken
# as the identity (their derivative is zero almost everywhere), and with the
# ReLU's and the clips' derivatives 1 on their closed active ranges.

def train_forward_backward(indptr, indices, m, rows, E, W1, b1, W2, b2, t, b, w_neg=1.0,
                           w_bal=1.0, w_ent=1.0, rounding=True):
    """Loss parts and gradients of one training step from the definition above.
    E, W1, W2 hold the (bf16) values the forward multiplies with; b1, b2 the
    biases.  Returns (loss dict, grads dict with dE, dW1, db1, dW2, db2, and
    the intermediates dict: e, pre, h, z, p, dz, dpre, de).  rounding=False
    drops the two bf16 roundings (for finite-difference checks)."""
    rnd = bf16_round if rounding else (lambda x: np.asarray(x, dtype=np.float64))
    rows = np.asarray(rows, dtype=np.int64)
    R = len(rows)
    B = R // 2
    e = rnd(embag(indptr, indices, E, rows))
    pre = e @ W1.T + b1
    h = rnd(np.maximum(pre, 0.0))
    z = (h @ W2.T + b2).reshape(R, t, b)
    zmax = z.max(axis=-1, keepdims=True)
    ex = np.exp(z - zmax)
    S = ex.sum(axis=-1, keepdims=True)
    p = ex / S
    logp = z - zmax - np.log(S)
    H = -(p * logp).sum(axis=-1)                          # [R, t]
    pu, pv = p[:B], p[B:]
    pw = np.roll(pv, 1, axis=0)                           # row i: v_{i-1}
    s = (pu * pv).sum(axis=-1)
    sn = (pu * pw).sum(axis=-1)                           # [B, t]
    sc = np.maximum(s, 1e-12)
    snc = np.clip(sn, 0.0, 1.0 - 1e-6)
    q = p.mean(axis=0)                                    # [t, b]
    loss = {"pos": float(-np.log(sc).mean()),
            "neg": float(-w_neg * np.log1p(-snc).mean()),
            "bal": float(w_bal * (q * np.log(q * b + 1e-12)).sum(axis=-1).mean()),
            "ent": float(w_ent * H.mean())}
    loss["total"] = loss["pos"] + loss["neg"] + loss["bal"] + loss["ent"]
    # dL/dp
    ds = np.where(s >= 1e-12, -1.0 / (sc * B * t), 0.0)
    dsn = np.where((sn >= 0.0) & (sn <= 1.0 - 1e-6), w_neg / ((1.0 - snc) * B * t), 0.0)
    g = np.zeros_like(p)
    g[:B] += ds[..., None] * pv + dsn[..., None] * pw
    g[B:] += ds[..., None] * pu + np.roll(dsn[..., None] * pu, -1, axis=0)
    g += (w_bal / t * (np.log(q * b + 1e-12) + q * b / (q * b + 1e-12)))[None] / R
    # through the softmax; the entropy's own derivative is -p (log p + H)
    dz = p * (g - (p * g).sum(axis=-1, keepdims=True))
    dz -= w_ent / (R * t) * p * (logp + H[..., None])
    dz = dz.reshape(R, t * b)
    dpre = (dz @ W2) * (pre > 0.0)
    de = dpre @ W1
    grads = {"dW2": dz.T @ h, "db2": dz.sum(axis=0), "dW1": dpre.T @ e, "db1": dpre.sum(axis=0),
             "dE": embag_backward(indptr, indices, m, de, rows)}
    inter = {"e": e, "pre": pre, "h": h, "z": z.reshape(R, t * b), "p": p, "dz": dz,
             "dpre": dpre, "de": de}
    return loss, grads, inter


def adam_step(param, grad, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) in float64, step counted
    from 1: returns (param, m1, m2)."""
    m1 = beta1 * m1 + (1.0 - beta1) * grad
    m2 = beta2 * m2 + (1.0 - beta2) * grad * grad
    mhat = m1 / (1.0 - beta1 ** step)
    vhat = m2 / (1.0 - beta2 ** step)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m1, m2
