"""Learned cluster assigner: training on exact KNN edges, and use in place of
FastRandomHash's top-level grouping.

The paper groups users by FastRandomHash only; this assigner is the library's
own addition.  Per configuration j it predicts a bucket for user u from an
embedding bag over u's items and a two-layer MLP (include/c2.h,
c2_assign_hidden / c2_assign_keys).  FastRandomHash stays in place twice:
users whose top logit does not clear the second by `min_gap` take their
FastRandomHash bucket (offset by b so the two key spaces stay apart), and
groups larger than the cap are split by FastRandomHash (c2_cluster_keys).
Local KNN and merge are unchanged, so the graph keeps the exact arithmetic.

Training (on the GPU, every step in the library's kernels): positive pairs
are exact KNN edges of a user subsample (c2_brute_force).  For pair (u, v)
and head j with bucket distributions p_j(u) = softmax(z_u[j*b:(j+1)*b]) the
loss is
    - log sum_c p_j(u,c) p_j(v,c)                 (collide with neighbours)
    - w_neg * log(1 - sum_c p_j(u,c) p_j(w,c))    (w: in-batch non-neighbour)
    + w_bal * sum_c q_j(c) log(q_j(c) b)          (use all buckets; q the batch mean)
    + w_ent * H(p_j(u))                           (be confident)
averaged over heads and pairs (include/c2.h, c2_assign_train_grad).  The
forward, loss and backward run as one call of the library (bf16 MFMA
products, fp32 softmax statistics), and the update as c2_adam_step on fp32
master weights, which also writes the bf16 copies the next forward and the
inference read.  Batches are drawn on the host from a seeded generator and
uploaded once.
"""

from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import c2

DIM, HIDDEN = c2.ASSIGN_DIM, c2.ASSIGN_HIDDEN


@dataclass
class TrainStats:
    steps: int
    seconds: float
    pairs: int
    first_loss: float
    last_loss: float


def _bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bf16 patterns, round to nearest even."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


class Assigner:
    """fp32 master weights (E, W1, b1, W2, b2) and the bf16 copies of E, W1,
    W2 that the kernels read, on the GPU."""

    def __init__(self, m: int, t: int, b: int, seed: int = 0, device="cuda"):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.m, self.t, self.b = m, t, b
        host = {"E": rng.standard_normal((m, DIM)) * 0.5,
                "W1": rng.standard_normal((HIDDEN, DIM)) / DIM ** 0.5,
                "b1": np.zeros(HIDDEN),
                "W2": rng.standard_normal((t * b, HIDDEN)) / HIDDEN ** 0.5,
                "b2": np.zeros(t * b)}
        self.master = {k: torch.from_numpy(v.astype(np.float32)).to(device) for k, v in host.items()}
        self.bf16 = {k: torch.from_numpy(_bf16_bits(host[k].astype(np.float32)).view(np.int16))
                     .to(device).view(torch.bfloat16) for k in ("E", "W1", "W2")}

    def inference_weights(self):
        """(E, W1, b1, W2, b2) as the kernels take them: bf16 matrices, fp32 biases."""
        return (self.bf16["E"], self.bf16["W1"], self.master["b1"], self.bf16["W2"],
                self.master["b2"])

    def keys(self, P: c2.DeviceProfiles, frh_keys: Optional[torch.Tensor] = None,
             min_gap: float = 0.0, weights=None, with_gap=False):
        E, W1, b1, W2, b2 = weights or self.inference_weights()
        h = c2.assign_hidden(P, E, W1, b1)
        return c2.assign_keys(h, W2, b2, self.t, self.b, frh_keys, min_gap, with_gap)


def subsample(P, rows: np.ndarray):
    """CSR of the listed users (host arrays in, host arrays out)."""
    ip = np.asarray(P.indptr, dtype=np.int64)
    lens = ip[rows + 1] - ip[rows]
    sub_ip = np.zeros(len(rows) + 1, dtype=np.int64)
    sub_ip[1:] = np.cumsum(lens)
    starts = np.repeat(ip[rows], lens)
    within = np.arange(int(sub_ip[-1])) - np.repeat(sub_ip[:-1], lens)
    return sub_ip, np.asarray(P.indices)[starts + within]


def exact_pairs(P, n_sub: int, k: int, seed: int = 0):
    """Exact KNN edges (u, v) among a seeded subsample of n_sub users, in the
    full data's user ids, from the library's brute force."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = np.sort(rng.choice(P.n, size=min(n_sub, P.n), replace=False)).astype(np.int64)
    ip, ix = subsample(P, rows)
    sP = c2.DeviceProfiles(ip, ix, len(rows), P.m)
    kid, _, _ = c2.brute_force(sP, k)
    ids = c2.to_u32(kid).astype(np.int64)
    u = np.repeat(np.arange(len(rows)), k)
    v = ids.ravel()
    ok = v != c2.C2_PAD
    return np.stack([rows[u[ok]], rows[v[ok]]], axis=1)


def train(A: Assigner, P: c2.DeviceProfiles, pairs: np.ndarray, steps: int = 400,
          batch: int = 1024, lr: float = 3e-3, w_neg: float = 1.0, w_bal: float = 3.0,
          w_ent: float = 1.0, seed: int = 0, log=None) -> TrainStats:
    """Adam on the objective above, `steps` batches of `batch` pairs drawn with
    replacement from `pairs` (host array [npairs][2] of user ids)."""
    dev = P.device
    rng = np.random.Generator(np.random.PCG64(seed))
    sel = rng.integers(0, pairs.shape[0], size=(steps, batch))
    rows = np.concatenate([pairs[sel, 0], pairs[sel, 1]], axis=1).astype(np.uint32)
    rows_d = torch.from_numpy(rows.view(np.int32)).to(dev)
    t, b = A.t, A.b
    names = ("E", "W1", "b1", "W2", "b2")
    ws = c2.train_workspace(2 * batch, t, b, dev)
    loss = torch.empty(5, dtype=torch.float32, device=dev)
    g = {k: torch.empty_like(A.master[k]) for k in names}
    m1 = {k: torch.zeros_like(A.master[k]) for k in names}
    m2 = {k: torch.zeros_like(A.master[k]) for k in names}
    out = (loss, g["E"], g["W1"], g["b1"], g["W2"], g["b2"])
    first = last = float("nan")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(steps):
        E, W1, b1, W2, b2 = A.inference_weights()
        c2.assign_train_grad(P, rows_d[step], E, W1, b1, W2, b2, t, b, w_neg, w_bal, w_ent,
                             ws=ws, out=out)
        for k in names:
            c2.adam_step(A.master[k], g[k], m1[k], m2[k], lr, step + 1,
                         param_bf16=A.bf16.get(k))
        if step == 0:
            first = float(loss[0])
        if log and (step % 100 == 0 or step == steps - 1):
            v = loss.tolist()
            log("train step %d loss %.4f (pos %.4f neg %.4f bal %.4f ent %.4f)" % (step, *v))
    last = float(loss[0])
    torch.cuda.synchronize()
    return TrainStats(steps, time.perf_counter() - t0, int(pairs.shape[0]), first, last)


def build(A: Assigner, P: c2.DeviceProfiles, tab: torch.Tensor, p: c2.Params,
          min_gap: float = 0.0, form=c2.FORM_PLAIN, tune: Optional[c2.Tuning] = None,
          weights=None, check: bool = True, with_ws: bool = False,
          knn_ws: Optional[torch.Tensor] = None):
    """The learned-assignment build: keys (FastRandomHash fallback below
    min_gap), clustering from keys with FastRandomHash splits, local KNN,
    merge.  p.b is FastRandomHash's bucket count; the keys span 2*max(b, A.b).
    In the batched form nothing waits on the host, so the call can be captured
    in a graph: pass check=False and a local-KNN workspace large enough for the
    partition (knn_ws, e.g. from c2.local_knn_workspace on an eager run), and
    call c2.check_complete on both workspaces (with_ws=True returns them:
    clustering, local KNN) after each replay.  With check=True the batched
    form checks both, growing the local-KNN store once if it was too small."""
    bucket = c2.hash_items(tab, p.b, P.m)
    frh = c2.frh_keys(P, bucket) if min_gap > 0 else None
    keys = A.keys(P, frh, min_gap, weights)
    kb = 2 * max(p.b, A.b)
    pk = c2.params(p.t, kb, p.cap, p.k)
    members, cl_off, cfg, ws = c2.cluster_keys(P, keys, bucket, pk, form, tune)
    if form == c2.FORM_BATCHED and check:
        c2.check_complete(ws)   # enough split rounds were enqueued (synchronous)
    if form == c2.FORM_PLAIN:
        # the plain form reports a small store synchronously (and the binding
        # grows a workspace it allocated itself)
        kws = knn_ws
        part = c2.local_knn(P, members, cl_off, cfg, pk, form, tune, ws=kws)
    else:
        kws = c2.workspace(P, pk, c2.OP_LOCAL_KNN) if knn_ws is None else knn_ws
        part = c2.local_knn(P, members, cl_off, cfg, pk, form, tune, ws=kws)
        if check:
            try:
                c2.check_complete(kws)
            except c2.C2Error as e:
                if e.status != c2.C2_E_WORKSPACE or knn_ws is not None:
                    raise
                kws = torch.empty(kws.numel() + c2.store_need_bytes(kws), dtype=torch.uint8,
                                  device=kws.device)
                part = c2.local_knn(P, members, cl_off, cfg, pk, form, tune, ws=kws)
                c2.check_complete(kws)
    out = c2.merge(P, part[0], part[1], pk)
    return (out, ws, kws) if with_ws else out
