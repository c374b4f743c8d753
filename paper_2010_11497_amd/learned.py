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

Training (on the GPU): positive pairs are exact KNN edges of a user subsample
(c2_brute_force).  For pair (u, v) and head j with bucket distributions
p_j(u) = softmax(z_u[j*b:(j+1)*b]) the loss is
    - log sum_c p_j(u,c) p_j(v,c)                 (collide with neighbours)
    - w_neg * log(1 - sum_c p_j(u,c) p_j(w,c))    (w: in-batch non-neighbour)
    + w_bal * KL(mean_u p_j(u) || uniform)        (use all buckets)
    + w_ent * H(p_j(u))                           (be confident)
averaged over heads and pairs.  The embedding bag runs through the library's
HIP kernels (c2_embag, c2_embag_backward); the two dense layers and the
softmax go through torch.  Weights are fp32 masters updated by Adam; the
forward reads a bf16 copy of E, and inference uses bf16 copies of all
matrices.
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


class Assigner:
    def __init__(self, m: int, t: int, b: int, seed: int = 0, device="cuda"):
        g = torch.Generator(device="cpu").manual_seed(seed)
        self.m, self.t, self.b = m, t, b
        self.E = (torch.randn(m, DIM, generator=g) * 0.5).to(device).requires_grad_()
        self.W1 = (torch.randn(HIDDEN, DIM, generator=g) / DIM ** 0.5).to(device).requires_grad_()
        self.b1 = torch.zeros(HIDDEN, device=device, requires_grad=True)
        self.W2 = (torch.randn(t * b, HIDDEN, generator=g) / HIDDEN ** 0.5).to(device).requires_grad_()
        self.b2 = torch.zeros(t * b, device=device, requires_grad=True)

    def params(self):
        return [self.E, self.W1, self.b1, self.W2, self.b2]

    def inference_weights(self):
        """(E, W1, b1, W2, b2) as the kernels take them: bf16 matrices, fp32 biases."""
        with torch.no_grad():
            return (self.E.detach().to(torch.bfloat16).contiguous(),
                    self.W1.detach().to(torch.bfloat16).contiguous(), self.b1.detach().contiguous(),
                    self.W2.detach().to(torch.bfloat16).contiguous(), self.b2.detach().contiguous())

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
    dev = P.device
    pairs_d = torch.from_numpy(pairs.astype(np.int32)).to(dev)
    opt = torch.optim.Adam(A.params(), lr=lr)
    gen = torch.Generator(device=dev).manual_seed(seed)
    t, b = A.t, A.b
    first = last = float("nan")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(steps):
        sel = torch.randint(0, pairs_d.shape[0], (batch,), device=dev, generator=gen)
        rows = torch.cat([pairs_d[sel, 0], pairs_d[sel, 1]]).contiguous()
        E16 = A.E.detach().to(torch.bfloat16).contiguous()
        e = c2.embag(P, E16, rows).requires_grad_()
        h = torch.relu(e @ A.W1.t() + A.b1)
        z = (h @ A.W2.t() + A.b2).view(2 * batch, t, b)
        p = torch.softmax(z, dim=-1)
        ent = -(p * torch.log_softmax(z, dim=-1)).sum(-1).mean()
        pu, pv = p[:batch], p[batch:]
        pos = (pu * pv).sum(-1).clamp_min(1e-12)
        neg = (pu * pv.roll(1, dims=0)).sum(-1).clamp(0.0, 1.0 - 1e-6)
        q = p.mean(0)
        bal = (q * torch.log(q * b + 1e-12)).sum(-1).mean()
        loss = (-torch.log(pos).mean() - w_neg * torch.log1p(-neg).mean() + w_bal * bal
                + w_ent * ent)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        dE = torch.zeros_like(A.E)
        c2.embag_backward(P, e.grad.contiguous(), dE, rows)
        A.E.grad = dE
        opt.step()
        if step == 0:
            first = float(loss.detach())
        if log and (step % 100 == 0 or step == steps - 1):
            log("train step %d loss %.4f (pos %.4f neg %.4f bal %.4f ent %.4f)"
                % (step, float(loss.detach()), float(-torch.log(pos).mean().detach()),
                   float(-torch.log1p(-neg).mean().detach()), float(bal.detach()),
                   float(ent.detach())))
    last = float(loss.detach())
    torch.cuda.synchronize()
    return TrainStats(steps, time.perf_counter() - t0, int(pairs.shape[0]), first, last)


def build(A: Assigner, P: c2.DeviceProfiles, tab: torch.Tensor, p: c2.Params,
          min_gap: float = 0.0, form=c2.FORM_PLAIN, tune: Optional[c2.Tuning] = None,
          weights=None, check: bool = True, with_ws: bool = False):
    """The learned-assignment build: keys (FastRandomHash fallback below
    min_gap), clustering from keys with FastRandomHash splits, local KNN,
    merge.  p.b is FastRandomHash's bucket count; the keys span 2*max(b, A.b).
    In the batched form nothing waits on the host, so the call can be captured
    in a graph: pass check=False there and call c2.check_complete on the
    clustering workspace (with_ws=True returns it) after each replay."""
    bucket = c2.hash_items(tab, p.b, P.m)
    frh = c2.frh_keys(P, bucket) if min_gap > 0 else None
    keys = A.keys(P, frh, min_gap, weights)
    kb = 2 * max(p.b, A.b)
    pk = c2.params(p.t, kb, p.cap, p.k)
    members, cl_off, cfg, ws = c2.cluster_keys(P, keys, bucket, pk, form, tune)
    if form == c2.FORM_BATCHED and check:
        c2.check_complete(ws)   # enough split rounds were enqueued (synchronous)
    part = c2.local_knn(P, members, cl_off, cfg, pk, form, tune)
    out = c2.merge(P, part[0], part[1], pk)
    return (out, ws) if with_ws else out
