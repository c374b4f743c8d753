"""Host-side measurement helpers for graphs and partitions produced on the GPU.

avg_sim and quality follow Eq. 1 and Eq. 2 of the paper (average Jaccard
similarity over the k*n edge slots, empty slots counting 0; quality is the
ratio to the exact graph).  Sums use math.fsum, so they do not depend on
summation order.  cluster_work counts the work units the benchmark's roofline
uses: same-cluster pairs (the paper's similarity computations) and each
cluster's local dictionary size.  edge_jaccard gives the exact intersection and
union of chosen edges, so that a graph built on estimated similarities
(GoldFinger fingerprints) is scored by the users' true similarities.
"""

from __future__ import annotations

import math

import numpy as np


def avg_sim(knn_I: np.ndarray, knn_U: np.ndarray) -> float:
    I = np.asarray(knn_I, dtype=np.int64).ravel()
    U = np.asarray(knn_U, dtype=np.int64).ravel()
    n, k = np.asarray(knn_I).shape
    ok = U > 0
    return math.fsum((I[ok] / U[ok]).tolist()) / (k * n)


def quality(approx_I, approx_U, exact_I, exact_U) -> float:
    return avg_sim(approx_I, approx_U) / avg_sim(exact_I, exact_U)


def cluster_work(members: np.ndarray, cl_off: np.ndarray, indptr: np.ndarray,
                 indices: np.ndarray, m: int) -> dict:
    """Per-cluster sizes s and local dictionary sizes D (items held by at least
    two members), plus the totals the roofline needs:
      pairs        = sum s(s-1)/2  (Jaccard evaluations, Section II-F)
      ordered      = sum s^2
      bitmap_ops   = sum 2 * s^2 * ceil(D/32)   (AND + popcount-accumulate)
      dense_ops    = sum 2 * s^2 * D            (0/1 matrix product)
      sparse_pairs = sum over clusters and items of f(f-1)/2, f = the item's
                     count in the cluster (the intersections' own work: a
                     lower bound for any method that touches only shared items)
    """
    off = np.asarray(cl_off, dtype=np.int64)
    s = np.diff(off)
    indptr = np.asarray(indptr, dtype=np.int64)
    lens = np.diff(indptr)
    mem = np.asarray(members, dtype=np.int64)
    cl_of_slot = np.repeat(np.arange(len(s), dtype=np.int64), s)
    D = np.zeros(len(s), dtype=np.int64)
    sparse = 0
    # clusters in chunks so that the (cluster, item) count table stays small
    chunk = max(1, (1 << 24) // max(m, 1))
    for c0 in range(0, len(s), chunk):
        c1 = min(len(s), c0 + chunk)
        slots = np.arange(off[c0], off[c1])
        users = mem[slots]
        reps = lens[users]
        cl = np.repeat(cl_of_slot[slots] - c0, reps)
        starts = np.repeat(indptr[users], reps)
        within = np.arange(int(reps.sum())) - np.repeat(np.cumsum(reps) - reps, reps)
        items = np.asarray(indices, dtype=np.int64)[starts + within]
        cnt = np.bincount(cl * m + items, minlength=(c1 - c0) * m).reshape(c1 - c0, m)
        D[c0:c1] = (cnt >= 2).sum(axis=1)
        sparse += int((cnt * (cnt - 1) // 2).sum())
    D[s < 2] = 0
    s2 = s * s
    return {
        "clusters": int(len(s)),
        "pairs": int((s * (s - 1) // 2).sum()),
        "ordered": int(s2.sum()),
        "bitmap_ops": int((2 * s2 * ((D + 31) // 32)).sum()),
        "dense_ops": int((2 * s2 * D).sum()),
        "sparse_pairs": sparse,
        "sizes": s,
        "dict": D,
    }


def edge_jaccard(indptr: np.ndarray, indices: np.ndarray, m: int, knn_id: np.ndarray,
                 pad: int = 0xFFFFFFFF, chunk: int = 1 << 16):
    """Exact |P_u & P_v| and |P_u | P_v| for every edge u -> knn_id[u, j]
    (0 and 0 for padded slots), from the profiles packed as bit rows."""
    indptr = np.asarray(indptr, dtype=np.int64)
    n = len(indptr) - 1
    words = (m + 63) // 64
    lens = np.diff(indptr)
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    cols = np.asarray(indices, dtype=np.int64)
    bits = np.zeros((n, words), dtype=np.uint64)
    np.bitwise_or.at(bits, (rows, cols >> 6), np.left_shift(np.uint64(1),
                                                           (cols & 63).astype(np.uint64)))
    ids = np.asarray(knn_id, dtype=np.int64)
    shape = ids.shape
    u = np.repeat(np.arange(n, dtype=np.int64), shape[1])
    v = ids.ravel()
    ok = v != pad
    I = np.zeros(v.shape, dtype=np.int64)
    U = np.zeros(v.shape, dtype=np.int64)
    sel = np.nonzero(ok)[0]
    for c0 in range(0, len(sel), chunk):
        e = sel[c0:c0 + chunk]
        inter = np.bitwise_count(bits[u[e]] & bits[v[e]]).sum(axis=1, dtype=np.int64)
        I[e] = inter
        U[e] = lens[u[e]] + lens[v[e]] - inter
    return I.reshape(shape), U.reshape(shape)


def cluster_work_torch(members, cl_off, cl_cfg_off, indptr, indices, m: int,
                       max_entries: int = 1 << 26) -> dict:
    """cluster_work on torch tensors (any device) for partitions too large for
    its dense count table.  The (cluster, item) entries of one hash
    configuration's clusters are taken in pieces of about max_entries, sorted
    as keys cluster*m + item and counted by runs: a run of length f is an item
    held by f members of that cluster."""
    import torch
    dev = members.device
    off = cl_off.to(torch.int64)
    s = off[1:] - off[:-1]
    ip = indptr.to(torch.int64)
    lens = ip[1:] - ip[:-1]
    mem = members.to(torch.int64)[: int(off[-1])]
    ix = indices.to(torch.int64)
    cs = torch.cat([torch.zeros(1, dtype=torch.int64, device=dev), torch.cumsum(lens[mem], 0)])
    ent = (cs[off[1:]] - cs[off[:-1]]).cpu().numpy()
    cfg = [int(x) for x in cl_cfg_off]
    bounds = []
    for j in range(len(cfg) - 1):
        e = ent[cfg[j]:cfg[j + 1]]
        if len(e) == 0:
            continue
        piece = (np.cumsum(e) - 1) // max_entries
        cut = np.nonzero(np.diff(piece))[0] + 1
        edges = [0] + cut.tolist() + [len(e)]
        bounds += [(cfg[j] + a, cfg[j] + b) for a, b in zip(edges[:-1], edges[1:])]
    D = torch.zeros(len(s), dtype=torch.int64, device=dev)
    sparse = 0
    for c0, c1 in bounds:
        users = mem[int(off[c0]):int(off[c1])]
        reps = lens[users]
        cl = torch.repeat_interleave(torch.arange(c0, c1, device=dev), s[c0:c1])
        cl = torch.repeat_interleave(cl, reps)
        starts = torch.repeat_interleave(ip[users], reps)
        within = torch.arange(int(reps.sum()), device=dev) - torch.repeat_interleave(
            torch.cumsum(reps, 0) - reps, reps)
        keys, _ = torch.sort(cl * m + ix[starts + within])
        run, f = torch.unique_consecutive(keys, return_counts=True)
        D += torch.bincount(run[f >= 2] // m, minlength=len(s))
        sparse += int((f * (f - 1) // 2).sum())
    D[s < 2] = 0
    s2 = s * s
    return {
        "clusters": int(len(s)),
        "pairs": int((s * (s - 1) // 2).sum()),
        "ordered": int(s2.sum()),
        "bitmap_ops": int((2 * s2 * ((D + 31) // 32)).sum()),
        "dense_ops": int((2 * s2 * D).sum()),
        "sparse_pairs": sparse,
        "sizes": s.cpu().numpy(),
        "dict": D.cpu().numpy(),
    }
