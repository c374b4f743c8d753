"""Python face of the CPU oracle (``c2_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the GPU library or its binding.

Every function takes plain numpy arrays (the seeded inputs) and returns numpy
arrays.  ``avg_sim`` and ``quality`` follow Eq. 1 and Eq. 2 of the paper
(average similarity over the k*n edge slots; quality = ratio to the exact
graph), summed with ``math.fsum`` so the result does not depend on order.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c2_oracle.c")
LIB = os.path.join(HERE, "liborc2.so")
PAD = 0xFFFFFFFF

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liborc2.so``."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-pthread", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.orc_validate.argtypes = [u32, u32, P, P]
        L.orc_validate.restype = i32
        L.orc_hash_items.argtypes = [P, u32, u64, u32, P]
        L.orc_frh_keys.argtypes = [u32, u32, P, P, P, u32, P]
        L.orc_cluster.argtypes = [u32, u32, P, P, P, u32, u32, P, P, P]
        L.orc_cluster.restype = i32
        L.orc_cluster_keys.argtypes = [u32, u32, P, P, P, P, u32, u32, P, P, P]
        L.orc_cluster_keys.restype = i32
        L.orc_local_knn.argtypes = [u32, u32, P, P, u32, u32, P, P, P, P, P, i32]
        L.orc_splitmix_at.argtypes = [u64, u64]
        L.orc_splitmix_at.restype = u64
        L.orc_local_knn_alg2.argtypes = [u32, u32, P, P, u32, u32, P, P, P, u32,
                                         ctypes.c_double, u32, u64, P, P, i32]
        L.orc_merge.argtypes = [u32, P, u32, u32, P, P, P, P, P]
        L.orc_brute_force.argtypes = [u32, u32, P, P, u32, P, u32, P, P, P, i32]
        L.orc_candidate_topk.argtypes = [u32, u32, P, P, u32, u32, P, P, P, P, u32,
                                         P, P, P, i32]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Result:
    """Arrays produced by one oracle build."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def validate(indptr, indices, n, m) -> int:
    ip, ix = _c(indptr, np.int64), _c(indices, np.uint32)
    return lib().orc_validate(n, m, _p(ip), _p(ix))


def hash_items(tab: np.ndarray, b: int, m: int) -> np.ndarray:
    """bucket[t][m] = h_j(i)."""
    tab = _c(tab, np.uint64)
    t = tab.shape[0]
    out = np.empty((t, m), dtype=np.uint32)
    lib().orc_hash_items(_p(tab), t, int(b), m, _p(out))
    return out


def frh_keys(indptr, indices, n, m, bucket) -> np.ndarray:
    """keys[t][n] = H_j(u) (Eq. 3)."""
    ip, ix, bk = _c(indptr, np.int64), _c(indices, np.uint32), _c(bucket, np.uint32)
    t = bk.shape[0]
    out = np.empty((t, n), dtype=np.uint32)
    lib().orc_frh_keys(n, m, _p(ip), _p(ix), _p(bk), t, _p(out))
    return out


def cluster(indptr, indices, n, m, bucket, cap):
    """Step 1 with recursive splitting.  Returns (members[t*n], cl_off[ncl+1],
    cl_cfg_off[t+1], max split depth)."""
    ip, ix, bk = _c(indptr, np.int64), _c(indices, np.uint32), _c(bucket, np.uint32)
    t = bk.shape[0]
    members = np.empty(t * n, dtype=np.uint32)
    cl_off = np.empty(t * n + 1, dtype=np.uint32)
    cfg = np.empty(t + 1, dtype=np.uint32)
    depth = lib().orc_cluster(n, m, _p(ip), _p(ix), _p(bk), t, cap, _p(members),
                              _p(cl_off), _p(cfg))
    ncl = int(cfg[t])
    return members, cl_off[: ncl + 1].copy(), cfg, depth


def cluster_keys(indptr, indices, n, m, keys0, bucket, cap):
    """Step 1 with the top-level groups given per user (keys0[t][n], e.g. a
    learned assignment) and FastRandomHash on `bucket` splitting every group
    larger than cap, starting from H_j(u).  Returns as cluster()."""
    ip, ix = _c(indptr, np.int64), _c(indices, np.uint32)
    k0, bk = _c(keys0, np.uint32), _c(bucket, np.uint32)
    t = bk.shape[0]
    members = np.empty(t * n, dtype=np.uint32)
    cl_off = np.empty(t * n + 1, dtype=np.uint32)
    cfg = np.empty(t + 1, dtype=np.uint32)
    depth = lib().orc_cluster_keys(n, m, _p(ip), _p(ix), _p(k0), _p(bk), t, cap, _p(members),
                                   _p(cl_off), _p(cfg))
    ncl = int(cfg[t])
    return members, cl_off[: ncl + 1].copy(), cfg, depth


def local_knn(indptr, indices, n, m, t, k, members, cl_off, cl_cfg_off, threads=1):
    """Step 2: part_id, part_I of shape [n][t][k]."""
    ip, ix = _c(indptr, np.int64), _c(indices, np.uint32)
    mem, off, cfg = _c(members, np.uint32), _c(cl_off, np.uint32), _c(cl_cfg_off, np.uint32)
    pid = np.empty((n, t, k), dtype=np.uint32)
    pI = np.empty((n, t, k), dtype=np.uint32)
    lib().orc_local_knn(n, m, _p(ip), _p(ix), t, k, _p(mem), _p(off), _p(cfg),
                        _p(pid), _p(pI), int(threads))
    return pid, pI


def local_knn_alg2(indptr, indices, n, m, t, k, members, cl_off, cl_cfg_off, rho=5,
                   delta=0.001, max_iter=30, seed=0, threads=1):
    """Step 2 as Algorithm 2: brute force in clusters of fewer than rho*k^2
    members, deterministic Hyrec (seeded SplitMix64 initial graph, synchronous
    neighbours-of-neighbours iterations) in the others."""
    ip, ix = _c(indptr, np.int64), _c(indices, np.uint32)
    mem, off, cfg = _c(members, np.uint32), _c(cl_off, np.uint32), _c(cl_cfg_off, np.uint32)
    pid = np.empty((n, t, k), dtype=np.uint32)
    pI = np.empty((n, t, k), dtype=np.uint32)
    lib().orc_local_knn_alg2(n, m, _p(ip), _p(ix), t, k, _p(mem), _p(off), _p(cfg), int(rho),
                             float(delta), int(max_iter), int(seed), _p(pid), _p(pI), int(threads))
    return pid, pI


def merge(indptr, n, t, k, part_id, part_I):
    """Step 3: knn_id, knn_I, knn_U of shape [n][k]."""
    ip = _c(indptr, np.int64)
    pid, pI = _c(part_id, np.uint32), _c(part_I, np.uint32)
    kid = np.empty((n, k), dtype=np.uint32)
    kI = np.empty((n, k), dtype=np.uint32)
    kU = np.empty((n, k), dtype=np.uint32)
    lib().orc_merge(n, _p(ip), t, k, _p(pid), _p(pI), _p(kid), _p(kI), _p(kU))
    return kid, kI, kU


def brute_force(indptr, indices, n, m, k, rows: Optional[Sequence[int]] = None, threads=1):
    """Exact KNN rows (all users by default): [len(rows)][k] x 3."""
    ip, ix = _c(indptr, np.int64), _c(indices, np.uint32)
    rows = np.arange(n, dtype=np.uint32) if rows is None else _c(rows, np.uint32)
    r = len(rows)
    kid = np.empty((r, k), dtype=np.uint32)
    kI = np.empty((r, k), dtype=np.uint32)
    kU = np.empty((r, k), dtype=np.uint32)
    lib().orc_brute_force(n, m, _p(ip), _p(ix), k, _p(rows), r, _p(kid), _p(kI), _p(kU),
                          int(threads))
    return kid, kI, kU


def candidate_topk(indptr, indices, n, m, t, k, members, cl_off, cl_cfg_off,
                   rows=None, threads=1):
    """The C^2 graph from its definition: top-k over users sharing a final
    cluster with u in some configuration."""
    ip, ix = _c(indptr, np.int64), _c(indices, np.uint32)
    mem, off, cfg = _c(members, np.uint32), _c(cl_off, np.uint32), _c(cl_cfg_off, np.uint32)
    rows = np.arange(n, dtype=np.uint32) if rows is None else _c(rows, np.uint32)
    r = len(rows)
    kid = np.empty((r, k), dtype=np.uint32)
    kI = np.empty((r, k), dtype=np.uint32)
    kU = np.empty((r, k), dtype=np.uint32)
    lib().orc_candidate_topk(n, m, _p(ip), _p(ix), t, k, _p(mem), _p(off), _p(cfg),
                             _p(rows), r, _p(kid), _p(kI), _p(kU), int(threads))
    return kid, kI, kU


def build_graph(indptr, indices, n, m, tab, b, cap, k, threads=1) -> Result:
    """The whole C^2 pipeline: hash, cluster, local KNN, merge."""
    bucket = hash_items(tab, b, m)
    members, cl_off, cfg, depth = cluster(indptr, indices, n, m, bucket, cap)
    t = bucket.shape[0]
    pid, pI = local_knn(indptr, indices, n, m, t, k, members, cl_off, cfg, threads)
    kid, kI, kU = merge(indptr, n, t, k, pid, pI)
    return Result(bucket=bucket, members=members, cl_off=cl_off, cl_cfg_off=cfg,
                  depth=depth, part_id=pid, part_I=pI, knn_id=kid, knn_I=kI, knn_U=kU)


def fingerprints(indptr, indices, n, g):
    """GoldFinger fingerprints (Section II-F): row u is the set of positions
    g[i] over the items i of P_u, as CSR (indptr int64[n+1], ascending rows).
    Written from the definition with numpy, independent of the C oracle."""
    ip = np.asarray(indptr, dtype=np.int64)
    ix = np.asarray(indices, dtype=np.int64)
    g = np.asarray(g, dtype=np.uint32)
    rows = [np.unique(g[ix[ip[u]:ip[u + 1]]]) for u in range(n)]
    fp_ip = np.zeros(n + 1, dtype=np.int64)
    fp_ip[1:] = np.cumsum([len(r) for r in rows])
    fp_ix = np.concatenate(rows).astype(np.uint32) if n else np.zeros(0, np.uint32)
    return fp_ip, fp_ix


def avg_sim(knn_I, knn_U, n_users: Optional[int] = None) -> float:
    """Eq. 1: sum of J over all edge slots divided by k*n; empty slots add 0."""
    kI = np.asarray(knn_I, dtype=np.int64)
    kU = np.asarray(knn_U, dtype=np.int64)
    n, k = kI.shape
    if n_users is None:
        n_users = n
    terms = [float(i) / float(u) for i, u in zip(kI.ravel().tolist(), kU.ravel().tolist()) if u > 0]
    return math.fsum(terms) / (k * n_users)


def quality(approx_I, approx_U, exact_I, exact_U) -> float:
    """Eq. 2: avg_sim(approximate) / avg_sim(exact)."""
    return avg_sim(approx_I, approx_U) / avg_sim(exact_I, exact_U)


def cluster_sets(members, cl_off, cl_cfg_off):
    """Partition as a list (per configuration) of frozensets of users."""
    t = len(cl_cfg_off) - 1
    out = []
    for j in range(t):
        cs = []
        for c in range(int(cl_cfg_off[j]), int(cl_cfg_off[j + 1])):
            cs.append(frozenset(int(x) for x in members[cl_off[c]:cl_off[c + 1]]))
        out.append(cs)
    return out
