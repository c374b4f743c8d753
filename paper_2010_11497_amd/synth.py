"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This module draws random numbers and lays them out; it holds none of the
method's arithmetic (no hashing, no clustering, no similarity).  Both the HIP
path and the CPU oracle receive what it produces as plain arrays.

What it produces
----------------
* Users with item-set profiles in CSR form (``indptr`` int64[n+1], ``indices``
  uint32[nnz], each row strictly increasing).  The paper's data model is a set
  of users, each with a subset of the item universe (Section II-A, "Notations
  and problem definition"); its datasets are binarised rating matrices whose
  users have at least 20 ratings (Section IV-A, Table 1).  The datasets are not
  available here, so synthetic power-law data of the same shape stands in:
    - profile size L_u = clamp(round(exp(N(mu, sigma))), lo, hi) with
      mu = ln(mean) - sigma^2 / 2, so that the unclamped mean is ``mean``;
    - item popularity rank r in [1, m] drawn with P(r) proportional to r^-s;
    - each profile takes the first L_u *distinct* ranks of an i.i.d. stream of
      such draws (successive sampling without replacement);
    - item id = perm[r - 1] for a seeded permutation, so popularity is not
      correlated with item id.
* The random tables of the item hash: ``uint64[t][4][256]`` raw 64-bit words
  from PCG64(hash_seed).  The paper uses t independently seeded generative
  hash functions (Section II-D); the tables are the random numbers the hash
  draws and are passed to both implementations as data.
"""

from __future__ import annotations

import dataclasses
from typing import Dict

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: data shape plus the method's parameters."""

    name: str
    n: int            # users
    m: int            # items
    mean: float       # mean profile size before clamping
    sigma: float      # lognormal sigma of the profile size
    lo: int           # minimum profile size
    hi: int           # maximum profile size
    zipf_s: float     # popularity exponent
    k: int            # neighbours per user
    t: int            # hash functions (clustering configurations)
    b: int            # buckets per hash function
    cap: int          # split threshold N: clusters larger than this are split
    data_seed: int
    hash_seed: int

    def params(self) -> dict:
        return dict(t=self.t, b=self.b, cap=self.cap, k=self.k)


# The five workloads.  Sizes follow the paper's MovieLens shapes where one
# exists (ml1M: 6,038 x 3,533; ml10M: 69,816 x 10,472; ml20M: 138,362 x 22,884
# with N = 4000), rounded.
WORKLOADS: Dict[str, Workload] = {
    w.name: w
    for w in [
        Workload("n2k_m1k", 2000, 1000, 50.0, 0.6, 5, 1000, 1.0,
                 10, 8, 64, 500, 1001, 2001),
        Workload("n6k_m3.7k", 6000, 3700, 165.0, 0.6, 20, 3700, 0.9,
                 30, 8, 1024, 2000, 1002, 2002),
        Workload("n70k_m10k", 70000, 10000, 140.0, 0.6, 20, 10000, 1.1,
                 30, 8, 4096, 2000, 1003, 2003),
        Workload("n140k_m27k", 140000, 27000, 140.0, 0.8, 20, 5000, 1.2,
                 30, 8, 8192, 4000, 1004, 2004),
        Workload("n500k_m50k", 500000, 50000, 80.0, 0.6, 5, 50000, 1.0,
                 30, 8, 8192, 4000, 1005, 2005),
    ]
}


@dataclasses.dataclass
class Profiles:
    n: int
    m: int
    indptr: np.ndarray   # int64[n+1]
    indices: np.ndarray  # uint32[nnz]

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def row(self, u: int) -> np.ndarray:
        return self.indices[self.indptr[u]:self.indptr[u + 1]]

    def lengths(self) -> np.ndarray:
        return np.diff(self.indptr)


def profile_sizes(rng: np.random.Generator, n: int, mean: float, sigma: float,
                  lo: int, hi: int) -> np.ndarray:
    mu = np.log(mean) - 0.5 * sigma * sigma
    raw = np.rint(np.exp(rng.normal(mu, sigma, size=n)))
    return np.clip(raw, lo, hi).astype(np.int64)


def _zipf_cdf(m: int, s: float) -> np.ndarray:
    w = np.arange(1, m + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def _first_distinct(rng, cdf, lengths, m, factor):
    """For each requested length L, draw ``factor*L + 16`` popularity ranks and
    keep the first L distinct ones in draw order.  Returns (ranks per row as a
    flat array ordered row-major, ok mask); rows without enough distinct draws
    are reported as not ok and must be drawn again."""
    nrow = len(lengths)
    draws = factor * lengths + 16
    total = int(draws.sum())
    u = rng.random(total)
    ranks = np.searchsorted(cdf, u, side="right")
    np.minimum(ranks, m - 1, out=ranks)
    rowid = np.repeat(np.arange(nrow, dtype=np.int64), draws)
    key = rowid * m + ranks
    uniq, first = np.unique(key, return_index=True)
    urow = uniq // m
    cnt = np.bincount(urow, minlength=nrow)
    ok = cnt >= lengths
    # order distinct draws of each row by first occurrence
    order = np.lexsort((first, urow))
    urow = urow[order]
    uval = (uniq % m)[order]
    start = np.zeros(nrow + 1, dtype=np.int64)
    start[1:] = np.cumsum(cnt)
    pos = np.arange(len(urow), dtype=np.int64) - start[urow]
    keep = (pos < lengths[urow]) & ok[urow]
    return urow[keep], uval[keep], ok


def sample_profiles(rng: np.random.Generator, lengths: np.ndarray, m: int,
                    s: float, chunk: int = 20000) -> Profiles:
    n = len(lengths)
    cdf = _zipf_cdf(m, s)
    perm = rng.permutation(m).astype(np.uint32)
    indptr = np.zeros(n + 1, dtype=np.int64)
    indptr[1:] = np.cumsum(lengths)
    indices = np.empty(int(indptr[-1]), dtype=np.uint32)
    for c0 in range(0, n, chunk):
        todo = np.arange(c0, min(n, c0 + chunk))
        factor = 3
        while len(todo):
            rows, vals, ok = _first_distinct(rng, cdf, lengths[todo], m, factor)
            items = perm[vals]
            # sort items ascending inside each finished row, then scatter the
            # rows to their CSR slots
            order = np.lexsort((items, rows))
            rows, items = rows[order], items[order]
            first = np.searchsorted(rows, rows, side="left")
            dest = indptr[todo[rows]] + (np.arange(len(rows)) - first)
            indices[dest] = items
            todo = todo[~ok]
            factor *= 2
    return Profiles(n=n, m=m, indptr=indptr, indices=indices)


def make_profiles(w: Workload) -> Profiles:
    rng = np.random.Generator(np.random.PCG64(w.data_seed))
    hi = min(w.hi, w.m)
    lengths = profile_sizes(rng, w.n, w.mean, w.sigma, w.lo, hi)
    return sample_profiles(rng, lengths, w.m, w.zipf_s)


def hash_tables(t: int, seed: int) -> np.ndarray:
    """uint64[t][4][256] random words for t tabulation hash functions.  Tables
    for t' < t are a prefix of those for t (nested seeds)."""
    g = np.random.PCG64(seed)
    return g.random_raw(t * 4 * 256).astype(np.uint64).reshape(t, 4, 256)


def minhash_tables(t: int, m: int, seed: int) -> np.ndarray:
    """uint32[t][m]: t seeded random permutations of the item ids, entry i of
    row j being the rank of item i.  Used as bucket tables with b = m they are
    the min-wise hash functions of MinHash (the paper's MinHash variant of its
    clustering, Section V-C and Table 4)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((t, m), dtype=np.uint32)
    for j in range(t):
        out[j] = rng.permutation(m).astype(np.uint32)
    return out


def random_profiles(seed: int, n: int, m: int, lo: int, hi: int,
                    zipf_s: float = 0.0) -> Profiles:
    """Small random instance for tests: sizes uniform in [lo, hi], items Zipf
    (s = 0 gives uniform items)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lengths = rng.integers(lo, hi + 1, size=n).astype(np.int64)
    lengths = np.minimum(lengths, m)
    return sample_profiles(rng, lengths, m, zipf_s)


def profiles_from_sets(sets, m: int) -> Profiles:
    n = len(sets)
    indptr = np.zeros(n + 1, dtype=np.int64)
    rows = [np.array(sorted(set(int(x) for x in s)), dtype=np.uint32) for s in sets]
    indptr[1:] = np.cumsum([len(r) for r in rows])
    indices = np.concatenate(rows) if n else np.zeros(0, np.uint32)
    return Profiles(n=n, m=m, indptr=indptr, indices=indices.astype(np.uint32))


def bf16_bits_from_normal(rng: np.random.Generator, shape, scale: float) -> np.ndarray:
    """uint16 bfloat16 patterns of seeded normal draws (the float32 draw's high
    half, i.e. truncated): random bf16 values, not a rounding of anything."""
    f = (rng.standard_normal(shape) * scale).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def assigner_weights(m: int, t: int, b: int, seed: int, dim: int = 64, hidden: int = 256):
    """Seeded random weights of the learned assigner: E [m][dim], W1
    [hidden][dim], W2 [t*b][hidden] as bf16 patterns (uint16), b1 [hidden] and
    b2 [t*b] float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    E = bf16_bits_from_normal(rng, (m, dim), 1.0)
    W1 = bf16_bits_from_normal(rng, (hidden, dim), 1.0 / np.sqrt(dim))
    b1 = (rng.standard_normal(hidden) * 0.1).astype(np.float32)
    W2 = bf16_bits_from_normal(rng, (t * b, hidden), 1.0 / np.sqrt(hidden))
    b2 = (rng.standard_normal(t * b) * 0.1).astype(np.float32)
    return E, W1, b1, W2, b2


def assigner_exact_weights(m: int, t: int, b: int, seed: int, dim: int = 64,
                           hidden: int = 256):
    """Seeded assigner weights whose products and sums are all exact in bf16
    and fp32: E holds integers 0..3, each W1 row adds two embedding
    dimensions, each W2 row picks one hidden unit (a seeded choice of b
    units per configuration, distinct when b <= hidden), biases are zero.
    Same layout as assigner_weights."""
    rng = np.random.Generator(np.random.PCG64(seed))
    E = rng.integers(0, 4, size=(m, dim)).astype(np.float32)
    W1 = np.zeros((hidden, dim), dtype=np.float32)
    for r in range(hidden):
        W1[r, rng.choice(dim, size=2, replace=False)] = 1.0
    W2 = np.zeros((t * b, hidden), dtype=np.float32)
    for j in range(t):
        W2[j * b + np.arange(b), rng.choice(hidden, size=b, replace=b > hidden)] = 1.0

    def bits(x):
        return (x.view(np.uint32) >> 16).astype(np.uint16)
    return (bits(E), bits(W1), np.zeros(hidden, dtype=np.float32), bits(W2),
            np.zeros(t * b, dtype=np.float32))


def hidden_inputs(n: int, seed: int, hidden: int = 256) -> np.ndarray:
    """Seeded stand-in for the hidden layer (uint16 bf16 patterns [n][hidden]):
    non-negative, about half exact zeros, as after a ReLU."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = np.abs(rng.standard_normal((n, hidden))).astype(np.float32)
    f[rng.random((n, hidden)) < 0.5] = 0.0
    return (f.view(np.uint32) >> 16).astype(np.uint16)
