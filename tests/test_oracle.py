"""Pins for the CPU oracle, against what the paper and mathematics fix.

None of these compare the oracle with itself: expected values come from the
paper's worked examples (fixtures under tests/golden/), from an exhaustive
rational brute force written independently here, from a different formulation
of the same clustering (a prefix trie over each user's sorted hash values),
from closed forms (Theorem 2's example), from special cases that reduce to a
textbook routine (identity tables: the hash is the item id, FastRandomHash is
the minimum), and from invariants (partition, monotonicity, quality <= 1).
"""
import json
import math
import os
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest

from paper_2010_11497_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PAD = 0xFFFFFFFF


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def csr(profiles):
    P = synth.profiles_from_sets(profiles, 1 + max(max(p) for p in profiles))
    return P.indptr, P.indices


# ------------------------------------------------------------------ helpers --

def exact_knn(sets, k, cand=None):
    """Exhaustive exact KNN with rational J, ties to the smaller id."""
    n = len(sets)
    out = []
    for u in range(n):
        pool = range(n) if cand is None else cand[u]
        rows = []
        for v in pool:
            if v == u:
                continue
            I = len(sets[u] & sets[v])
            U = len(sets[u] | sets[v])
            rows.append((-Fraction(I, U), v, I, U))
        rows.sort()
        rows = rows[:k]
        ids = [r[1] for r in rows] + [PAD] * (k - len(rows))
        Is = [r[2] for r in rows] + [0] * (k - len(rows))
        Us = [r[3] for r in rows] + [0] * (k - len(rows))
        out.append((ids, Is, Us))
    return (np.array([o[0] for o in out], dtype=np.uint32),
            np.array([o[1] for o in out], dtype=np.uint32),
            np.array([o[2] for o in out], dtype=np.uint32))


def trie_partition(sets, bucket_row, cap):
    """The split rule restated as a prefix trie: a user's cluster path is a
    prefix of its sorted distinct hash values; a node holding more than cap
    users is split by the next value; users with no next value or alone with
    theirs stay in the node.  Returns clusters in the order children (by
    value) before the users that stayed."""
    seqs = [tuple(sorted(set(bucket_row[i] for i in s))) for s in sets]
    count = Counter()
    for q in seqs:
        for d in range(1, len(q) + 1):
            count[q[:d]] += 1
    keys = []
    for q in seqs:
        d = 1
        while True:
            node = q[:d]
            if d == 1 and count[node] <= cap:
                keys.append(node)
                break
            if d > 1 and count[node] <= cap:
                keys.append(node)
                break
            # node is split
            if d == len(q):
                keys.append(node + (math.inf,))
                break
            child = q[: d + 1]
            if count[child] == 1:
                keys.append(node + (math.inf,))
                break
            d += 1
    groups = {}
    for u, key in enumerate(keys):
        groups.setdefault(key, []).append(u)
    return [groups[key] for key in sorted(groups)]


def oracle_sets(members, cl_off, cl_cfg_off, j):
    return [sorted(int(x) for x in members[cl_off[c]:cl_off[c + 1]])
            for c in range(int(cl_cfg_off[j]), int(cl_cfg_off[j + 1]))]


# ------------------------------------------------------------ worked example --

def test_frh_worked_example(orc):
    g = load("frh_worked_example.json")
    ip, ix = csr(g["profiles"])
    bucket = np.array(g["bucket"], dtype=np.uint32)
    keys = orc.frh_keys(ip, ix, 2, g["m"], bucket)
    assert keys.tolist() == g["expected_keys"]
    members, cl_off, cfg, _ = orc.cluster(ip, ix, 2, g["m"], bucket, cap=10)
    for j in range(2):
        assert oracle_sets(members, cl_off, cfg, j) == g["expected_clusters_per_config"][j]
    pid, pI = orc.local_knn(ip, ix, 2, g["m"], 2, 1, members, cl_off, cfg)
    kid, kI, kU = orc.merge(ip, 2, 2, 1, pid, pI)
    e = g["expected_knn"]
    assert kid.tolist() == e["id"] and kI.tolist() == e["I"] and kU.tolist() == e["U"]
    # in configuration 1 they are apart: padding
    assert pid[0, 0, 0] == PAD and pid[0, 1, 0] == 1


@pytest.mark.parametrize("name", ["fig3_split.json", "singleton_stays.json"])
def test_split_fixtures(orc, name):
    g = load(name)
    n = len(g["profiles"])
    P = synth.profiles_from_sets(g["profiles"], g["m"])
    bucket = np.array(g["bucket"], dtype=np.uint32)
    members, cl_off, cfg, depth = orc.cluster(P.indptr, P.indices, n, g["m"], bucket, g["cap"])
    got = oracle_sets(members, cl_off, cfg, 0)
    assert got == g["expected_clusters"]
    assert [len(c) for c in got] == g["expected_sizes"]
    assert depth == 1


# ---------------------------------------------------------------- hashing --

def identity_tables(t=1):
    T = np.zeros((t, 4, 256), dtype=np.uint64)
    for c in range(4):
        T[:, c, :] = (np.arange(256, dtype=np.uint64) << np.uint64(8 * c + 32))
    return T


def test_hash_identity_tables(orc):
    # x = i << 32; with b = 2^32 the bucket is the item id itself, with
    # b = 2^q it is the top q bits of the 32-bit id
    m = 70000
    T = identity_tables()
    assert np.array_equal(orc.hash_items(T, 2 ** 32, m)[0], np.arange(m, dtype=np.uint32))
    for q in (1, 5, 17):
        assert np.array_equal(orc.hash_items(T, 2 ** q, m)[0],
                              (np.arange(m, dtype=np.uint64) >> np.uint64(32 - q)).astype(np.uint32))
    # FastRandomHash with the identity hash is the smallest item of the profile
    P = synth.random_profiles(3, 50, m, 1, 40)
    keys = orc.frh_keys(P.indptr, P.indices, P.n, m, orc.hash_items(T, 2 ** 32, m))
    assert keys[0].tolist() == [int(P.row(u).min()) for u in range(P.n)]


def test_hash_uniform_and_in_range(orc):
    m, b = 200000, 1000
    tab = synth.hash_tables(3, 99)
    bk = orc.hash_items(tab, b, m)
    assert bk.max() < b
    for j in range(3):
        cnt = np.bincount(bk[j], minlength=b)
        chi2 = float(((cnt - m / b) ** 2 / (m / b)).sum())
        # chi-square with b-1 dof: mean 999, sd ~44.7; 6 sd bound
        assert chi2 < 999 + 6 * 44.7, chi2
    # different seeds give different functions
    assert not np.array_equal(bk[0], bk[1])


# --------------------------------------------------------- exact KNN, ties --

def tiny_instances():
    out = []
    for seed in range(6):
        P = synth.random_profiles(100 + seed, 40, 25, 1, 8)
        out.append([set(P.row(u).tolist()) for u in range(P.n)])
    # adversarial: identical, nested, disjoint profiles -> many equal J
    out.append([{1, 2, 3}] * 6 + [{1, 2}, {1}, {4}, {5, 6}, {4, 5, 6}, {1, 2, 3, 4}])
    out.append([{i} for i in range(10)] + [{0, 1}, {2, 3}])
    return out


@pytest.mark.parametrize("case", range(8))
@pytest.mark.parametrize("k", [1, 3, 7])
def test_brute_force_vs_rational(orc, case, k):
    sets = tiny_instances()[case]
    m = 1 + max(max(s) for s in sets)
    P = synth.profiles_from_sets(sets, m)
    got = orc.brute_force(P.indptr, P.indices, P.n, m, k)
    want = exact_knn(sets, k)
    for a, b in zip(got, want):
        assert np.array_equal(a, b)


# ------------------------------------------------------------ clustering --

def small_workload(seed, n=300, m=120, b=16, cap=40, t=3, zipf=1.0, lo=1, hi=20):
    P = synth.random_profiles(seed, n, m, lo, hi, zipf)
    tab = synth.hash_tables(t, seed + 7)
    return P, tab, b, cap


@pytest.mark.parametrize("seed,b,cap", [(1, 16, 40), (2, 8, 10), (3, 64, 5), (4, 4, 100),
                                        (5, 2, 3), (6, 128, 1), (7, 16, 2)])
def test_partition_matches_trie(orc, seed, b, cap):
    P, tab, b, cap = small_workload(seed, b=b, cap=cap)
    bucket = orc.hash_items(tab, b, P.m)
    members, cl_off, cfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, bucket, cap)
    sets = [set(P.row(u).tolist()) for u in range(P.n)]
    for j in range(tab.shape[0]):
        got = oracle_sets(members, cl_off, cfg, j)
        assert sorted(sum(got, [])) == list(range(P.n))        # a partition
        assert got == trie_partition(sets, bucket[j].tolist(), cap)


def test_identical_profiles_single_cluster(orc):
    sets = [{3, 5, 9, 11}] * 50
    P = synth.profiles_from_sets(sets, 12)
    tab = synth.hash_tables(2, 5)
    bucket = orc.hash_items(tab, 4, 12)
    members, cl_off, cfg, _ = orc.cluster(P.indptr, P.indices, 50, 12, bucket, 10)
    assert np.array_equal(np.diff(cl_off.astype(np.int64)), [50, 50])


# -------------------------------------------- local KNN + merge = definition --

@pytest.mark.parametrize("seed,b,cap,k", [(11, 16, 40, 5), (12, 8, 15, 10), (13, 64, 30, 3),
                                          (14, 4, 200, 8)])
def test_merge_equals_candidate_definition(orc, seed, b, cap, k):
    P, tab, b, cap = small_workload(seed, b=b, cap=cap)
    r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, b, cap, k)
    sets = [set(P.row(u).tolist()) for u in range(P.n)]
    t = tab.shape[0]
    cand = [set() for _ in range(P.n)]
    for j in range(t):
        for c in range(int(r.cl_cfg_off[j]), int(r.cl_cfg_off[j + 1])):
            mem = [int(x) for x in r.members[r.cl_off[c]:r.cl_off[c + 1]]]
            for u in mem:
                cand[u].update(mem)
    want = exact_knn(sets, k, cand=[sorted(c) for c in cand])
    for a, w in zip((r.knn_id, r.knn_I, r.knn_U), want):
        assert np.array_equal(a, w)
    d = orc.candidate_topk(P.indptr, P.indices, P.n, P.m, t, k, r.members, r.cl_off, r.cl_cfg_off)
    for a, w in zip(d, want):
        assert np.array_equal(a, w)


@pytest.mark.parametrize("n,cap", [(60, 100), (60, 7)])
def test_one_bucket_is_brute_force(orc, n, cap):
    P = synth.random_profiles(21, n, 40, 1, 10, 0.8)
    tab = synth.hash_tables(3, 4)
    k = 6
    r = orc.build_graph(P.indptr, P.indices, n, P.m, tab, 1, cap, k)
    assert np.array_equal(np.diff(r.cl_off.astype(np.int64)), [n] * 3)
    bf = orc.brute_force(P.indptr, P.indices, n, P.m, k)
    for a, w in zip((r.knn_id, r.knn_I, r.knn_U), bf):
        assert np.array_equal(a, w)


def per_user_sum(kI, kU):
    return [sum((Fraction(int(i), int(u)) for i, u in zip(ri, ru) if u), Fraction(0))
            for ri, ru in zip(kI, kU)]


def test_quality_monotone_in_t_and_cap(orc):
    P = synth.random_profiles(31, 400, 150, 3, 25, 1.0)
    k = 8
    bf = orc.brute_force(P.indptr, P.indices, P.n, P.m, k)
    best = per_user_sum(bf[1], bf[2])
    prev = None
    for t in (1, 2, 4, 8):          # nested tables: t' < t is a prefix
        tab = synth.hash_tables(t, 77)
        r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, 32, 30, k)
        cur = per_user_sum(r.knn_I, r.knn_U)
        assert all(c <= e for c, e in zip(cur, best))      # quality <= 1 per user
        if prev is not None:
            assert all(c >= p for c, p in zip(cur, prev))
        prev = cur
    prev = None
    tab = synth.hash_tables(4, 78)
    for cap in (5, 20, 60, 400):
        r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, 32, cap, k)
        cur = per_user_sum(r.knn_I, r.knn_U)
        if prev is not None:
            assert all(c >= p for c, p in zip(cur, prev))
        prev = cur
    q = orc.quality(r.knn_I, r.knn_U, bf[1], bf[2])
    assert 0 < q <= 1.0


# ------------------------------------------------------------ Theorem 1 --

def test_theorem1_collision_rate(orc):
    """P[H(u1) = H(u2)] = |h(P1) & h(P2)| / |h(P1 | P2)| (Section III, proof of
    Theorem 1), checked over many seeds, and the per-seed bounds of that ratio
    in terms of J and the collision count kappa."""
    rng = np.random.Generator(np.random.PCG64(5))
    m, b, S = 3000, 64, 1500
    base = rng.choice(m, size=40, replace=False)
    pairs = [
        (set(base[:30].tolist()), set(base[10:40].tolist())),      # J = 0.5
        (set(base[:20].tolist()), set(base[15:40].tolist())),      # J = 0.125
        (set(base[:35].tolist()), set(base[:30].tolist())),        # nested
    ]
    for P1, P2 in pairs:
        J = len(P1 & P2) / len(P1 | P2)
        P = synth.profiles_from_sets([P1, P2], m)
        hits, ratios = [], []
        for s in range(S):
            tab = synth.hash_tables(1, 10_000 + s)
            bk = orc.hash_items(tab, b, m)
            keys = orc.frh_keys(P.indptr, P.indices, 2, m, bk)[0]
            h = bk[0]
            h1, h2 = set(h[list(P1)].tolist()), set(h[list(P2)].tolist())
            r = len(h1 & h2) / len(h1 | h2)
            ell = len(P1 | P2)
            kap = ell - len(h1 | h2) / 1.0
            x = kap / ell
            assert (J - x) / (1 - x) - 1e-12 <= r <= (J + x) / (1 - x) + 1e-12
            hits.append(1.0 if keys[0] == keys[1] else 0.0)
            ratios.append(r)
        p_hat, r_bar = np.mean(hits), np.mean(ratios)
        sd = math.sqrt(max(r_bar * (1 - r_bar), 1e-6) / S)
        assert abs(p_hat - r_bar) < 4 * sd, (p_hat, r_bar, J)


def test_minhash_limit(orc):
    """With b = 2^32 there are (almost) no collisions, so FastRandomHash is
    MinHash and the collision rate is the Jaccard similarity."""
    rng = np.random.Generator(np.random.PCG64(6))
    m, S = 100000, 3000
    base = rng.choice(m, size=60, replace=False)
    P1, P2 = set(base[:40].tolist()), set(base[20:60].tolist())   # J = 1/3
    P = synth.profiles_from_sets([P1, P2], m)
    hits = 0
    for s in range(S):
        bk = orc.hash_items(synth.hash_tables(1, 50_000 + s), 2 ** 32, m)
        keys = orc.frh_keys(P.indptr, P.indices, 2, m, bk)[0]
        hits += keys[0] == keys[1]
    J = 1 / 3
    sd = math.sqrt(J * (1 - J) / S)
    assert abs(hits / S - J) < 4 * sd + 0.01


def test_minhash_permutations_exact(orc):
    """MinHash clustering (Section V-C, Table 4) keys a user by the smallest
    permutation rank among its items.  Over all m! permutations the two users'
    keys agree in exactly J * m! of them (min-wise independence of a uniform
    permutation), so the oracle's key must reproduce that count exactly."""
    import itertools
    m = 6
    perms = np.array(list(itertools.permutations(range(m))), dtype=np.uint32)   # 720 x 6
    for A, B in [({0, 1, 2, 3}, {2, 3, 4}), ({5}, {5}), ({0}, {1}), ({0, 1, 2, 3, 4, 5}, {1})]:
        P = synth.profiles_from_sets([A, B], m)
        keys = orc.frh_keys(P.indptr, P.indices, 2, m, perms)
        same = int((keys[:, 0] == keys[:, 1]).sum())
        assert Fraction(same, len(perms)) == Fraction(len(A & B), len(A | B))
        # the key is the rank of the user's first item under the permutation
        assert all(keys[j, 0] == min(perms[j, i] for i in A) for j in range(0, 720, 37))


def test_minhash_tables_are_permutations():
    tab = synth.minhash_tables(5, 1000, 3)
    assert tab.shape == (5, 1000) and tab.dtype == np.uint32
    for row in tab:
        assert np.array_equal(np.sort(row), np.arange(1000, dtype=np.uint32))
    assert not np.array_equal(tab[0], tab[1])
    assert np.array_equal(tab, synth.minhash_tables(5, 1000, 3))


def test_minhash_clusters_are_min_items(orc):
    """With b = m and cap >= n nothing splits: there is one cluster per item
    that is some user's minimum, t*m clusters at most, and each cluster is
    exactly the users whose minimum rank is that item's."""
    P = synth.random_profiles(11, 400, 150, 1, 15, 1.0)
    t = 3
    tab = synth.minhash_tables(t, P.m, 12)
    members, off, cfg, depth = orc.cluster(P.indptr, P.indices, P.n, P.m, tab, P.n)
    keys = orc.frh_keys(P.indptr, P.indices, P.n, P.m, tab)
    assert depth == 0 and int(cfg[-1]) <= t * P.m
    for j in range(t):
        want = {}
        for u in range(P.n):
            row = P.indices[P.indptr[u]:P.indptr[u + 1]]
            if len(row):
                assert keys[j, u] == tab[j, row].min()
            want.setdefault(int(keys[j, u]), []).append(u)
        got = [members[off[c]:off[c + 1]].tolist() for c in range(cfg[j], cfg[j + 1])]
        assert got == [want[v] for v in sorted(want)]


# ------------------------------------- externally assigned top level ----

def test_cluster_keys_with_frh_keys_is_frh(orc):
    """Top-level groups given as the FastRandomHash keys themselves: the
    oversized ones first split by H_j (one group, every member shares it), then
    by H\\eta as usual, so the partition and its order equal Step 1's."""
    for seed, (n, m, t, b, cap) in enumerate([(400, 150, 3, 16, 30), (300, 2000, 4, 128, 2),
                                              (500, 100, 2, 4, 60)]):
        P = synth.random_profiles(30 + seed, n, m, 1, 25, 1.0)
        bucket = orc.hash_items(synth.hash_tables(t, 40 + seed), b, m)
        keys = orc.frh_keys(P.indptr, P.indices, n, m, bucket)
        a = orc.cluster(P.indptr, P.indices, n, m, bucket, cap)
        k = orc.cluster_keys(P.indptr, P.indices, n, m, keys, bucket, cap)
        for x, y in zip(a[:3], k[:3]):
            assert np.array_equal(x, y)


def test_cluster_keys_no_split_groups_by_key(orc):
    """cap >= n: the clusters are the users grouped by key, ascending."""
    P = synth.random_profiles(33, 300, 100, 1, 10, 1.0)
    rng = np.random.Generator(np.random.PCG64(34))
    keys = rng.integers(0, 40, size=(2, P.n), dtype=np.uint32)
    bucket = orc.hash_items(synth.hash_tables(2, 35), 16, P.m)
    mem, off, cfg, depth = orc.cluster_keys(P.indptr, P.indices, P.n, P.m, keys, bucket, P.n)
    assert depth == 0
    for j in range(2):
        got = [mem[off[c]:off[c + 1]].tolist() for c in range(cfg[j], cfg[j + 1])]
        want = [np.nonzero(keys[j] == v)[0].tolist() for v in np.unique(keys[j])]
        assert got == want


def test_cluster_keys_split_uses_frh_from_the_start(orc):
    """One key for everybody and cap < n: the result is Step 1 on the same
    users with a single top-level group, i.e. FRH with b = 1 bucket value
    spread by the item hash: every final cluster is within cap or is the
    users that stayed, and it is a partition of all users."""
    P = synth.random_profiles(36, 400, 300, 2, 30, 1.1)
    t, cap = 3, 25
    bucket = orc.hash_items(synth.hash_tables(t, 37), 64, P.m)
    keys = np.zeros((t, P.n), dtype=np.uint32)
    mem, off, cfg, depth = orc.cluster_keys(P.indptr, P.indices, P.n, P.m, keys, bucket, cap)
    assert depth >= 1
    frh = orc.frh_keys(P.indptr, P.indices, P.n, P.m, bucket)
    for j in range(t):
        users = np.sort(mem[j * P.n:(j + 1) * P.n])
        assert np.array_equal(users, np.arange(P.n))
        # the first-level sub-clusters follow ascending H_j
        first = [int(frh[j, mem[off[c]]]) for c in range(cfg[j], cfg[j + 1])]
        assert first[0] == frh[j].min()


# ------------------------------------------- Algorithm 2, Hyrec branch ----

def test_splitmix_published_outputs(orc):
    """The generator of Hyrec's initial graph is SplitMix64: its published
    first outputs from state 0."""
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert [orc.lib().orc_splitmix_at(0, c) for c in range(4)] == want


def test_alg2_without_hyrec_is_brute_force(orc):
    P = synth.random_profiles(50, 400, 200, 1, 30, 1.0)
    bucket = orc.hash_items(synth.hash_tables(3, 51), 16, P.m)
    mem, off, cfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, bucket, 80)
    a = orc.local_knn(P.indptr, P.indices, P.n, P.m, 3, 5, mem, off, cfg)
    b = orc.local_knn_alg2(P.indptr, P.indices, P.n, P.m, 3, 5, mem, off, cfg, rho=1000)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def hyrec_case(orc, seed, n=300, k=4, max_iter=30):
    P = synth.random_profiles(seed, n, 120, 2, 25, 1.0)
    t = 1
    mem = np.arange(n, dtype=np.uint32)
    off = np.array([0, n], dtype=np.uint32)
    cfg = np.array([0, 1], dtype=np.uint32)
    pid, pI = orc.local_knn_alg2(P.indptr, P.indices, n, P.m, t, k, mem, off, cfg, rho=5,
                                 max_iter=max_iter, seed=seed)
    return P, pid[:, 0], pI[:, 0]


def test_hyrec_lists_are_valid(orc):
    """Every Hyrec list holds distinct co-members other than u, with their
    exact intersection, in the exact order."""
    k = 4
    for max_iter in (0, 1, 30):
        P, pid, pI = hyrec_case(orc, 52, k=k, max_iter=max_iter)
        rows = [set(P.indices[P.indptr[u]:P.indptr[u + 1]].tolist()) for u in range(P.n)]
        for u in range(P.n):
            ids = [int(v) for v in pid[u] if v != 0xFFFFFFFF]
            assert len(ids) == len(set(ids)) and u not in ids and len(ids) >= 1
            keys = []
            for q, v in enumerate(ids):
                I = len(rows[u] & rows[v])
                assert pI[u, q] == I
                keys.append((Fraction(I, len(rows[u] | rows[v])), -v))
            assert keys == sorted(keys, reverse=True)


def test_hyrec_converges_towards_brute_force(orc):
    """Hyrec refines its random start: the graph after the iterations is far
    better than the initial one and close to brute force's (Eq. 2)."""
    k = 8                                   # rho*k^2 = 320 <= 400 members
    P, pid0, pI0 = hyrec_case(orc, 53, n=400, k=k, max_iter=0)
    _, pid, pI = hyrec_case(orc, 53, n=400, k=k, max_iter=30)
    bid, bI, bU = orc.brute_force(P.indptr, P.indices, P.n, P.m, k)
    lens = np.diff(P.indptr)

    def avg(ids, I):
        tot = 0.0
        for u in range(P.n):
            for q in range(k):
                v = ids[u, q]
                if v != 0xFFFFFFFF:
                    tot += I[u, q] / (lens[u] + lens[v] - I[u, q])
        return tot / (k * P.n)
    exact = orc.avg_sim(bI, bU)
    assert avg(pid, pI) > 0.93 * exact
    assert avg(pid, pI) > avg(pid0, pI0) + 0.3 * exact


def test_hyrec_independent_of_threads(orc):
    P = synth.random_profiles(54, 500, 150, 2, 20, 1.0)
    bucket = orc.hash_items(synth.hash_tables(2, 55), 2, P.m)
    mem, off, cfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, bucket, P.n)
    a = orc.local_knn_alg2(P.indptr, P.indices, P.n, P.m, 2, 3, mem, off, cfg, seed=9, threads=1)
    b = orc.local_knn_alg2(P.indptr, P.indices, P.n, P.m, 2, 3, mem, off, cfg, seed=9, threads=8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------- GoldFinger (II-F) ----

def test_fingerprints_brute_force(orc):
    """The fingerprint of a profile is the set of its items' positions."""
    rng = np.random.Generator(np.random.PCG64(21))
    for B in (1, 7, 64, 1000):
        P = synth.random_profiles(22 + B, 60, 300, 1, 80, 1.0)
        g = rng.integers(0, B, size=P.m, dtype=np.uint32)
        ip, ix = orc.fingerprints(P.indptr, P.indices, P.n, g)
        assert ip[0] == 0 and ip[-1] == len(ix)
        for u in range(P.n):
            want = sorted({int(g[i]) for i in P.indices[P.indptr[u]:P.indptr[u + 1]]})
            assert ix[ip[u]:ip[u + 1]].tolist() == want


def test_fingerprints_injective_position_is_identity(orc):
    """With B = m and g(i) = i nothing collides: the fingerprint is the
    profile and the GoldFinger estimate is the exact Jaccard index."""
    P = synth.random_profiles(23, 200, 90, 1, 30, 1.2)
    ip, ix = orc.fingerprints(P.indptr, P.indices, P.n, np.arange(P.m, dtype=np.uint32))
    assert np.array_equal(ip, P.indptr) and np.array_equal(ix, P.indices)


def test_fingerprints_of_union_and_fill(orc):
    """F(A | B) = F(A) | F(B), F(A & B) is inside F(A) & F(B), and with the
    seeded item hash into B positions a profile of s items fills
    B(1 - (1 - 1/B)^s) positions on average (a uniform hash)."""
    B, m = 1024, 20000
    g = orc.hash_items(synth.hash_tables(1, 24), B, m)[0]
    rng = np.random.Generator(np.random.PCG64(25))
    sets = []
    for _ in range(200):
        base = rng.choice(m, size=500, replace=False)
        sets += [set(base[:300].tolist()), set(base[150:450].tolist())]
    P = synth.profiles_from_sets(sets + [a | b for a, b in zip(sets[::2], sets[1::2])] +
                                 [a & b for a, b in zip(sets[::2], sets[1::2])], m)
    ip, ix = orc.fingerprints(P.indptr, P.indices, P.n, g)
    F = [set(ix[ip[u]:ip[u + 1]].tolist()) for u in range(P.n)]
    npair = len(sets) // 2
    for q in range(npair):
        Fa, Fb = F[2 * q], F[2 * q + 1]
        assert F[len(sets) + q] == Fa | Fb
        assert F[len(sets) + npair + q] <= Fa & Fb
    fill = np.mean([len(F[u]) for u in range(len(sets))])
    want = B * (1 - (1 - 1 / B) ** 300)
    sd = math.sqrt(B * math.exp(-300 / B) * (1 - (1 + 300 / B) * math.exp(-300 / B)))
    assert abs(fill - want) < 4 * sd / math.sqrt(len(sets)) + 0.5


def test_edge_jaccard_matches_sets():
    from paper_2010_11497_amd import metrics
    P = synth.random_profiles(26, 80, 150, 1, 40, 1.0)
    rng = np.random.Generator(np.random.PCG64(27))
    ids = rng.integers(0, P.n, size=(P.n, 5)).astype(np.uint32)
    ids[::7, 4] = 0xFFFFFFFF
    I, U = metrics.edge_jaccard(P.indptr, P.indices, P.m, ids)
    rows = [set(P.indices[P.indptr[u]:P.indptr[u + 1]].tolist()) for u in range(P.n)]
    for u in range(P.n):
        for j in range(5):
            v = int(ids[u, j])
            if v == 0xFFFFFFFF:
                assert I[u, j] == 0 and U[u, j] == 0
            else:
                assert I[u, j] == len(rows[u] & rows[v]) and U[u, j] == len(rows[u] | rows[v])


# ------------------------------------------------------------ Theorem 2 --

def test_theorem2_example_constant():
    """The example after Theorem 2 (ell = 256, b = 4096) prints 0.078, 0.234
    and probability 0.998; those follow from d = 1.5 (the text says 0.5)."""
    ell, b = 256, 4096
    mean = ell * (ell - 1) / (2 * b)
    for d, lo, hi, p in [(1.5, 0.078, 0.234, 0.998), (0.5, 0.047, 0.140, 0.578)]:
        dens = (1 + d) * (ell - 1) / (2 * b)
        prob = 1 - (math.exp(d) / (1 + d) ** (1 + d)) ** mean
        assert round(dens, 3) == lo and round(3 * dens, 2) == round(hi, 2) and round(prob, 3) == p


def test_theorem2_tail_holds(orc):
    """Empirical tail of the collision density kappa/ell under the oracle's
    hash stays below the Chernoff bound of Theorem 2."""
    ell, b, d, S = 256, 4096, 0.5, 400
    m = 100000
    rng = np.random.Generator(np.random.PCG64(8))
    thr = (1 + d) * (ell - 1) / (2 * b)
    bound = (math.exp(d) / (1 + d) ** (1 + d)) ** (ell * (ell - 1) / (2 * b))
    over = 0
    for s in range(S):
        items = rng.choice(m, size=ell, replace=False)
        h = orc.hash_items(synth.hash_tables(1, 70_000 + s), b, m)[0][items]
        kappa = ell - len(set(h.tolist()))
        over += kappa / ell >= thr
    # bound = 0.42; allow binomial noise
    assert over / S <= bound + 4 * math.sqrt(bound * (1 - bound) / S)


# ------------------------------------------------------------ validation --

def test_validate(orc):
    ok = synth.profiles_from_sets([{0, 2}, {1}], 3)
    assert orc.validate(ok.indptr, ok.indices, 2, 3) == 0
    assert orc.validate(ok.indptr, ok.indices, 2, 2) == -2          # item out of range
    assert orc.validate(np.array([0, 2, 2]), ok.indices[:2], 2, 3) == -2   # empty row
    assert orc.validate(np.array([0, 2, 3]), np.array([2, 0, 1], np.uint32), 2, 3) == -2
    assert orc.validate(np.array([0, 2, 3]), np.array([1, 1, 1], np.uint32), 2, 3) == -2


def test_cluster_work_sparse_pairs_identity(orc):
    """Summed over same-cluster pairs, |P_u & P_v| counts every item once per
    pair of members holding it: sum_{pairs} I = sum_{clusters, items} f(f-1)/2."""
    from paper_2010_11497_amd import metrics
    P = synth.random_profiles(60, 300, 100, 1, 25, 1.0)
    bucket = orc.hash_items(synth.hash_tables(3, 61), 8, P.m)
    mem, off, cfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, bucket, 50)
    work = metrics.cluster_work(mem, off, P.indptr, P.indices, P.m)
    rows = [set(P.indices[P.indptr[u]:P.indptr[u + 1]].tolist()) for u in range(P.n)]
    tot = 0
    for c in range(len(off) - 1):
        S = mem[off[c]:off[c + 1]].tolist()
        tot += sum(len(rows[a] & rows[b]) for i, a in enumerate(S) for b in S[i + 1:])
    assert work["sparse_pairs"] == tot
    assert work["pairs"] == sum(len(S) * (len(S) - 1) // 2 for S in
                                (mem[off[c]:off[c + 1]] for c in range(len(off) - 1)))



def test_cluster_work_torch_equals_dense_count(orc):
    """The run-counting form (pieces of a few thousand entries, so that clusters
    are cut into several pieces per configuration) gives the dense count
    table's dictionary sizes and sums."""
    import torch
    from paper_2010_11497_amd import metrics
    P = synth.random_profiles(62, 500, 120, 1, 30, 1.0)
    bucket = orc.hash_items(synth.hash_tables(4, 63), 8, P.m)
    mem, off, cfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, bucket, 60)
    ref = metrics.cluster_work(mem, off, P.indptr, P.indices, P.m)
    got = metrics.cluster_work_torch(torch.from_numpy(mem.astype(np.int64)),
                                     torch.from_numpy(off.astype(np.int64)), cfg,
                                     torch.from_numpy(P.indptr),
                                     torch.from_numpy(P.indices.astype(np.int64)), P.m,
                                     max_entries=700)
    for key in ("clusters", "pairs", "ordered", "bitmap_ops", "dense_ops", "sparse_pairs"):
        assert got[key] == ref[key], key
    assert np.array_equal(got["sizes"], ref["sizes"]) and np.array_equal(got["dict"], ref["dict"])

# ------------------------------------------------- Eq. 1 and Eq. 2 by hand --

# A graph of 4 users with k = 3.  User 0 keeps an edge with I = 0, user 1 an
# edge with I = 0 and one padded slot, user 3 only padded slots.  By hand, its
# Jaccard values sum to 1/2 + 1/5 + 0 + 1 + 0 + 1/2 + 1/4 + 1/8 = 103/40, so
# Eq. 1 over the k*n = 12 slots gives 103/480.  The "exact" graph beside it
# sums to 31/30 + 23/18 + 13/12 + 1/10 = 629/180, i.e. 629/2160, so Eq. 2
# gives (103/480) / (629/2160) = 927/1258.
EQ_APPROX = ([[2, 1, 0], [3, 0, 0], [1, 1, 1], [0, 0, 0]],
             [[4, 5, 7], [3, 9, 0], [2, 4, 8], [0, 0, 0]])
EQ_EXACT = ([[2, 1, 1], [3, 1, 1], [1, 1, 1], [1, 0, 0]],
            [[4, 3, 5], [3, 6, 9], [2, 3, 4], [10, 0, 0]])


def test_eq1_eq2_hand_computed(orc):
    """Eq. 1 divides by k*n whatever the number of filled slots, and counts
    I = 0 edges as 0; Eq. 2 is the ratio of two Eq. 1 values.  Both the
    oracle's and the benchmark's implementations against the hand values."""
    from paper_2010_11497_amd import metrics
    aI, aU = (np.array(x, dtype=np.uint32) for x in EQ_APPROX)
    eI, eU = (np.array(x, dtype=np.uint32) for x in EQ_EXACT)
    for mod in (orc, metrics):
        assert mod.avg_sim(aI, aU) == pytest.approx(103 / 480, rel=1e-15)
        assert mod.avg_sim(eI, eU) == pytest.approx(629 / 2160, rel=1e-15)
        assert mod.quality(aI, aU, eI, eU) == pytest.approx(927 / 1258, rel=1e-15)
        # the exact graph against itself
        assert mod.quality(eI, eU, eI, eU) == 1.0


# ------------------------------- Algorithm 2, Hyrec, restated in Python ----

def splitmix64(seed, c):
    """Output c + 1 of SplitMix64 from state `seed` (Steele, Lea and Flood,
    2014): the state advances by the golden gamma 0x9E3779B97F4A7C15 and is
    passed through the published 64-bit mixer."""
    z = (seed + 0x9E3779B97F4A7C15 * (c + 1)) % (1 << 64)
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) % (1 << 64)
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) % (1 << 64)
    return z ^ (z >> 31)


def hyrec_python(sets, S, cl, k, seed, delta, max_iter, own=True, sync=True):
    """Reading R25 of Algorithm 2's Hyrec branch on one cluster (members S,
    ascending ids, cluster index cl), with rational Jaccard values:
      start:  member a draws k members q = 0..k-1 (SplitMix64 output number
              (cl << 40) | (a << 12) | q, modulo s - 1, shifted past a) and
              keeps the k best distinct;
      step:   synchronously, a's new list is the k best distinct of its own
              list and its neighbours' lists, a itself excluded;
      stop:   after a step in which fewer than delta*k*s entries of the new
              lists were absent from the old ones, or after max_iter steps.
    own=False and sync=False give two plausible misreadings (a's own list left
    out; lists replaced during the step), used to show the pin catches them.
    Returns the member positions per list and the number of steps taken."""
    s = len(S)

    def J(a, b):
        return Fraction(len(sets[S[a]] & sets[S[b]]), len(sets[S[a]] | sets[S[b]]))

    def best(a, pool):
        return sorted(set(pool) - {a}, key=lambda b: (-J(a, b), b))[:k]

    lists = []
    for a in range(s):
        draws = []
        for q in range(k):
            b = splitmix64(seed, (cl << 40) | (a << 12) | q) % (s - 1)
            draws.append(b + 1 if b >= a else b)
        lists.append(best(a, draws))
    steps = 0
    while steps < max_iter:
        new = [list(x) for x in lists]
        src = lists if sync else new
        for a in range(s):
            pool = (list(src[a]) if own else []) + [c for b in src[a] for c in src[b]]
            new[a] = best(a, pool)
        updates = sum(len(set(new[a]) - set(lists[a])) for a in range(s))
        lists = new
        steps += 1
        if updates < delta * k * s:
            break
    return lists, steps


def hyrec_partition(seed, s=16, lead=3, m=40):
    """t = 1 partition of lead + s users: a small cluster first (brute force
    under rho = 1 when lead < k^2), then one of s members at cluster index 1
    (Hyrec), the members interleaved so that positions differ from ids."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = lead + s
    sets = [set(rng.choice(m, size=int(rng.integers(2, 9)), replace=False).tolist())
            for _ in range(n)]
    perm = rng.permutation(n)
    first = np.sort(perm[:lead]).astype(np.uint32)
    hy = np.sort(perm[lead:]).astype(np.uint32)
    members = np.concatenate([first, hy])
    cl_off = np.array([0, lead, n], dtype=np.uint32)
    cfg = np.array([0, 2], dtype=np.uint32)
    return sets, members, cl_off, cfg, hy.tolist()


def hyrec_oracle_rows(orc, sets, members, cl_off, cfg, k, seed, delta, max_iter):
    P = synth.profiles_from_sets(sets, 1 + max(max(x) for x in sets))
    pid, pI = orc.local_knn_alg2(P.indptr, P.indices, len(sets), P.m, 1, k, members, cl_off,
                                 cfg, rho=1, delta=delta, max_iter=max_iter, seed=seed)
    return pid[:, 0], pI[:, 0]


def expected_rows(sets, S, lists, k):
    out = {}
    for a, u in enumerate(S):
        ids = [S[b] for b in lists[a]]
        I = [len(sets[u] & sets[v]) for v in ids]
        out[u] = (ids + [PAD] * (k - len(ids)), I + [0] * (k - len(ids)))
    return out


@pytest.mark.parametrize("k,seed", [(2, 61), (3, 62), (2, 63)])
def test_hyrec_steps_equal_restatement(orc, k, seed):
    """The oracle's Hyrec lists equal the Python restatement exactly after 0,
    1 and 2 synchronous steps (delta = 0: no early stop); the cluster sits at
    index 1, so the draw counter's cluster field is exercised."""
    sets, members, cl_off, cfg, S = hyrec_partition(seed)
    for max_iter in (0, 1, 2):
        lists, steps = hyrec_python(sets, S, 1, k, seed, 0.0, max_iter)
        assert steps == max_iter
        pid, pI = hyrec_oracle_rows(orc, sets, members, cl_off, cfg, k, seed, 0.0, max_iter)
        for u, (ids, I) in expected_rows(sets, S, lists, k).items():
            assert pid[u].tolist() == ids and pI[u].tolist() == I, (max_iter, u)


def test_hyrec_restatement_separates_misreadings():
    """Premise of the step pin: on its cases, leaving a member's own list out
    of its candidates, or replacing lists during a step, changes the lists."""
    diff_own = diff_sync = False
    for k, seed in [(2, 61), (3, 62), (2, 63)]:
        sets, _, _, _, S = hyrec_partition(seed)
        for it in (1, 2):
            ref, _ = hyrec_python(sets, S, 1, k, seed, 0.0, it)
            diff_own |= hyrec_python(sets, S, 1, k, seed, 0.0, it, own=False)[0] != ref
            diff_sync |= hyrec_python(sets, S, 1, k, seed, 0.0, it, sync=False)[0] != ref
    assert diff_own and diff_sync


def test_hyrec_stop_rule_is_strict(orc):
    """The stop rule 'fewer than delta*k*s changed entries': with k*s = 32 the
    threshold delta*k*s is an exact integer.  A case whose steps change u1 > u2
    entries (u2 >= 1) and whose third step still changes the lists stops after
    step 2 for delta*32 = u2 + 1, and runs on for delta*32 = u2 (not fewer)."""
    k, s = 2, 16
    for seed in range(100, 200):
        sets, members, cl_off, cfg, S = hyrec_partition(seed, s=s)
        l1, _ = hyrec_python(sets, S, 1, k, seed, 0.0, 1)
        l2, _ = hyrec_python(sets, S, 1, k, seed, 0.0, 2)
        l3, _ = hyrec_python(sets, S, 1, k, seed, 0.0, 3)
        l0, _ = hyrec_python(sets, S, 1, k, seed, 0.0, 0)
        u1 = sum(len(set(l1[a]) - set(l0[a])) for a in range(s))
        u2 = sum(len(set(l2[a]) - set(l1[a])) for a in range(s))
        if u1 > u2 >= 1 and l3 != l2:
            break
    else:
        pytest.fail("no seed with the premise")
    for thr, want_steps in ((u2 + 1, 2), (u2, None)):
        delta = thr / (k * s)
        assert delta * k * s == thr
        lists, steps = hyrec_python(sets, S, 1, k, seed, delta, 30)
        if want_steps is not None:
            assert steps == 2 and lists == l2
        else:
            assert steps > 2
        pid, pI = hyrec_oracle_rows(orc, sets, members, cl_off, cfg, k, seed, delta, 30)
        for u, (ids, I) in expected_rows(sets, S, lists, k).items():
            assert pid[u].tolist() == ids and pI[u].tolist() == I, (thr, u)
