"""GPU parity: every stage of the HIP path, through the C ABI, against the CPU
oracle on the same seeded inputs.  Integer outputs must match bit for bit.

Stage isolation: c2_local_knn is fed the oracle's partition and c2_merge the
oracle's partial lists, so a mismatch names the stage.  The clustering order
is part of the contract (ascending hash values, sub-clusters before the users
that stay), so partitions are compared as raw arrays, and also as sets so a
failure says whether only the order differs.
"""
import functools
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_11497_amd import c2, synth  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
THREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def u32(t):
    return c2.to_u32(t)


def gpu_inputs(P, tab):
    return c2.DeviceProfiles.from_synth(P), c2.tables_to_device(tab)


def partition_sets(members, cl_off, cfg):
    t = len(cfg) - 1
    return [sorted(tuple(sorted(members[cl_off[c]:cl_off[c + 1]].tolist()))
                   for c in range(cfg[j], cfg[j + 1])) for j in range(t)]


def cases():
    out = []
    for seed, (n, m, lo, hi, zipf, t, b, cap, k) in enumerate([
            (300, 120, 1, 20, 1.0, 3, 16, 40, 5),
            (500, 200, 2, 30, 1.1, 4, 8, 25, 10),
            (257, 64, 1, 12, 0.7, 2, 4, 100, 32),
            (400, 300, 1, 40, 1.2, 8, 32, 3, 7),
            (130, 40, 1, 6, 0.0, 1, 1, 7, 4),        # one bucket: one cluster per config
            (90, 2000, 1, 5, 0.0, 5, 128, 1, 3),     # cap 1: everything splits
    ]):
        P = synth.random_profiles(500 + seed, n, m, lo, hi, zipf)
        tab = synth.hash_tables(t, 900 + seed)
        out.append(("rand%d" % seed, P, tab, b, cap, k))
    return out


CASES = cases()


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle


# ------------------------------------------------------------- hashing ----

@pytest.mark.parametrize("t,b,m", [(1, 3, 5), (8, 1024, 3700), (3, 1, 1000), (64, 8192, 4097),
                                   (2, (1 << 24), 131072)])
def test_hash_items(orc, t, b, m):
    say("hash_items", t, b, m)
    tab = synth.hash_tables(t, 31 + t)
    got = u32(c2.hash_items(c2.tables_to_device(tab), b, m))
    assert np.array_equal(got, orc.hash_items(tab, b, m))


@pytest.mark.parametrize("name,P,tab,b,cap,k", CASES, ids=[c[0] for c in CASES])
def test_frh_keys(orc, name, P, tab, b, cap, k):
    say("frh_keys", name)
    dP, dtab = gpu_inputs(P, tab)
    bucket = c2.hash_items(dtab, b, P.m)
    got = u32(c2.frh_keys(dP, bucket))
    assert np.array_equal(got, orc.frh_keys(P.indptr, P.indices, P.n, P.m, u32(bucket)))


# ---------------------------------------------------------- clustering ----

# clustering paths: one workgroup per configuration (all rounds in LDS, used
# automatically up to 8192 users) and the grid rounds (any size)
CPATHS = {"workgroup": c2.CLUSTER_WORKGROUP, "grid": c2.CLUSTER_GRID}


def check_cluster(orc, P, bucket_np, cap, form, dP=None, dbucket=None, path=0):
    t = bucket_np.shape[0]
    dP = dP or c2.DeviceProfiles.from_synth(P)
    dbucket = dbucket if dbucket is not None else torch.as_tensor(bucket_np.view(np.int32)).cuda()
    p = c2.params(t, int(bucket_np.max()) + 1, cap, 1)
    tu = c2.tuning(split_rounds=64 if form else 0, cluster_path=path)
    members, cl_off, cfg, ws = c2.cluster(dP, dbucket, p, form, tu)
    torch.cuda.synchronize()
    if form == c2.FORM_BATCHED:
        c2.check_complete(ws)
    gm, gcfg = u32(members), u32(cfg)
    goff = u32(cl_off)[: gcfg[-1] + 1]
    om, ooff, ocfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, bucket_np, cap)
    assert partition_sets(gm, goff, gcfg) == partition_sets(om, ooff, ocfg)
    assert np.array_equal(gcfg, ocfg)
    assert np.array_equal(goff, ooff)
    assert np.array_equal(gm, om)


@pytest.mark.parametrize("path", list(CPATHS))
@pytest.mark.parametrize("form", [c2.FORM_PLAIN, c2.FORM_BATCHED])
@pytest.mark.parametrize("fixture", ["fig3_split.json", "singleton_stays.json",
                                     "frh_worked_example.json"])
def test_cluster_fixtures(orc, fixture, form, path):
    say("cluster fixture", fixture, form, path)
    g = json.load(open(os.path.join(GOLDEN, fixture)))
    P = synth.profiles_from_sets(g["profiles"], g["m"])
    bucket = np.array(g["bucket"], dtype=np.uint32)
    check_cluster(orc, P, bucket, g.get("cap", 10), form, path=CPATHS[path])


@pytest.mark.parametrize("path", list(CPATHS))
@pytest.mark.parametrize("form", [c2.FORM_PLAIN, c2.FORM_BATCHED])
@pytest.mark.parametrize("name,P,tab,b,cap,k", CASES, ids=[c[0] for c in CASES])
def test_cluster_random(orc, name, P, tab, b, cap, k, form, path):
    say("cluster", name, form, path)
    check_cluster(orc, P, orc.hash_items(tab, b, P.m), cap, form, path=CPATHS[path])


@pytest.mark.parametrize("path", list(CPATHS))
def test_cluster_identical_profiles_deep(orc, path):
    # 40 identical users with 30 distinct hash values: a chain of splits deeper
    # than the workgroup path's 4 precomputed values per user
    say("cluster deep chain", path)
    sets = [set(range(30))] * 40
    P = synth.profiles_from_sets(sets, 30)
    bucket = np.arange(30, dtype=np.uint32)[None, :]
    check_cluster(orc, P, bucket, 5, c2.FORM_PLAIN, path=CPATHS[path])


@pytest.mark.parametrize("n", [8192, 8193])
def test_cluster_workgroup_size_limit(orc, n):
    # the largest configuration the workgroup path takes, and one user more
    # (the automatic choice then runs the grid rounds)
    say("cluster size limit", n)
    P = synth.random_profiles(77, n, 600, 1, 25, 1.0)
    tab = synth.hash_tables(2, 78)
    check_cluster(orc, P, orc.hash_items(tab, 64, P.m), 300, c2.FORM_BATCHED)


@pytest.mark.parametrize("path", list(CPATHS))
def test_batched_reports_incomplete(orc, path):
    say("incomplete", path)
    sets = [set(range(30))] * 40
    P = synth.profiles_from_sets(sets, 30)
    dP = c2.DeviceProfiles.from_synth(P)
    bucket = torch.as_tensor(np.arange(30, dtype=np.int32)[None, :]).cuda()
    p = c2.params(1, 30, 5, 1)
    _, _, _, ws = c2.cluster(dP, bucket, p, c2.FORM_BATCHED,
                             c2.tuning(split_rounds=3, cluster_path=CPATHS[path]))
    with pytest.raises(c2.C2Error) as e:
        c2.check_complete(ws)
    assert e.value.status == -6


# ------------------------------------------------------------ local KNN ----

PATHS = {"auto": 0, "mfma": 2, "bitmap": 1 << 30}


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("form", [c2.FORM_PLAIN, c2.FORM_BATCHED])
@pytest.mark.parametrize("name,P,tab,b,cap,k", CASES, ids=[c[0] for c in CASES])
def test_local_knn_on_oracle_partition(orc, name, P, tab, b, cap, k, form, path):
    say("local_knn", name, form, path)
    t = tab.shape[0]
    om, ooff, ocfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, orc.hash_items(tab, b, P.m), cap)
    dP = c2.DeviceProfiles.from_synth(P)
    dev = lambda a: torch.as_tensor(a.astype(np.uint32).view(np.int32)).cuda()
    pid, pI = c2.local_knn(dP, dev(om), dev(ooff), dev(ocfg), c2.params(t, b, cap, k), form,
                           c2.tuning(mfma_min_rows=PATHS[path]))
    wid, wI = orc.local_knn(P.indptr, P.indices, P.n, P.m, t, k, om, ooff, ocfg, THREADS)
    assert np.array_equal(u32(pid), wid)
    assert np.array_equal(u32(pI), wI)


@pytest.mark.parametrize("name,P,tab,b,cap,k", CASES, ids=[c[0] for c in CASES])
def test_merge_on_oracle_lists(orc, name, P, tab, b, cap, k):
    say("merge", name)
    t = tab.shape[0]
    r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, b, cap, k, THREADS)
    dP = c2.DeviceProfiles.from_synth(P)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a).view(np.int32)).cuda()
    got = c2.merge(dP, dev(r.part_id), dev(r.part_I), c2.params(t, b, cap, k))
    for g, w in zip(got, (r.knn_id, r.knn_I, r.knn_U)):
        assert np.array_equal(u32(g), w)


# ------------------------------------------------------------ end to end ----

@pytest.mark.parametrize("form", [c2.FORM_PLAIN, c2.FORM_BATCHED])
@pytest.mark.parametrize("name,P,tab,b,cap,k", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("path", list(CPATHS))
def test_build(orc, name, P, tab, b, cap, k, form, path):
    say("build", name, form, path)
    t = tab.shape[0]
    dP, dtab = gpu_inputs(P, tab)
    got = c2.build(dP, dtab, c2.params(t, b, cap, k), form,
                   c2.tuning(split_rounds=64 if form else 0, cluster_path=CPATHS[path]))
    r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, b, cap, k, THREADS)
    for g, w in zip(got, (r.knn_id, r.knn_I, r.knn_U)):
        assert np.array_equal(u32(g), w)


@pytest.mark.parametrize("b", [(1 << 31) - 1, 1 << 31, 3 << 29])
def test_build_wide_bucket_range(orc, b):
    """Bucket counts up to 2^31: hashing, the partition (the split's 64-bit
    sort keys then hold a 32-bit value field) and the whole build in both
    forms against the oracle."""
    say("wide bucket range", b)
    P = synth.random_profiles(81, 3000, 2000, 1, 40, 1.0)
    t, cap, k = 4, 100, 10
    tab = synth.hash_tables(t, 82)
    dP, dtab = gpu_inputs(P, tab)
    bucket = orc.hash_items(tab, b, P.m)
    assert int(bucket.max()) >= 1 << 24                 # values past the former limit
    assert np.array_equal(u32(c2.hash_items(dtab, b, P.m)), bucket)
    p = c2.params(t, b, cap, k)
    om, ooff, ocfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, bucket, cap)
    for form in (c2.FORM_PLAIN, c2.FORM_BATCHED):
        assert_same_partition(gpu_partition(dP, c2.hash_items(dtab, b, P.m), p, form),
                              (om, ooff, ocfg))
    r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, b, cap, k, THREADS)
    for form in (c2.FORM_PLAIN, c2.FORM_BATCHED):
        for g, want in zip(c2.build(dP, dtab, p, form, c2.tuning(split_rounds=64)),
                           (r.knn_id, r.knn_I, r.knn_U)):
            assert np.array_equal(u32(g), want)


def test_brute_force(orc):
    for seed, (n, m, k) in enumerate([(300, 100, 5), (700, 3000, 32), (65, 20, 64 // 2), (2, 3, 4),
                                      (1000, 130, 17), (129, 64, 8)]):
        say("brute force", n, m, k)
        P = synth.random_profiles(70 + seed, n, m, 1, 25, 1.0)
        got = c2.brute_force(c2.DeviceProfiles.from_synth(P), k)
        want = orc.brute_force(P.indptr, P.indices, P.n, P.m, k, threads=THREADS)
        for g, w in zip(got, want):
            assert np.array_equal(u32(g), w)


def test_single_user_and_pair(orc):
    for sets in ([{0, 1}], [{0}, {0}], [{0}, {1}]):
        P = synth.profiles_from_sets(sets, 2)
        tab = synth.hash_tables(2, 3)
        dP, dtab = gpu_inputs(P, tab)
        for form in (c2.FORM_PLAIN, c2.FORM_BATCHED):
            got = c2.build(dP, dtab, c2.params(2, 4, 1, 3), form)
            r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, 4, 1, 3)
            for g, w in zip(got, (r.knn_id, r.knn_I, r.knn_U)):
                assert np.array_equal(u32(g), w)


def test_validate_rejects_bad_profiles():
    good = synth.profiles_from_sets([{0, 2}, {1}], 3)
    c2.validate(c2.DeviceProfiles.from_synth(good))
    for indptr, indices, m in [([0, 2, 2], [0, 2], 3),          # empty row
                               ([0, 2, 3], [2, 0, 1], 3),       # unsorted
                               ([0, 2, 3], [0, 2, 1], 2)]:      # item >= m
        bad = c2.DeviceProfiles(np.array(indptr), np.array(indices, np.uint32), 2, m)
        with pytest.raises(c2.C2Error) as e:
            c2.validate(bad)
        assert e.value.status == -2


@pytest.mark.parametrize("path", list(CPATHS))
def test_graph_replays_match_eager(orc, path):
    say("graph replays", path)
    P = synth.random_profiles(44, 600, 300, 2, 30, 1.0)
    tab = synth.hash_tables(4, 45)
    dP, dtab = gpu_inputs(P, tab)
    p = c2.params(4, 16, 40, 10)
    eager = [u32(x) for x in c2.build(dP, dtab, p, c2.FORM_PLAIN)]
    g = c2.Graph(dP, dtab, p, c2.tuning(cluster_path=CPATHS[path]))
    for rep in range(3):
        out = g.launch()
        torch.cuda.synchronize()
        g.check()
        for a, b in zip(out, eager):
            assert np.array_equal(u32(a), b), rep
        # eager work between replays
        c2.build(dP, dtab, p, c2.FORM_BATCHED)
        torch.cuda.synchronize()
    g.close()


def test_determinism_repeated_runs():
    w = synth.WORKLOADS["n2k_m1k"]
    P = synth.make_profiles(w)
    tab = synth.hash_tables(w.t, w.hash_seed)
    dP, dtab = gpu_inputs(P, tab)
    p = c2.params(w.t, w.b, w.cap, w.k)
    ref = [u32(x) for x in c2.build(dP, dtab, p, c2.FORM_BATCHED)]
    for _ in range(4):
        again = [u32(x) for x in c2.build(dP, dtab, p, c2.FORM_BATCHED)]
        for a, b in zip(again, ref):
            assert np.array_equal(a, b)


# ------------------------------------------------------- named workloads ----

@pytest.mark.parametrize("name", ["n2k_m1k", "n6k_m3.7k"])
def test_workload_full_parity(orc, name):
    w = synth.WORKLOADS[name]
    say("workload", name)
    P = synth.make_profiles(w)
    tab = synth.hash_tables(w.t, w.hash_seed)
    dP, dtab = gpu_inputs(P, tab)
    p = c2.params(w.t, w.b, w.cap, w.k)
    r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, w.b, w.cap, w.k, THREADS)
    for form in (c2.FORM_PLAIN, c2.FORM_BATCHED):
        got = c2.build(dP, dtab, p, form)
        for g, want in zip(got, (r.knn_id, r.knn_I, r.knn_U)):
            assert np.array_equal(u32(g), want)
    # the launch configuration the benchmark times: graph replays of the
    # batched build with the autotuner's schedule for this workload
    from paper_2010_11497_amd import autotune
    g = c2.Graph(dP, dtab, p, c2.tuning(**(autotune.load_table(name) or {})))
    for _ in range(2):
        out = g.launch()
        torch.cuda.synchronize()
        g.check()
        for a, want in zip(out, (r.knn_id, r.knn_I, r.knn_U)):
            assert np.array_equal(u32(a), want)
    g.close()
    bf = c2.brute_force(dP, w.k)
    rows = np.random.Generator(np.random.PCG64(1)).choice(P.n, size=200, replace=False)
    want = orc.brute_force(P.indptr, P.indices, P.n, P.m, w.k, rows=rows, threads=THREADS)
    for g, ww in zip(bf, want):
        assert np.array_equal(u32(g)[rows], ww)


@functools.lru_cache(maxsize=2)
def workload_profiles(name):
    """The named workload's profiles, generated once per session (the 500,000
    user workload takes tens of seconds to draw)."""
    return synth.make_profiles(synth.WORKLOADS[name])


def tuned_graph(dP, dtab, p, name, t, cap):
    """The launch configuration the benchmark times: the batched build captured
    as a graph with the autotuner's schedule for this workload and setting."""
    from paper_2010_11497_amd import autotune
    return c2.Graph(dP, dtab, p, c2.tuning(**(autotune.load_table(name, t, cap) or {})))


def gpu_partition(dP, bucket, p, form):
    members, cl_off, cfg, ws = c2.cluster(dP, bucket, p, form, c2.tuning(split_rounds=64))
    if form == c2.FORM_BATCHED:
        c2.check_complete(ws)
    return members, cl_off, cfg


def assert_same_partition(got, want):
    gm, goff, gcfg = got
    om, ooff, ocfg = want
    gcfg = u32(gcfg)
    assert np.array_equal(gcfg, ocfg)
    assert np.array_equal(u32(goff)[: gcfg[-1] + 1], ooff)
    assert np.array_equal(u32(gm), om)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("name", ["n70k_m10k", "n140k_m27k", "n500k_m50k"])
def test_workload_whole_graph(orc, name):
    """The three large workloads at their own t and N: the whole partition in
    both forms and the whole graph (knn_id, knn_I, knn_U of every user) from the
    tuned graph form on two replays and from the plain form, against the
    oracle's complete build."""
    w = synth.WORKLOADS[name]
    say("workload whole graph", name)
    P = workload_profiles(name)
    tab = synth.hash_tables(w.t, w.hash_seed)
    dP, dtab = gpu_inputs(P, tab)
    p = c2.params(w.t, w.b, w.cap, w.k)
    r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, w.b, w.cap, w.k, THREADS)
    say("oracle build done", name)
    bucket = c2.hash_items(dtab, w.b, w.m)
    for form in (c2.FORM_PLAIN, c2.FORM_BATCHED):
        assert_same_partition(gpu_partition(dP, bucket, p, form),
                              (r.members, r.cl_off, r.cl_cfg_off))
    want = (r.knn_id, r.knn_I, r.knn_U)
    g = tuned_graph(dP, dtab, p, name, w.t, w.cap)
    for _ in range(2):
        out = g.launch()
        torch.cuda.synchronize()
        g.check()
        for a, ww in zip(out, want):
            assert np.array_equal(u32(a), ww)
    g.close()
    for a, ww in zip(c2.build(dP, dtab, p, c2.FORM_PLAIN), want):
        assert np.array_equal(u32(a), ww)


def test_long_profiles_take_exact_fallback(orc):
    # profiles of 2^15 items or more leave the 16-bit key range of the MFMA
    # path; the general path must still match the oracle bit for bit
    rng = np.random.Generator(np.random.PCG64(77))
    m = 40000
    sets = []
    for u in range(150):
        size = 33000 if u % 25 == 0 else int(rng.integers(5, 400))
        sets.append(set(rng.choice(m, size=size, replace=False).tolist()))
    P = synth.profiles_from_sets(sets, m)
    k = 7
    got = c2.brute_force(c2.DeviceProfiles.from_synth(P), k)
    want = orc.brute_force(P.indptr, P.indices, P.n, P.m, k, threads=THREADS)
    for g, w in zip(got, want):
        assert np.array_equal(u32(g), w)
    tab = synth.hash_tables(3, 78)
    dP, dtab = gpu_inputs(P, tab)
    got = c2.build(dP, dtab, c2.params(3, 4, 60, k), c2.FORM_BATCHED)
    r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, 4, 60, k, THREADS)
    for g, w in zip(got, (r.knn_id, r.knn_I, r.knn_U)):
        assert np.array_equal(u32(g), w)


def test_merge_wide_unions(orc):
    # unions of 2^16 items or more: the merge leaves the 32-bit key order for
    # the exact comparison there (users with such a union among their
    # candidates), both from indptr (c2_merge) and from the build's lengths
    rng = np.random.Generator(np.random.PCG64(81))
    m = 120000
    sets = []
    for u in range(48):
        size = 40000 if u % 4 == 0 else int(rng.integers(5, 300))
        sets.append(set(rng.choice(m, size=size, replace=False).tolist()))
    P = synth.profiles_from_sets(sets, m)
    k, t, b, cap = 6, 3, 2, 1000
    tab = synth.hash_tables(t, 82)
    r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, b, cap, k, THREADS)
    big = np.arange(P.n) % 4 == 0
    assert (r.knn_U[big] >= 65536).any() and (r.knn_U[~big] < 65536).all()
    dP, dtab = gpu_inputs(P, tab)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a).view(np.int32)).cuda()
    got = c2.merge(dP, dev(r.part_id), dev(r.part_I), c2.params(t, b, cap, k))
    for g, w in zip(got, (r.knn_id, r.knn_I, r.knn_U)):
        assert np.array_equal(u32(g), w)
    got = c2.build(dP, dtab, c2.params(t, b, cap, k), c2.FORM_BATCHED)
    for g, w in zip(got, (r.knn_id, r.knn_I, r.knn_U)):
        assert np.array_equal(u32(g), w)


# ------------------------------------------------- MinHash clustering ----

@pytest.mark.parametrize("path", list(CPATHS))
@pytest.mark.parametrize("n,m,lo,hi,zipf,t,k", [(600, 250, 1, 25, 1.1, 4, 10),
                                               (2000, 1000, 5, 60, 1.0, 8, 30),
                                               (300, 40, 1, 6, 0.0, 2, 5)])
def test_minhash_build(orc, n, m, lo, hi, zipf, t, k, path):
    """MinHash clustering (b = m, per-item permutation ranks, no split) through
    the same three stages, against the oracle's stages on the same table."""
    say("minhash", n, m, t, k, path)
    P = synth.random_profiles(7000 + n, n, m, lo, hi, zipf)
    tab = synth.minhash_tables(t, m, 7100 + n)
    dP = c2.DeviceProfiles.from_synth(P)
    p = c2.params(t, m, n, k)
    got = c2.build_from_buckets(dP, torch.as_tensor(tab.view(np.int32)).cuda(), p,
                                c2.tuning(cluster_path=CPATHS[path]))
    om, ooff, ocfg, depth = orc.cluster(P.indptr, P.indices, n, m, tab, n)
    assert depth == 0
    pid, pI = orc.local_knn(P.indptr, P.indices, n, m, t, k, om, ooff, ocfg, THREADS)
    want = orc.merge(P.indptr, n, t, k, pid, pI)
    for g, w in zip(got, want):
        assert np.array_equal(u32(g), w)


# ------------------------------------------------ GoldFinger (II-F) ----

def check_fingerprint(orc, P, g, B):
    dP = c2.DeviceProfiles.from_synth(P)
    FP = c2.fingerprint(dP, torch.as_tensor(g.view(np.int32)).cuda(), B)
    ip, ix = orc.fingerprints(P.indptr, P.indices, P.n, g)
    assert FP.n == P.n and FP.m == B and FP.nnz == len(ix)
    assert np.array_equal(FP.indptr.cpu().numpy(), ip)
    assert np.array_equal(u32(FP.indices), ix)
    return dP, FP, ip, ix


@pytest.mark.parametrize("B", [1, 31, 64, 1000, 1024, 8192])
@pytest.mark.parametrize("n,m,lo,hi", [(1, 10, 1, 10), (257, 500, 1, 40), (1003, 20000, 50, 3000)])
def test_fingerprint(orc, n, m, lo, hi, B):
    say("fingerprint", n, m, B)
    P = synth.random_profiles(8000 + n, n, m, lo, hi, 1.0)
    g = orc.hash_items(synth.hash_tables(1, 8100 + B), B, m)[0]
    check_fingerprint(orc, P, g, B)


def test_fingerprint_rejects_bad_positions():
    P = synth.random_profiles(8200, 50, 100, 1, 10, 0.0)
    dP = c2.DeviceProfiles.from_synth(P)
    g = torch.zeros(P.m, dtype=torch.int32, device="cuda")
    g[int(P.indices[0])] = 64                 # >= B: detected on the device
    with pytest.raises(c2.C2Error):
        c2.fingerprint(dP, g, 64)
    for B in (0, 8193):
        with pytest.raises(c2.C2Error):
            c2.fingerprint(dP, g, B)


@pytest.mark.parametrize("name", ["n2k_m1k", "n6k_m3.7k"])
def test_goldfinger_build(orc, name):
    """Clusters from FastRandomHash on the profiles, local KNN and merge on
    1024-bit fingerprints, against the oracle's stages on the oracle's
    fingerprints."""
    w = synth.WORKLOADS[name]
    say("goldfinger", name)
    P = synth.make_profiles(w)
    tab = synth.hash_tables(w.t, w.hash_seed)
    B = 1024
    g = orc.hash_items(synth.hash_tables(1, w.hash_seed + 2), B, P.m)[0]
    dP, FP, ip, ix = check_fingerprint(orc, P, g, B)
    p = c2.params(w.t, w.b, w.cap, w.k)
    got = c2.build_goldfinger(dP, FP, c2.tables_to_device(tab), p)
    bucket = orc.hash_items(tab, w.b, P.m)
    om, ooff, ocfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, bucket, w.cap)
    pid, pI = orc.local_knn(ip, ix, P.n, B, w.t, w.k, om, ooff, ocfg, THREADS)
    want = orc.merge(ip, P.n, w.t, w.k, pid, pI)
    for a, b in zip(got, want):
        assert np.array_equal(u32(a), b)


@pytest.mark.parametrize("name", ["n140k_m27k", "n500k_m50k"])
def test_brute_force_sampled_large(orc, name):
    """The exact graph that scores every quality figure, at the two largest
    workloads: 200 seeded rows against the oracle's brute force over all n."""
    w = synth.WORKLOADS[name]
    say("brute force sampled", name)
    P = workload_profiles(name)
    dP = c2.DeviceProfiles.from_synth(P)
    bf = c2.brute_force(dP, w.k)
    torch.cuda.synchronize()
    rows = np.random.Generator(np.random.PCG64(17)).choice(P.n, size=200, replace=False)
    want = orc.brute_force(P.indptr, P.indices, P.n, P.m, w.k, rows=rows, threads=THREADS)
    for g, ww in zip(bf, want):
        assert np.array_equal(u32(g)[rows], ww)


# ------------------------------------------- per-cluster dictionaries ----

SHAPES = {"default": {}, "all128": dict(tile32_max=1, tile64_max=1),
          "all64": dict(tile32_max=1, tile64_max=1 << 30), "all32": dict(tile32_max=1 << 30)}


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("form", [c2.FORM_PLAIN, c2.FORM_BATCHED])
@pytest.mark.parametrize("name,P,tab,b,cap,k", CASES + [
    ("sparse", synth.random_profiles(9600, 3000, 20000, 5, 120, 1.0), synth.hash_tables(4, 9601),
     64, 400, 16)], ids=[c[0] for c in CASES] + ["sparse"])
def test_local_knn_tile_shapes(orc, name, P, tab, b, cap, k, form, shape):
    """The local KNN with each MFMA tile shape forced on every cluster (32-,
    64- and 128-row tiles: short row pieces, partial blocks and tiles that
    overhang the cluster) against the oracle on the oracle's partition."""
    say("local_knn shape", name, form, shape)
    t = tab.shape[0]
    om, ooff, ocfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, orc.hash_items(tab, b, P.m), cap)
    dP = c2.DeviceProfiles.from_synth(P)
    dev = lambda a: torch.as_tensor(a.astype(np.uint32).view(np.int32)).cuda()
    pid, pI = c2.local_knn(dP, dev(om), dev(ooff), dev(ocfg), c2.params(t, b, cap, k), form,
                           c2.tuning(**SHAPES[shape]))
    wid, wI = orc.local_knn(P.indptr, P.indices, P.n, P.m, t, k, om, ooff, ocfg, THREADS)
    assert np.array_equal(u32(pid), wid)
    assert np.array_equal(u32(pI), wI)


def _blocks_partition(n, t, size, seed):
    """t configurations, each a seeded permutation of the users cut into
    consecutive clusters of `size` (members ascending inside a cluster)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    members, off, cfg = [], [0], [0]
    for j in range(t):
        perm = np.arange(n) if j == 0 else rng.permutation(n)
        for a in range(0, n, size):
            members.append(np.sort(perm[a:a + size]))
            off.append(off[-1] + len(members[-1]))
        cfg.append(len(off) - 1)
    return (np.concatenate(members).astype(np.uint32), np.asarray(off, np.uint32),
            np.asarray(cfg, np.uint32))


def _store_words(P, om, ooff, k=10, group_tiles=16):
    """Words of store the partition needs: first the scratch of split row
    blocks (clusters of the 64 x 128 shape spanning more than group_tiles
    column tiles: ceil(s/64) row blocks times min(4, ceil(tiles/group_tiles))
    column groups, a slot of 64 rows x k u64 keys each; rounded up to 64
    words), then the dictionary rows: rows padded to 32 (or s below 32), 8
    words per 256 dictionary items (at least 8)."""
    ip = np.asarray(P.indptr)
    need, slots = 0, 0
    for c in range(len(ooff) - 1):
        mem = om[ooff[c]:ooff[c + 1]]
        if len(mem) < 2:
            continue
        s = len(mem)
        tiles = (s + 127) // 128
        if s > 64 and tiles > group_tiles:
            slots += (s + 63) // 64 * min(4, (tiles + group_tiles - 1) // group_tiles)
        items = np.concatenate([P.indices[ip[u]:ip[u + 1]] for u in mem])
        D = int((np.bincount(items, minlength=P.m) >= 2).sum())
        rows = s if s < 32 else (s + 31) // 32 * 32
        need += rows * 8 * max(1, (D + 255) // 256)
    return (slots * 64 * k * 2 + 63) // 64 * 64 + need


@pytest.mark.parametrize("group_tiles", [0, 2])
@pytest.mark.parametrize("form", [c2.FORM_PLAIN, c2.FORM_BATCHED])
def test_local_knn_store_sizes(orc, form, group_tiles):
    """The store takes whatever workspace the caller passes beyond the fixed
    part: exactly the partition's scratch and dictionary rows suffice and give
    the oracle's lists; one 256-word row block less is reported (plain form:
    C2_E_WORKSPACE from the call; batched form: from c2_check_complete).  With
    group_tiles 2 the 400-member clusters split their row blocks in two column
    groups, whose scratch takes the front of the store."""
    n, m, t, k, size = 3000, 16384, 2, 10, 400
    P = synth.random_profiles(77, n, m, 70, 95)
    om, ooff, ocfg = _blocks_partition(n, t, size, 78)
    need = _store_words(P, om, ooff, k, group_tiles or 16)
    tune = c2.tuning(group_tiles=group_tiles)
    say("local_knn store sizes", form, group_tiles, need)
    dP = c2.DeviceProfiles.from_synth(P)
    dev = lambda a: torch.as_tensor(a.astype(np.uint32).view(np.int32)).cuda()
    p = c2.params(t, 64, size, k)
    fixed = c2.workspace_bytes(dP, p, c2.OP_LOCAL_KNN_MIN) - 4096
    wid, wI = orc.local_knn(P.indptr, P.indices, P.n, P.m, t, k, om, ooff, ocfg, THREADS)
    ws = torch.empty(fixed + 4 * need, dtype=torch.uint8, device="cuda")
    pid, pI = c2.local_knn(dP, dev(om), dev(ooff), dev(ocfg), p, form, tune, ws=ws)
    if form == c2.FORM_BATCHED:
        c2.check_complete(ws)
    assert np.array_equal(u32(pid), wid)
    assert np.array_equal(u32(pI), wI)
    assert c2.store_need_bytes(ws) == 4 * need
    small = torch.empty(fixed + 4 * (need - 256), dtype=torch.uint8, device="cuda")
    with pytest.raises(c2.C2Error) as e:
        c2.local_knn(dP, dev(om), dev(ooff), dev(ocfg), p, form, tune, ws=small)
        c2.check_complete(small)
    assert e.value.status == -3
    assert c2.store_need_bytes(small) == 4 * need
    # the binding grows a workspace it allocated itself and runs again
    pid, pI = c2.local_knn(dP, dev(om), dev(ooff), dev(ocfg), p, c2.FORM_PLAIN, tune)
    assert np.array_equal(u32(pid), wid)


@pytest.mark.parametrize("form", [c2.FORM_PLAIN, c2.FORM_BATCHED])
def test_local_knn_clusters_of_thousands(orc, form):
    """Clusters of 8000, 6200 and 4100 members at the default schedule: their
    row blocks split into 4, 4 and 3 column groups whose lists the last group
    to finish merges from the scratch at the front of the store (the learned
    assigner's N = 8000 reaches such clusters); against the oracle's lists."""
    n, m, k = 18300, 4000, 30
    P = synth.random_profiles(79, n, m, 5, 40, 1.0)
    rng = np.random.Generator(np.random.PCG64(80))
    perm = rng.permutation(n)
    cuts = [0, 8000, 14200, 18300]
    om = np.concatenate([np.sort(perm[a:b]) for a, b in zip(cuts[:-1], cuts[1:])]).astype(np.uint32)
    ooff = np.asarray(cuts, np.uint32)
    ocfg = np.asarray([0, 3], np.uint32)
    say("local_knn clusters of thousands", form)
    dP = c2.DeviceProfiles.from_synth(P)
    dev = lambda a: torch.as_tensor(a.view(np.int32)).cuda()
    p = c2.params(1, 64, 8000, k)
    # sized by a plain run (the default store is smaller than these clusters need)
    ws = c2.local_knn_workspace(dP, dev(om), dev(ooff), dev(ocfg), p)
    assert ws.numel() > c2.workspace_bytes(dP, p, c2.OP_LOCAL_KNN)
    pid, pI = c2.local_knn(dP, dev(om), dev(ooff), dev(ocfg), p, form, ws=ws)
    if form == c2.FORM_BATCHED:
        c2.check_complete(ws)
    wid, wI = orc.local_knn(P.indptr, P.indices, P.n, P.m, 1, k, om, ooff, ocfg, THREADS)
    assert np.array_equal(u32(pid), wid)
    assert np.array_equal(u32(pI), wI)


@pytest.mark.parametrize("m", [200000, 1 << 19])
@pytest.mark.parametrize("form", [c2.FORM_PLAIN, c2.FORM_BATCHED])
def test_local_knn_wide_item_universe(orc, form, m):
    """Item universes beyond the 131,072 of the previous bit-row design: a
    DBLP-sized one (Table 1: 203,030 items) and the library's limit 2^19
    (dictionary bitmaps of 64 KiB each in LDS), against the oracle on the
    oracle's partition, and the whole build."""
    n, t, b, cap, k = 1500, 3, 16, 300, 12
    P = synth.random_profiles(91, n, m, 20, 400, 0.9)
    tab = synth.hash_tables(t, 92)
    om, ooff, ocfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, orc.hash_items(tab, b, P.m), cap)
    say("local_knn wide", form, m)
    dP = c2.DeviceProfiles.from_synth(P)
    dev = lambda a: torch.as_tensor(a.astype(np.uint32).view(np.int32)).cuda()
    wid, wI = orc.local_knn(P.indptr, P.indices, P.n, P.m, t, k, om, ooff, ocfg, THREADS)
    p = c2.params(t, b, cap, k)
    # long profiles over a wide universe need more store than the default: the
    # plain form reports the need (the binding then grows its workspace); the
    # batched form is given a workspace of that size and checked afterwards
    ws = torch.empty(c2.workspace_bytes(dP, p, c2.OP_LOCAL_KNN_MIN) + 4 * _store_words(P, om, ooff),
                     dtype=torch.uint8, device="cuda")
    pid, pI = c2.local_knn(dP, dev(om), dev(ooff), dev(ocfg), p, form,
                           ws=None if form == c2.FORM_PLAIN else ws)
    if form == c2.FORM_BATCHED:
        c2.check_complete(ws)
    assert np.array_equal(u32(pid), wid)
    assert np.array_equal(u32(pI), wI)
    wsb = torch.empty(c2.workspace_bytes(dP, p, c2.OP_BUILD) + 4 * _store_words(P, om, ooff),
                      dtype=torch.uint8, device="cuda")
    got = c2.build(dP, c2.tables_to_device(tab), p, form, c2.tuning(split_rounds=64),
                   ws=None if form == c2.FORM_PLAIN else wsb)
    if form == c2.FORM_BATCHED:
        c2.check_complete(wsb)
    r = orc.build_graph(P.indptr, P.indices, P.n, P.m, tab, b, cap, k, THREADS)
    for g, w in zip(got, (r.knn_id, r.knn_I, r.knn_U)):
        assert np.array_equal(u32(g), w)


def test_tile_shapes_agree_n6k():
    w = synth.WORKLOADS["n6k_m3.7k"]
    P = synth.make_profiles(w)
    dP, dtab = gpu_inputs(P, synth.hash_tables(w.t, w.hash_seed))
    p = c2.params(w.t, w.b, w.cap, w.k)
    ref = c2.build(dP, dtab, p, c2.FORM_BATCHED, c2.tuning(split_rounds=16))
    for shape in ("all128", "all32"):
        got = c2.build(dP, dtab, p, c2.FORM_BATCHED, c2.tuning(split_rounds=16, **SHAPES[shape]))
        torch.cuda.synchronize()
        for a, b2 in zip(ref, got):
            assert torch.equal(a, b2)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("name,t,cap", [("n140k_m27k", 32, 4000), ("n500k_m50k", 32, 4000)])
def test_workload_quality_setting(orc, name, t, cap):
    """The large workloads at the setting the benchmark reports at quality 0.95
    (32 hash configurations, N = 4000): the whole partition in both forms
    against the oracle's, and the tuned graph form's graph on sampled users
    against the definition (top-k over the users sharing a final cluster).
    The oracle's whole graph would take several minutes here."""
    w = synth.WORKLOADS[name]
    say("workload quality setting", name, t, cap)
    P = workload_profiles(name)
    tab = synth.hash_tables(t, w.hash_seed)
    dP, dtab = gpu_inputs(P, tab)
    p = c2.params(t, w.b, cap, w.k)
    om, ooff, ocfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, orc.hash_items(tab, w.b, w.m),
                                    cap)
    bucket = c2.hash_items(dtab, w.b, w.m)
    for form in (c2.FORM_PLAIN, c2.FORM_BATCHED):
        assert_same_partition(gpu_partition(dP, bucket, p, form), (om, ooff, ocfg))
    g = tuned_graph(dP, dtab, p, name, t, cap)
    out = [u32(x) for x in g.launch()]
    torch.cuda.synchronize()
    g.check()
    g.close()
    rows = np.random.Generator(np.random.PCG64(8)).choice(P.n, size=200, replace=False)
    want = orc.candidate_topk(P.indptr, P.indices, P.n, P.m, t, w.k, om, ooff, ocfg,
                              rows=rows, threads=THREADS)
    for a, ww in zip(out, want):
        assert np.array_equal(a[rows], ww)
