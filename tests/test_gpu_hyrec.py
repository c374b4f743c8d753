"""GPU parity of Algorithm 2 (brute force below rho*k^2 members, the
deterministic Hyrec at or above) against the oracle, through the C ABI."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_11497_amd import c2, synth  # noqa: E402

THREADS = 16


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle


def run_both(orc, P, mem, off, cfg, t, k, rho=5, max_iter=30, seed=0):
    dP = c2.DeviceProfiles.from_synth(P)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()
    got = c2.local_knn_alg2(dP, d(mem), d(off), d(cfg), c2.params(t, 1, P.n, k), rho, max_iter,
                            0.001, seed)
    torch.cuda.synchronize()
    want = orc.local_knn_alg2(P.indptr, P.indices, P.n, P.m, t, k, mem, off, cfg, rho, 0.001,
                              max_iter, seed, THREADS)
    return [c2.to_u32(x) for x in got], want


@pytest.mark.parametrize("n,k,lo,hi,seed,max_iter", [(400, 8, 2, 25, 1, 30), (700, 10, 5, 60, 2, 30),
                                                     (5200, 32, 2, 8, 3, 3), (81, 4, 1, 10, 4, 30)])
def test_hyrec_single_cluster(orc, n, k, lo, hi, seed, max_iter):
    say("hyrec single cluster", n, k)
    P = synth.random_profiles(9000 + n, n, 150, lo, hi, 1.0)
    mem = np.arange(n, dtype=np.uint32)
    got, want = run_both(orc, P, mem, np.array([0, n]), np.array([0, 1]), 1, k,
                         max_iter=max_iter, seed=seed)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


@pytest.mark.parametrize("name,P,t,b,cap,k", [
    ("mixed", synth.random_profiles(9100, 3000, 800, 2, 40, 1.0), 3, 4, 3000, 10),
    ("capped", synth.random_profiles(9102, 2500, 600, 2, 30, 1.0), 4, 8, 400, 8),
])
def test_alg2_on_a_partition(orc, name, P, t, b, cap, k):
    """Clusters below and above rho*k^2 in one partition: split clusters just
    under N and stay-behind groups above it."""
    say("alg2 partition", name)
    tab = synth.hash_tables(t, 9101 if name == "mixed" else 9103)
    bucket = orc.hash_items(tab, b, P.m)
    mem, off, cfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, bucket, cap)
    sizes = np.diff(off.astype(np.int64))
    assert (sizes >= 5 * k * k).any() and (sizes < 5 * k * k).any()
    got, want = run_both(orc, P, mem, off, cfg, t, k, seed=7)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_alg2_without_big_clusters_is_local_knn(orc):
    P = synth.random_profiles(9200, 500, 300, 1, 30, 1.0)
    tab = synth.hash_tables(2, 9201)
    bucket = orc.hash_items(tab, 16, P.m)
    mem, off, cfg, _ = orc.cluster(P.indptr, P.indices, P.n, P.m, bucket, 60)
    got, _ = run_both(orc, P, mem, off, cfg, 2, 5, rho=1000)
    dP = c2.DeviceProfiles.from_synth(P)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()
    ref = c2.local_knn(dP, d(mem), d(off), d(cfg), c2.params(2, 1, 60, 5))
    torch.cuda.synchronize()
    assert np.array_equal(got[0], c2.to_u32(ref[0])) and np.array_equal(got[1], c2.to_u32(ref[1]))


def test_alg2_rejects_long_profiles_in_hyrec_clusters():
    m = 40000
    sets = [set(range(0, m, 1))] + [{i, i + 1} for i in range(99)]
    P = synth.profiles_from_sets(sets, m)
    dP = c2.DeviceProfiles.from_synth(P)
    n = P.n
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()
    with pytest.raises(c2.C2Error):
        c2.local_knn_alg2(dP, d(np.arange(n)), d([0, n]), d([0, 1]), c2.params(1, 1, n, 2))
