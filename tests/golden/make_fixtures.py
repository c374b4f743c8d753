"""Writes the hand-built clustering fixtures in this folder.

Expected values come from how each fixture is built, not from any
implementation: users are drawn into groups whose FastRandomHash values are
fixed by construction, so the partition the method must produce is known.
Run: python tests/golden/make_fixtures.py
"""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def fig3():
    """Recursive splitting example of Section II-D (Fig. 3): 100 users, b = 3,
    N = 40.  The first top-level cluster holds 75 users and is split with
    H minus its index into 18 users that stay (no item hashed above it), 34
    and 23; the other two top-level clusters hold 10 and 15 users.  Buckets are
    numbered from 0 here, the paper numbers them from 1."""
    rng = np.random.Generator(np.random.PCG64(7))
    m, b, N = 30, 3, 40
    bucket = [i // 10 for i in range(m)]          # items 0-9 -> 0, 10-19 -> 1, 20-29 -> 2
    b0, b1, b2 = list(range(0, 10)), list(range(10, 20)), list(range(20, 30))

    def pick(pool, lo, hi):
        k = int(rng.integers(lo, hi + 1))
        return [int(x) for x in rng.choice(pool, size=k, replace=False)]

    groups = {"stay": [], "to_1": [], "to_2": [], "top_1": [], "top_2": []}
    profiles = []
    plan = ["stay"] * 18 + ["to_1"] * 34 + ["to_2"] * 23 + ["top_1"] * 10 + ["top_2"] * 15
    order = rng.permutation(len(plan))
    for u, gi in enumerate(order):
        g = plan[gi]
        if g == "stay":
            p = pick(b0, 1, 4)
        elif g == "to_1":
            p = pick(b0, 1, 3) + pick(b1, 1, 3) + (pick(b2, 1, 2) if rng.random() < 0.5 else [])
        elif g == "to_2":
            p = pick(b0, 1, 3) + pick(b2, 1, 3)
        elif g == "top_1":
            p = pick(b1, 1, 3) + (pick(b2, 1, 2) if rng.random() < 0.5 else [])
        else:
            p = pick(b2, 1, 4)
        profiles.append(sorted(p))
        groups[g].append(u)
    return {
        "citation": "Section II-D, recursive splitting, Fig. 3 (|U|=100, b=3, N=40; sizes 75, 10, 15; "
                    "the 75 split into 18, 34, 23)",
        "m": m, "b": b, "cap": N, "bucket": [bucket],
        "profiles": profiles,
        "expected_clusters": [sorted(groups[g]) for g in ["to_1", "to_2", "stay", "top_1", "top_2"]],
        "expected_sizes": [34, 23, 18, 10, 15],
    }


def singleton_stays():
    """Users alone in their new cluster stay in the split cluster (Section II-D).
    One top-level cluster of 6 users, N = 3.  Next hash values: 1, 1, 2, 3,
    none, none.  The pair with value 1 forms a new cluster; the users with 2
    and 3 are alone and stay, with the two users that have no item above 0."""
    m, b, cap = 8, 4, 3
    bucket = [0, 0, 1, 1, 2, 3, 0, 0]
    profiles = [[0, 2], [1, 3], [0, 4], [1, 5], [0], [1, 6, 7]]
    return {
        "citation": "Section II-D: users alone in their new cluster remain in the split cluster",
        "m": m, "b": b, "cap": cap, "bucket": [bucket], "profiles": profiles,
        "expected_clusters": [[0, 1], [2, 3, 4, 5]],
        "expected_sizes": [2, 4],
    }


def worked_example():
    """FastRandomHash worked examples of Section II-D (Eq. 3 and Fig. 2): items
    i1..i5, b = 3, h1 = (2, 3, 2, 1, 3), h2 = (1, 3, 3, 2, 1) in the paper's
    1-based buckets; P_u = {i1, i2, i3}, P_v = {i3, i4, i5}.  H1(u) = 2,
    H1(v) = 1, H2(u) = H2(v) = 1.  Here items and buckets are 0-based."""
    return {
        "citation": "Section II-D: the Eq. 3 example (Fig. 2) and the second hash function example",
        "m": 5, "b": 3,
        "bucket": [[1, 2, 1, 0, 2], [0, 2, 2, 1, 0]],
        "profiles": [[0, 1, 2], [2, 3, 4]],
        "expected_keys": [[1, 0], [0, 0]],
        # with k = 1 and no split: u and v are co-clustered only under h2; they
        # share i3, so I = 1 and U = 5
        "expected_knn": {"id": [[1], [0]], "I": [[1], [1]], "U": [[5], [5]]},
        "expected_clusters_per_config": [[[1], [0]], [[0, 1]]],
    }


if __name__ == "__main__":
    for name, fn in [("fig3_split.json", fig3), ("singleton_stays.json", singleton_stays),
                     ("frh_worked_example.json", worked_example)]:
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(fn(), f, indent=1)
        print("wrote", name)
