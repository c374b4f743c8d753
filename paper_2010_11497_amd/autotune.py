"""Autotuner for the local-KNN schedule of libc2.so.

For one workload it builds the graph form of the batched build for every
point of a small grid over the c2_tuning fields that change the schedule and
the tile shapes but not the arithmetic -- persistent waves of the MFMA
launch, how many column tiles a work item takes before a row block is split,
and the cluster sizes up to which 32- and 64-row tiles are used (128 above)
-- times each (median of repeated replays), checks that every point produces
the same graph, and writes the fastest point to tuning/<workload>.json.
bench.py reads that table.

Run on the GPU:  python -m paper_2010_11497_amd.autotune --workload n6k_m3.7k
(each grid axis can be replaced from the command line, e.g. --mfma-min-rows 2,64)
"""
import argparse
import itertools
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_DIR = os.path.join(HERE, "tuning")
GRID = {
    "persistent_wgs": [1024],
    "group_tiles": [2, 4, 8, 16, 32],
    "tile32_max": [16, 32],
    "tile64_max": [64, 96],
}


def table_path(workload: str) -> str:
    return os.path.join(TABLE_DIR, "%s.json" % workload)


def load_table(workload: str):
    """The tuned c2_tuning fields for a workload, or None."""
    path = table_path(workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)["best"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="n6k_m3.7k")
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--out", default=None)
    for key in GRID:
        ap.add_argument("--" + key.replace("_", "-"), default=None,
                        help="comma-separated values (default %s)" % GRID[key])
    args = ap.parse_args()
    grid = {key: ([int(x) for x in getattr(args, key).split(",")] if getattr(args, key)
                  else GRID[key]) for key in GRID}

    import numpy as np
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2010_11497_amd import c2, synth

    w = synth.WORKLOADS[args.workload]
    P = synth.make_profiles(w)
    tab = synth.hash_tables(w.t, w.hash_seed)
    dP = c2.DeviceProfiles.from_synth(P)
    dtab = c2.tables_to_device(tab)
    p = c2.params(w.t, w.b, w.cap, w.k)
    results, ref = [], None
    for vals in itertools.product(*grid.values()):
        point = dict(zip(grid.keys(), vals))
        g = c2.Graph(dP, dtab, p, c2.tuning(**point))
        for _ in range(2):
            g.launch()
        torch.cuda.synchronize()
        g.check()
        ts = []
        for _ in range(args.reps):
            t0 = time.perf_counter()
            g.launch()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        out = [c2.to_u32(x) for x in g.out]
        g.close()
        if ref is None:
            ref = out
        elif not all(np.array_equal(a, b) for a, b in zip(out, ref)):
            raise SystemExit("tuning point %s changed the graph" % point)
        ms = float(np.median(ts))
        results.append({"point": point, "build_ms": ms})
        print(json.dumps({"workload": w.name, **point, "build_ms": round(ms, 4)}), flush=True)
    best = min(results, key=lambda r: r["build_ms"])
    out = {"workload": w.name, "best": best["point"], "best_build_ms": best["build_ms"],
           "grid": grid, "results": results,
           "device": torch.cuda.get_device_name(0)}
    path = args.out or table_path(w.name)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("best", json.dumps(best), "->", path, flush=True)


if __name__ == "__main__":
    main()
