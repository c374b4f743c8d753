#!/usr/bin/env python3
"""Benchmark: Cluster-and-Conquer KNN-graph builds on one MI355X.

A step is one whole build of the method on one batch of synthetic input with
the profiles already resident in HBM: item hashing, FastRandomHash keys,
clustering with recursive splitting, brute-force local KNN in every cluster,
and the merge (Sections II-D to II-G).  The timed form is the batched build
replayed as a HIP graph; the plain (host-driven) form is timed beside it.

value = Jaccard evaluations per second of whole-build time, where a Jaccard
evaluation is one same-cluster pair (the paper's count of similarity
computations, Section II-F).  The line also carries the quality of the graph
against the exact graph (Eq. 2), the roofline of the dominant kernel (the
pairwise local-KNN kernel, timed with HIP events on its own stream), and the
CPU oracle timed on the host's cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Jaccard evals/s + KNN-graph build time at quality≥0.95, plain vs batched vs "
          "learned")
DEFAULT_WORKLOAD = "n6k_m3.7k"
VALU_PEAK = 256 * 4 * 16 * 2.4e9      # int32 lane-ops/s: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
MFMA_FP4_PEAK = 10.1e15               # dense fp4 (e2m1) MFMA flop/s
KNN_KERNEL = "k_knn_mfma"
MFMA_MIN_DEFAULT = 2                  # library default: clusters of >= 2 members take the MFMA path
KNN_SOURCES = ["paper_2010_11497_amd/csrc/k_knn.hip", "paper_2010_11497_amd/csrc/c2_internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    for f in KNN_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload):
    """HBM bytes per launch of the local-KNN kernel from the committed PMC
    summary (FETCH_SIZE and WRITE_SIZE scaled by a device copy of known size),
    only if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (KNN_KERNEL, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    return d.get("bytes_per_launch")


def mfma_busy_from_profiles(workload):
    """Hardware MFMA busy share of the local-KNN kernel (SQ_VALU_MFMA_BUSY_CYCLES
    over the dispatch's cycles times the SIMD count) from the committed PMC
    summary, only if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "%s_%s_mfma_busy.json" % (KNN_KERNEL, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    return d.get("mfma_busy_frac") if d.get("source_hash") == source_hash() else None


def cpu_baseline(P, tab, w, E, budget_s):
    """The oracle as it stands, on the host's cores, on whole builds of the same
    workload repeated until about budget_s seconds have passed."""
    from oracle import oracle
    threads = min(16, os.cpu_count() or 1)
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.build_graph(P.indptr, P.indices, P.n, P.m, tab, w.b, w.cap, w.k, threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el / reps * (reps + 1) > 3 * budget_s:
            break
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return {"value": E * reps / el, "unit": "Jaccard evals/s", "cores": threads, "kind": "oracle",
            "host_cpus": os.cpu_count(), "cpu_model": model,
            "sample": "%d whole build(s) of %s (hash, cluster, local KNN on a %d-thread pool "
                      "largest cluster first, merge): %.2f s each" % (reps, w.name, threads, el / reps)}


def upload_ms(P, torch, reps=5):
    """Time of the one-time host-to-device copy of the CSR (pinned source),
    the PCIe leg that the resident-input build time excludes."""
    hp = torch.from_numpy(P.indptr).pin_memory()
    hi = torch.from_numpy(P.indices.view("int32")).pin_memory()
    dp = torch.empty_like(hp, device="cuda")
    di = torch.empty_like(hi, device="cuda")
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dp.copy_(hp, non_blocking=True)
        di.copy_(hi, non_blocking=True)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return sorted(ts)[len(ts) // 2]


def minhash_ablation(args, w, P, dP, c2, metrics, synth, torch, np, bf):
    """The paper's MinHash variant of the clustering (Section V-C, Table 4): t
    min-wise permutations of the items as bucket tables (b = m), no split,
    then the same local KNN and merge.  Timed in the plain eager form, beside
    which the FastRandomHash build's plain form is reported."""
    tab = synth.minhash_tables(w.t, w.m, w.hash_seed + 1)
    dtab = torch.as_tensor(tab.view(np.int32)).cuda()
    p = c2.params(w.t, w.m, w.n, w.k)
    members, cl_off, cfg, _ = c2.cluster(dP, dtab, p, c2.FORM_PLAIN)
    ncl = int(c2.to_u32(cfg)[-1])
    work = metrics.cluster_work(c2.to_u32(members), c2.to_u32(cl_off)[: ncl + 1], P.indptr,
                                P.indices, P.m)
    out = None
    for _ in range(args.warmup):
        out = c2.build_from_buckets(dP, dtab, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = c2.build_from_buckets(dP, dtab, p)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    q = None
    if bf is not None:
        q = metrics.quality(c2.to_u32(out[1]), c2.to_u32(out[2]), c2.to_u32(bf[1]),
                            c2.to_u32(bf[2]))
    log("MinHash clustering: %d clusters, max %d, %d evals, plain build %.3f ms, quality %s"
        % (ncl, int(work["sizes"].max()), work["pairs"], ms, q))
    return {"build_ms_plain": ms, "quality": q, "jaccard_evals": int(work["pairs"]),
            "clusters": ncl, "max_cluster": int(work["sizes"].max()),
            "tables": "t seeded permutations of the m items (b = m), cap = n"}


def goldfinger_variant(args, w, P, dP, c2, metrics, synth, torch, np, bf, B=1024):
    """The paper's default local similarity (Section II-F, Section V-D and
    Table 5): the same clusters, local KNN and merge on B-bit GoldFinger
    fingerprints.  The fingerprints are computed once (timed apart); the
    graph is scored by the exact similarity of the edges it chose."""
    gtab = c2.tables_to_device(synth.hash_tables(1, w.hash_seed + 2))
    dtab = c2.tables_to_device(synth.hash_tables(w.t, w.hash_seed))
    g = c2.hash_items(gtab, B, w.m)[0]
    p = c2.params(w.t, w.b, w.cap, w.k)
    ws = c2.workspace(dP, c2.params(1, B, 1, 1), c2.OP_FINGERPRINT)
    FP = c2.fingerprint(dP, g, B, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        FP = c2.fingerprint(dP, g, B, ws)
    fp_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    out = None
    for _ in range(args.warmup):
        out = c2.build_goldfinger(dP, FP, dtab, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = c2.build_goldfinger(dP, FP, dtab, p)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    q = None
    if bf is not None:
        I, U = metrics.edge_jaccard(P.indptr, P.indices, P.m, c2.to_u32(out[0]))
        q = metrics.quality(I, U, c2.to_u32(bf[1]), c2.to_u32(bf[2]))
    log("GoldFinger %d bits: fingerprints %.3f ms (nnz %d -> %d), plain build %.3f ms, "
        "quality %s" % (B, fp_ms, P.nnz, FP.nnz, ms, q))
    return {"bits": B, "fingerprint_ms": fp_ms, "fingerprint_nnz": FP.nnz,
            "build_ms_plain": ms, "quality": q,
            "quality_def": "exact similarity of the chosen edges over the exact graph's"}


def time_to_quality(args, w, P, dP, c2, metrics, synth, torch, np, bf,
                    ts=(1, 2, 4, 8, 10, 12, 16), caps=(500, 1000, 2000, 3000, 4000, 10000)):
    """The synthetic analogue of the paper's sensitivity study (Section VI,
    Figs. 6-7): plain builds over the number of hash configurations t (nested
    tables) and the split threshold N, each timed and scored against the exact
    graph, next to the brute force itself (quality 1).  The fastest setting with
    quality >= 0.95 is also timed as a HIP-graph replay of the batched form."""
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c2.brute_force(dP, w.k)
    torch.cuda.synchronize()
    res = {"brute_force_ms": (time.perf_counter() - t1) * 1e3, "points": []}
    eI, eU = c2.to_u32(bf[1]), c2.to_u32(bf[2])
    reps = 3
    for t in ts:
        dtab = c2.tables_to_device(synth.hash_tables(t, w.hash_seed))
        for cap in caps:
            p = c2.params(t, w.b, cap, w.k)
            ws = c2.build_workspace(dP, dtab, p)
            out = c2.build(dP, dtab, p, c2.FORM_PLAIN, ws=ws)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(reps):
                out = c2.build(dP, dtab, p, c2.FORM_PLAIN, ws=ws, out=out)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t1) * 1e3 / reps
            q = metrics.quality(c2.to_u32(out[1]), c2.to_u32(out[2]), eI, eU)
            res["points"].append({"t": t, "N": cap, "build_ms_plain": ms, "quality": q})
            log("t=%2d N=%5d: plain build %8.3f ms, quality %.4f" % (t, cap, ms, q))
    ok = [x for x in res["points"] if x["quality"] >= 0.95]
    if ok:
        best = min(ok, key=lambda x: x["build_ms_plain"])
        dtab = c2.tables_to_device(synth.hash_tables(best["t"], w.hash_seed))
        p = c2.params(best["t"], w.b, best["N"], w.k)
        from paper_2010_11497_amd import autotune
        tuned = autotune.load_table(w.name) if (best["t"], best["N"]) == (w.t, w.cap) else None
        g = c2.Graph(dP, dtab, p, c2.tuning(**(tuned or {})))
        g.launch()
        torch.cuda.synchronize()
        g.check()
        t1 = time.perf_counter()
        for _ in range(reps):
            g.launch()
        torch.cuda.synchronize()
        best = dict(best, build_ms_graph=(time.perf_counter() - t1) * 1e3 / reps)
        g.close()
        res["fastest_at_0.95"] = best
        log("fastest setting with quality >= 0.95: %s" % best)
    return res


def hyrec_variant(args, w, P, dP, dtab, c2, metrics, torch, np, bf, rho=5):
    """Algorithm 2's two branches side by side: the workload clustered
    without splitting (cap = n, so the large top-level clusters reach rho*k^2
    members), then the local KNN by brute force everywhere (c2_local_knn) and
    by Algorithm 2 (Hyrec in the clusters of at least rho*k^2 members), each
    merged and scored."""
    p = c2.params(w.t, w.b, P.n, w.k)
    bucket = c2.hash_items(dtab, w.b, w.m)
    members, cl_off, cfg, _ = c2.cluster(dP, bucket, p, c2.FORM_PLAIN)
    ncl = int(c2.to_u32(cfg)[-1])
    sizes = np.diff(c2.to_u32(cl_off)[: ncl + 1].astype(np.int64))
    big = sizes >= rho * w.k * w.k
    res = {"rho": rho, "clusters": ncl, "hyrec_clusters": int(big.sum()),
           "hyrec_members": int(sizes[big].sum()), "max_cluster": int(sizes.max())}
    ws_bf = c2.workspace(dP, p, c2.OP_LOCAL_KNN)
    ws_a2 = c2.workspace(dP, p, c2.OP_LOCAL_KNN_ALG2)
    for name, fn in (("brute_force", lambda: c2.local_knn(dP, members, cl_off, cfg, p, ws=ws_bf)),
                     ("alg2", lambda: c2.local_knn_alg2(dP, members, cl_off, cfg, p, rho=rho,
                                                         ws=ws_a2))):
        part = fn()
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 5))
        t1 = time.perf_counter()
        for _ in range(reps):
            part = fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / reps
        out = c2.merge(dP, part[0], part[1], p)
        q = None
        if bf is not None:
            q = metrics.quality(c2.to_u32(out[1]), c2.to_u32(out[2]), c2.to_u32(bf[1]),
                                c2.to_u32(bf[2]))
        res[name] = {"local_knn_ms": ms, "quality": q}
        log("unsplit clusters, %s: local KNN %.3f ms, quality %s" % (name, ms, q))
    return res


def learned_graph(args, A, dP, tab, p, gap, tb, W, ref, c2, torch, learned):
    """The batched learned build captured once as a graph, with the fewest
    split rounds that complete, and replayed: the time per replay, and whether
    every replay (checked after each, with the split-round status) equals the
    eager batched result `ref`."""
    try:
        # the fewest split rounds that complete on this data (synchronous
        # status check), as the FastRandomHash graph learns them from a plain run
        rounds = 64
        for r in (2, 4, 8, 16, 32):
            try:
                learned.build(A, dP, tab, p, gap, c2.FORM_BATCHED, c2.tuning(split_rounds=r),
                              weights=W)
                rounds = r
                break
            except c2.C2Error:
                continue
        tb = c2.tuning(split_rounds=rounds)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, capture_error_mode="thread_local"):
            gout, gws = learned.build(A, dP, tab, p, gap, c2.FORM_BATCHED, tb, weights=W,
                                      check=False, with_ws=True)
        equal = True
        for _ in range(max(args.warmup, 2)):
            g.replay()
            torch.cuda.synchronize()
            c2.check_complete(gws)
            equal &= all(torch.equal(a, b) for a, b in zip(gout, ref))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / args.steps
        c2.check_complete(gws)
        equal &= all(torch.equal(a, b) for a, b in zip(gout, ref))
        del g
        return {"build_ms_graph": ms, "graph_split_rounds": rounds,
                "graph_equals_eager": bool(equal)}
    except Exception as e:  # report, do not lose the rest of the leg
        return {"build_ms_graph": None, "graph_error": str(e)[:200]}


def learned_variant(args, w, P, dP, dtab, p, c2, metrics, torch, np, bf, plain_ms, batched_ms):
    """The learned cluster assigner: trained here on exact KNN edges of a
    100,000-user subsample, then the learned-assignment build (assignment,
    clustering from keys with FastRandomHash splits, local KNN, merge) timed in
    the plain and batched eager forms and scored against the exact graph.  Heads
    and split threshold default to the workload's t and N."""
    from paper_2010_11497_amd import learned, synth
    b = 8192 if w.n >= 100000 else w.b
    T = args.learned_t or w.t
    cap = args.learned_cap or w.cap
    t0 = time.perf_counter()
    pairs = learned.exact_pairs(P, 100000, w.k, seed=1)
    A = learned.Assigner(P.m, T, b, seed=2)
    st = learned.train(A, dP, pairs, steps=args.learned_steps, batch=2048, w_bal=1.0, w_neg=1.0,
                       w_ent=1.0, lr=3e-3, log=log)
    train_s = time.perf_counter() - t0
    W = A.inference_weights()
    tabT = c2.tables_to_device(synth.hash_tables(T, w.hash_seed)) if T != w.t else dtab
    pT = c2.params(T, w.b, cap, w.k)
    res = {"buckets": b, "heads": T, "N": cap, "train_s": train_s, "train_steps": st.steps,
           "train_pairs": st.pairs, "loss": [st.first_loss, st.last_loss], "min_gap": {}}
    tb = c2.tuning(split_rounds=64)
    for gap in (0.0, 0.5):
        entry = {}
        for form, tu, key in ((c2.FORM_PLAIN, None, "build_ms_plain"),
                              (c2.FORM_BATCHED, tb, "build_ms_batched")):
            out = None
            for _ in range(args.warmup):
                out = learned.build(A, dP, tabT, pT, gap, form, tu, weights=W)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                out = learned.build(A, dP, tabT, pT, gap, form, tu, weights=W)
            torch.cuda.synchronize()
            entry[key] = (time.perf_counter() - t1) * 1e3 / args.steps
        entry.update(learned_graph(args, A, dP, tabT, pT, gap, tb, W, out, c2, torch, learned))
        q = None
        if bf is not None:
            q = metrics.quality(c2.to_u32(out[1]), c2.to_u32(out[2]), c2.to_u32(bf[1]),
                                c2.to_u32(bf[2]))
        entry["quality"] = q
        res["min_gap"][str(gap)] = entry
        log("learned assigner (t=%d, N=%d, min_gap %.1f): plain %.3f ms, batched %.3f ms, "
            "graph %s ms (equal %s), quality %s" % (T, cap, gap, entry["build_ms_plain"],
                                                   entry["build_ms_batched"],
                                                   entry.get("build_ms_graph"),
                                                   entry.get("graph_equals_eager"), q))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        A.keys(dP, None, 0.0, W)
    torch.cuda.synchronize()
    res["assign_ms"] = (time.perf_counter() - t1) * 1e3 / args.steps
    res["frh_build_ms"] = {"plain": plain_ms, "batched": batched_ms}
    # FastRandomHash's time to the same quality bar: more hash configurations
    # until the graph reaches quality 0.95 (plain form)
    if bf is not None:
        from paper_2010_11497_amd import synth
        sweep = []
        for t in (w.t, w.t + 2, w.t + 4, w.t + 8):
            tab_t = c2.tables_to_device(synth.hash_tables(t, w.hash_seed))
            p_t = c2.params(t, w.b, w.cap, w.k)
            out = c2.build(dP, tab_t, p_t, c2.FORM_PLAIN)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                out = c2.build(dP, tab_t, p_t, c2.FORM_PLAIN)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t1) * 1e3 / args.steps
            q = metrics.quality(c2.to_u32(out[1]), c2.to_u32(out[2]), c2.to_u32(bf[1]),
                                c2.to_u32(bf[2]))
            sweep.append({"t": t, "build_ms_plain": ms, "quality": q})
            log("FastRandomHash t=%d: plain build %.3f ms, quality %.4f" % (t, ms, q))
            if q >= 0.95:
                break
        res["frh_t_sweep"] = sweep
    log("assignment (hidden layer + keys) %.3f ms; training %.1f s" % (res["assign_ms"], train_s))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the MinHash-clustering (Table 4) and GoldFinger (Table 5) "
                         "variants")
    ap.add_argument("--learned", action="store_true",
                    help="also train the learned cluster assigner on this workload and time the "
                         "learned-assignment build beside the FastRandomHash forms")
    ap.add_argument("--learned-steps", type=int, default=1000)
    ap.add_argument("--learned-t", type=int, default=0,
                    help="heads (hash configurations) of the learned build (default: the workload's t)")
    ap.add_argument("--learned-cap", type=int, default=0,
                    help="split threshold N of the learned build (default: the workload's)")
    ap.add_argument("--sweep", action="store_true",
                    help="time-to-quality curve: plain builds over t and the split threshold N, "
                         "beside GPU brute force, and the fastest setting with quality >= 0.95")
    ap.add_argument("--sweep-t", default="1,2,4,8,10,12,16",
                    help="hash-configuration counts of the sweep (comma separated)")
    ap.add_argument("--sweep-n", default="500,1000,2000,3000,4000,10000",
                    help="split thresholds N of the sweep (comma separated)")
    ap.add_argument("--hyrec", action="store_true",
                    help="also time Algorithm 2 (Hyrec in clusters of at least 5k^2 members) "
                         "against brute force on the workload's unsplit clusters")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X and has no "
              "multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2010_11497_amd import c2, metrics, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = synth.WORKLOADS[args.workload]
    log("workload", w.name, "n=%d m=%d t=%d b=%d cap=%d k=%d" % (w.n, w.m, w.t, w.b, w.cap, w.k))
    P = synth.make_profiles(w)
    tab = synth.hash_tables(w.t, w.hash_seed)
    dP = c2.DeviceProfiles.from_synth(P)
    h2d_ms = upload_ms(P, torch)
    log("CSR upload from pinned host memory: %.3f ms" % h2d_ms)
    dtab = c2.tables_to_device(tab)
    p = c2.params(w.t, w.b, w.cap, w.k)
    c2.validate(dP)

    # partition statistics for the work counts (GPU clustering, read back)
    bucket = c2.hash_items(dtab, w.b, w.m)
    members, cl_off, cfg, _ = c2.cluster(dP, bucket, p, c2.FORM_PLAIN)
    ncl = int(c2.to_u32(cfg)[-1])
    work = metrics.cluster_work(c2.to_u32(members), c2.to_u32(cl_off)[: ncl + 1], P.indptr,
                                P.indices, P.m)
    E = work["pairs"]
    log("clusters %d, Jaccard evals %d, max cluster %d" % (ncl, E, int(work["sizes"].max())))

    # HIP-graph form of the batched build, with the autotuner's schedule if one
    # was recorded for this workload
    from paper_2010_11497_amd import autotune
    tuned = autotune.load_table(w.name) or {}
    log("tuning", tuned if tuned else "built-in defaults")
    g = c2.Graph(dP, dtab, p, c2.tuning(**tuned))
    for _ in range(args.warmup):
        g.launch()
    torch.cuda.synchronize()
    g.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.launch()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    log("graph build: %.3f ms/step" % graph_ms)
    out_graph = [c2.to_u32(x) for x in g.out]

    # batched (eager) and plain forms, same arithmetic
    def timed(form):
        ws = torch.empty_like(g.ws)
        tu = c2.tuning(**tuned)
        out = None
        for _ in range(args.warmup):
            out = c2.build(dP, dtab, p, form, tu, ws=ws, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = c2.build(dP, dtab, p, form, tu, ws=ws, out=out)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps, [c2.to_u32(x) for x in out]
    batched_ms, out_b = timed(c2.FORM_BATCHED)
    plain_ms, out_p = timed(c2.FORM_PLAIN)

    # dominant kernel: HIP events that the library records on its stream right
    # before and after the pairwise local-KNN kernel, over K batched builds
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    ws = torch.empty_like(g.ws)
    tu = c2.tuning(events=ev, **tuned)
    out = None
    knn = []
    for _ in range(args.steps):
        out = c2.build(dP, dtab, p, c2.FORM_BATCHED, tu, ws=ws, out=out)
        ev[1].synchronize()
        knn.append(ev[0].elapsed_time(ev[1]))
    knn_ms = sum(knn) / len(knn)
    log("local-KNN kernel: %.3f ms (events, avg of %d batched builds)" % (knn_ms, len(knn)))
    log("batched eager: %.3f ms, plain: %.3f ms" % (batched_ms, plain_ms))
    same = all(np.array_equal(a, b) for a, b in zip(out_graph, out_b)) and \
        all(np.array_equal(a, b) for a, b in zip(out_graph, out_p))
    if not same:
        raise SystemExit("forms disagree: graph, batched and plain builds differ")

    if args.calibrate_copy_mb:
        src = torch.empty(args.calibrate_copy_mb << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d MiB x 3" % args.calibrate_copy_mb)

    quality = None
    if not args.no_quality:
        bf = c2.brute_force(dP, w.k)
        torch.cuda.synchronize()
        quality = metrics.quality(out_graph[1], out_graph[2], c2.to_u32(bf[1]), c2.to_u32(bf[2]))
        log("quality %.4f" % quality)

    learned_leg = None
    if args.learned:
        learned_leg = learned_variant(args, w, P, dP, dtab, p, c2, metrics, torch, np,
                                      bf if quality is not None else None, plain_ms, batched_ms)
    sweep_leg = None
    if args.sweep and quality is not None:
        sweep_leg = time_to_quality(args, w, P, dP, c2, metrics, synth, torch, np, bf,
                                    tuple(int(x) for x in args.sweep_t.split(",")),
                                    tuple(int(x) for x in args.sweep_n.split(",")))
    hyrec_leg = None
    if args.hyrec:
        hyrec_leg = hyrec_variant(args, w, P, dP, dtab, c2, metrics, torch, np,
                                  bf if quality is not None else None)
    ablation = gold = None
    if not args.no_ablation:
        ablation = minhash_ablation(args, w, P, dP, c2, metrics, synth, torch, np,
                                    bf if quality is not None else None)
        gold = goldfinger_variant(args, w, P, dP, c2, metrics, synth, torch, np,
                                  bf if quality is not None else None)

    mfma_min = int(tuned.get("mfma_min_rows", MFMA_MIN_DEFAULT))
    big = work["sizes"] >= mfma_min
    ops = int((2 * work["sizes"][big].astype(np.int64) ** 2 * work["dict"][big]).sum())
    achieved = ops / (knn_ms * 1e-3)
    roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": MFMA_FP4_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": achieved / MFMA_FP4_PEAK,
            "traffic": traffic_from_profiles(w.name), "kernel": KNN_KERNEL,
            "hw_mfma_busy_frac": mfma_busy_from_profiles(w.name),
            "ops_per_launch": ops,
            "sparse_lower_bound_ops": int(work["sparse_pairs"]),
            "ops_def": "sum over clusters with >= %d members of 2*s^2*D: the 0/1 product of the "
                       "members' rows over the cluster's local dictionary (D = items held by >= "
                       "2 members), computed on e2m1 (fp4) MFMA with fp32 accumulation, exact"
                       % mfma_min}

    line = {
        "metric": METRIC, "value": E / (graph_ms * 1e-3), "unit": "Jaccard evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": graph_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp4",
        "data": "synthetic: seeded lognormal profile sizes, Zipf item popularity",
        "config": {"workload": w.name, "n": w.n, "m": w.m, "nnz": P.nnz, "t": w.t, "b": w.b,
                   "cap": w.cap, "k": w.k, "form": "batched build replayed as a HIP graph",
                   "tuning": tuned or "defaults"},
        "build_ms": {"graph": graph_ms, "batched": batched_ms, "plain": plain_ms},
        "quality": quality, "jaccard_evals": E, "clusters": ncl,
        "evals_vs_brute_force": E / (P.n * (P.n - 1) / 2),
        "minhash_ablation": ablation, "goldfinger": gold, "learned": learned_leg, "hyrec": hyrec_leg, "time_to_quality": sweep_leg,
        "h2d_csr_ms": h2d_ms, "evals_per_s_incl_h2d": E / ((graph_ms + h2d_ms) * 1e-3),
        "local_knn_ms": knn_ms, "local_knn_evals_per_s": E / (knn_ms * 1e-3),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(P, tab, w, E, args.cpu_budget)
        line["cpu_baseline"] = cb
        log("cpu oracle: %.3g evals/s on %d threads" % (cb["value"], cb["cores"]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
