"""Benchmark: exact top-k closeness on one MI355X.

One step = one whole top-k query on a resident graph (reachability, initial
bounds, processing order, pruned searches, readback), on the undirected
Barabasi-Albert workload n = 2^20, m = 5, seed 2 (5,242,865 edges), k = 10.

Prints one JSON line.  value = GTEPS = arcs scanned by the searches (the
paper's work count m_vis) / wall time of the step.  roofline: the dominant
traversal kernel's algorithmic bytes over its HIP-event time (measured by
the library on the stream it launches on).  cpu_baseline: the CPU oracle
(textbook BFS) timed on a bounded sample of sources of the same graph.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "top-k closeness wall time & GTEPS (frac. HBM peak), batched vs plain; p50/p99"
HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {0: "k_plain", 1: "k_batch", 2: "k_swarm"}
MODE_NAMES = {0: "plain", 1: "batched", 2: "hybrid"}
WORKLOADS = {
    "ba2k": "BA undirected n=2000 m=5 seed=1",
    "ba1m": "BA undirected n=1048576 m=5 seed=2 (5,242,865 edges)",
    "rmat20": "R-MAT directed scale 20 edge factor 16 (a,b,c,d)=(.57,.19,.19,.05) seed=3",
    "grid2000": "2000x2000 4-neighbour grid, 5% edges deleted, 1000 shortcuts, largest component, seed=4",
}


# the sources each profiled kernel is compiled from (its file and the
# headers it includes)
KERNEL_SOURCES = {
    "k_batch": ["k_batch.hip", "dev_common.hpp", "engine.hpp"],
    "k_swarm": ["k_swarm.hip", "dev_common.hpp", "engine.hpp"],
    "k_plain": ["k_plain.hip", "dev_common.hpp", "engine.hpp"],
}


def kernel_source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1704_01077_amd", "csrc")
    for f in KERNEL_SOURCES.get(kernel, sorted(x for x in os.listdir(csrc) if x.endswith((".hip", ".hpp")))):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_key(kernel: str, k: int, mode: str, width: int, relabel: bool = False) -> str:
    return "%s k=%d %s W=%d%s" % (kernel, k, mode, width, " relabelled" if relabel else "")


def load_traffic(kernel: str, workload: str, k: int, mode: str, width: int, relabel: bool = False):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel, workload, k, mode, batch width and vertex order; null when
    there is none or the kernel's sources changed since the counters were
    taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        rec = d.get(workload, {}).get(traffic_key(kernel, k, mode, width, relabel))
        if not rec or rec.get("source_hash") != kernel_source_hash(kernel):
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def _read_csvs(d: str, suffix: str):
    import csv
    rows = []
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                with open(os.path.join(root, f)) as fh:
                    rows += list(csv.DictReader(fh))
    return rows


def _kernel_durations(d: str):
    """{kernel name: [durations in ns]} from a rocprofv3 --kernel-trace folder
    (CSV output, or the rocpd SQLite database that is its default format)."""
    out = {}
    for r in _read_csvs(d, "kernel_trace.csv"):
        out.setdefault(r["Kernel_Name"], []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    if not out:
        import sqlite3
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith("results.db"):
                    db = sqlite3.connect(os.path.join(root, f))
                    for name, dur in db.execute("select name, duration from kernels"):
                        out.setdefault(name, []).append(int(dur))
                    db.close()
    return out


def stats_table(d: str) -> str:
    """Markdown table of per-kernel durations from a rocprofv3 --kernel-trace folder."""
    rows = sorted(_kernel_durations(d).items(), key=lambda kv: -sum(kv[1]))
    out = ["| kernel | calls | total us | avg us | min us | max us |", "|---|---|---|---|---|---|"]
    for name, ds in rows:
        out.append("| %s | %d | %.1f | %.1f | %.1f | %.1f |" % (
            name.split("(")[0], len(ds), sum(ds) / 1e3, sum(ds) / len(ds) / 1e3, min(ds) / 1e3, max(ds) / 1e3))
    return "\n".join(out)


def traffic_from(fetch_dir: str, write_dir: str, workload: str, kernel: str, last: int, copy_bytes: int,
                 k: int, mode: str, width: int, relabel: bool = False):
    """HBM bytes per launch of `kernel` from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled so that the
    largest copy dispatch (a device copy of copy_bytes) reads and writes
    exactly copy_bytes; the mean over the last `last` dispatches of the
    kernel.  Stores the record in profiles/traffic.json and returns it."""
    def per_dispatch(d, counter):
        vals = {}
        rows = [(r["Dispatch_Id"], r["Kernel_Name"], r["Counter_Name"], r["Counter_Value"])
                for r in _read_csvs(d, "counter_collection.csv")]
        if not rows:   # rocpd SQLite output (the default format of rocprofv3)
            import sqlite3
            for root, _, files in os.walk(d):
                for f in files:
                    if f.endswith("results.db"):
                        db = sqlite3.connect(os.path.join(root, f))
                        rows += db.execute("select dispatch_id, kernel_name, counter_name, value "
                                           "from counters_collection").fetchall()
                        db.close()
        for disp, name, cname, value in rows:
            if cname != counter:
                continue
            key = (int(disp), name)
            vals[key] = vals.get(key, 0.0) + float(value)
        return sorted(vals.items(), key=lambda kv: kv[0][0])
    rec = {"source_hash": kernel_source_hash(kernel), "copy_bytes": copy_bytes, "k": k, "mode": mode,
           "batch_width": width, "relabel": bool(relabel)}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        disp = per_dispatch(d, counter)
        copies = [v for (i, name), v in disp if "copy" in name.lower()]
        mine = [v for (i, name), v in disp if name.split("(")[0].split("<")[0].endswith(kernel)]
        if not copies or not mine:
            raise SystemExit("no %s dispatches of the copy or of %s under %s" % (counter, kernel, d))
        scale = copy_bytes / (max(copies) * 1024.0)
        mine = mine[-last:]
        rec[counter.lower() + "_kib"] = [round(v, 1) for v in mine]
        rec[counter.lower() + "_scale"] = round(scale, 5)
        rec[counter.lower() + "_bytes"] = float(np.mean(mine)) * 1024.0 * scale
    rec["bytes_per_launch"] = int(rec["fetch_size_bytes"] + rec["write_size_bytes"])
    path = os.path.join(ROOT, "profiles", "traffic.json")
    d = json.load(open(path)) if os.path.exists(path) else {}
    d.setdefault(workload, {})[traffic_key(kernel, k, mode, width, relabel)] = rec
    json.dump(d, open(path, "w"), indent=1, sort_keys=True)
    return rec


def cpu_baseline(g, seconds: float):
    """Oracle BFS from a seeded sample of sources, all host cores."""
    import oracle
    rng = np.random.default_rng(1234)
    # calibrate: one source (mostly the oracle's adjacency build, which every
    # call repeats) and 64 sources, then a sample sized for ~seconds
    t0 = time.perf_counter()
    oracle.sums(g.n, g.edges, g.directed, sources=np.zeros(1, np.int32))
    t1 = time.perf_counter() - t0
    probe = rng.integers(0, g.n, size=64).astype(np.int32)
    t0 = time.perf_counter()
    oracle.sums(g.n, g.edges, g.directed, sources=probe)
    per_src = max((time.perf_counter() - t0 - t1) / 63.0, 1e-6)
    count = int(max(64, min(200000, (seconds - t1) / per_src)))
    src = rng.integers(0, g.n, size=count).astype(np.int32)
    t0 = time.perf_counter()
    S, r = oracle.sums(g.n, g.edges, g.directed, sources=src)
    wall = time.perf_counter() - t0
    # arcs scanned by a textbook BFS from s = sum of out-degrees over R(s):
    # every arc when the graph is connected; otherwise estimated as
    # r(s) times the average out-degree
    exact = bool((r == g.n).all())
    arcs = int(g.arcs) * count if exact else int(float(np.sum(r)) * g.arcs / g.n)
    teps = arcs / wall
    full_s = wall / count * g.n
    return {"value": teps / 1e9, "unit": "GTEPS", "cores": oracle.threads(), "kind": "oracle",
            "sample": "textbook BFS from %d seeded random sources of the same graph (%.1f s)%s; "
                      "all-sources extrapolation %.0f s" % (count, wall, "" if exact else
                                                            ", arcs estimated from reach", full_s),
            "wall_s": wall, "sources": count, "all_sources_extrapolated_s": full_s}


def reach_bench(args):
    """Reachability bounds of one workload (Sect. 8.4, Alg. 6), computed once
    per graph on the device: --steps fresh uploads, each timed from the call
    to the arrays in host memory.  All runs must give the same alpha, omega
    and partition.  Prints one JSON line."""
    import torch
    import graphgen
    from paper_1704_01077_amd import tkc
    torch.cuda.init()
    g = graphgen.workload(args.workload)
    ctx = tkc.Context(0)
    out = {"metric": "reachability bounds (SCC + Alg. 6) wall time", "unit": "ms", "higher_is_better": False,
           "config": {"workload": WORKLOADS.get(args.workload, args.workload), "n": g.n}}
    walls, libs, first, same, used = [], [], None, True, None
    for i in range(max(1, args.steps)):
        dg = tkc.Graph.from_graphgen(ctx, g)
        torch.cuda.synchronize()
        t = time.perf_counter()
        a, o, sc = dg.reach()
        walls.append((time.perf_counter() - t) * 1e3)
        used, ms = dg.reach_info()
        libs.append(ms)
        if first is None:
            first = (a, o, sc)
        else:
            same = same and bool(np.array_equal(a, first[0]) and np.array_equal(o, first[1]))
            if sc is not None:
                same = same and len(set(zip(sc.tolist(), first[2].tolist()))) == len(set(sc.tolist()))
        dg.free()
        print("bench: reach run %d %.1f ms" % (i, walls[-1]), file=sys.stderr, flush=True)
    if first[2] is not None:
        out["components"] = int(len(set(first[2].tolist())))
    out["path_used"] = {1: "device, parallel steps", 2: "device, with the one-thread pass"}.get(used, used)
    out["wall_ms_p50"] = round(float(np.percentile(walls, 50)), 3)
    out["library_ms_p50"] = round(float(np.percentile(libs, 50)), 3)
    out["runs"] = len(walls)
    out["same_result"] = same
    out["value"] = out["library_ms_p50"]
    print(json.dumps(out))


def harmonic_bench(args):
    """Top-k harmonic centrality (Sect. 2 with f(d) = 1/d) on --workload:
    --warmup untimed queries, then --steps timed ones.  Prints one JSON line."""
    import torch
    import graphgen
    from paper_1704_01077_amd import tkc
    torch.cuda.init()
    g = graphgen.workload(args.workload)
    ctx = tkc.Context(0)
    dg = tkc.Graph.from_graphgen(ctx, g)
    mode = args.mode
    for _ in range(args.warmup):
        tkc.topk_harmonic(dg, args.k, args.variant, mode)
    torch.cuda.synchronize()
    walls = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        ids, h, st = tkc.topk_harmonic(dg, args.k, args.variant, mode)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
    walls = np.array(walls)
    out = {"metric": "top-k harmonic centrality wall time", "value": round(float(walls.mean()), 4), "unit": "ms",
           "higher_is_better": False, "steps": args.steps, "warmup": args.warmup, "dtype": "f64",
           "config": {"workload": WORKLOADS.get(args.workload, args.workload), "k": args.k,
                      "variant": args.variant, "variant_used": st["variant_used"], "mode": mode,
                      "mode_used": MODE_NAMES.get(st["mode_used"], st["mode_used"])},
           "wall_ms_p50": round(float(np.percentile(walls, 50)), 4),
           "wall_ms_p99": round(float(np.percentile(walls, 99)), 4),
           "m_vis": st["m_vis"],
           "phase_ms": {"reach": st["ms_reach"], "bounds": st["ms_bounds"], "traverse": st["ms_traverse"]},
           "searches": {"started": st["bfs_started"], "exact": st["bfs_exact"], "cut": st["bfs_cut"],
                        "skipped": st["skipped"], "max_level": st["max_level"]},
           "top": [[int(i), float(x)] for i, x in zip(ids[:3], h[:3])]}
    print(json.dumps(out))


def serve_bench(args):
    """Serving mix: a resident pool of seeded graphs (BA, R-MAT, king-move
    lattices; n log-uniform in [1e3, 1e6], average degree 8-16), top-k
    requests with k uniform over {1, 10, 100} on a uniform graph.  First the
    saturation throughput (every request submitted at once), then Poisson
    arrivals at a fraction of it; latency = completion - submission."""
    import threading
    import torch
    import graphgen
    from paper_1704_01077_amd import tkc
    torch.cuda.init()
    t0 = time.perf_counter()
    pool = graphgen.serving_pool(args.serve_graphs)
    print("serve: %d graphs generated in %.1f s" % (len(pool), time.perf_counter() - t0), file=sys.stderr, flush=True)
    ctx = tkc.Context(0)
    dgs = [tkc.Graph.from_graphgen(ctx, g) for g in pool]
    srv = tkc.Server(ctx, int(args.serve_budget_gb * (1 << 30)), args.serve_slots)
    gids = [srv.add(d) for d in dgs]
    if args.serve_pack > 0:
        srv.enable_packing(args.serve_pack)
        print("serve: packing on for graphs of at most %d vertices: %s" % (args.serve_pack, srv.info()),
              file=sys.stderr, flush=True)
    rng = np.random.default_rng(args.serve_seed)
    solo_ans = {}      # (graph, k) -> (ids, S) of the request served alone
    mismatch = [0]

    def run(reqs, gaps=None):
        """Submit (graph, k) requests (with arrival gaps in seconds) and
        collect them; returns (wall seconds, latencies in ms)."""
        tickets = [None] * len(reqs)
        lat = [0.0] * len(reqs)

        def submitter():
            t_next = time.perf_counter()
            for i, (gi, k) in enumerate(reqs):
                if gaps is not None:
                    t_next += gaps[i]
                    d = t_next - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                tickets[i] = srv.submit(gids[gi], k, "auto")
        th = threading.Thread(target=submitter)
        start = time.perf_counter()
        th.start()
        for i, (gi, k) in enumerate(reqs):
            while tickets[i] is None:
                time.sleep(0.0002)
            ids, S, r, f, ms = srv.result(tickets[i], k)
            lat[i] = ms
            key = (gi, k)
            if key in solo_ans:
                if not (np.array_equal(solo_ans[key][0], ids) and np.array_equal(solo_ans[key][1], S)):
                    mismatch[0] += 1
            else:
                solo_ans[key] = (ids.copy(), S.copy())   # the warm-up: one request at a time
            if len(reqs) > 1 and (i + 1) % 500 == 0:
                print("serve: %d/%d requests done (%.1f s)" % (i + 1, len(reqs), time.perf_counter() - start),
                      file=sys.stderr, flush=True)
        th.join()
        return time.perf_counter() - start, np.array(lat)

    # warm-up: one request per graph and k, one at a time (fills the per-graph
    # preprocessing caches; gives the solo time of every request kind)
    solo = {}
    for gi in range(len(pool)):
        for k in (1, 10, 100):
            w, l = run([(gi, k)])
            solo[(gi, k)] = l[0]
        if gi % 8 == 7:
            print("serve: warm-up %d/%d graphs" % (gi + 1, len(pool)), file=sys.stderr, flush=True)
    print("serve: warm-up done, solo latency p50 %.2f ms max %.1f ms (graph %s)" % (
        np.percentile(list(solo.values()), 50), max(solo.values()),
        pool[max(solo, key=solo.get)[0]].name), file=sys.stderr, flush=True)

    def draw(count):
        return [(int(rng.integers(len(pool))), int(rng.choice([1, 10, 100]))) for _ in range(count)]

    sat_reqs = draw(args.serve_sat)
    wall, lat_sat = run(sat_reqs)
    lam_sat = len(sat_reqs) / wall
    print("serve: saturation %.1f req/s" % lam_sat, file=sys.stderr, flush=True)
    lam = args.serve_load * lam_sat
    reqs = draw(args.serve_requests)
    gaps = rng.exponential(1.0 / lam, size=len(reqs))
    wall, lat = run(reqs, gaps)
    solo_sum = sum(solo[q] for q in reqs)
    out = {
        "metric": "serving mix: throughput and latency (continuous batching)",
        "value": round(len(reqs) / wall, 3), "unit": "requests/s", "higher_is_better": True,
        "n_gpus": 1, "data": "synthetic",
        "config": {"workload": "%d seeded graphs (BA, R-MAT, king lattices), n log-uniform 1e3-1e6, "
                               "k uniform in {1,10,100}, Poisson arrivals" % len(pool),
                   "requests": len(reqs), "slots": args.serve_slots, "hbm_budget_gb": args.serve_budget_gb,
                   "arrival_rate": round(lam, 3), "load": args.serve_load,
                   "resident_arcs": int(sum(g.arcs for g in pool))},
        "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
        "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
        "latency_ms_max": round(float(lat.max()), 3),
        "saturation_req_s": round(lam_sat, 3),
        "saturation_latency_ms_p50": round(float(np.percentile(lat_sat, 50)), 3),
        "solo_sum_s": round(solo_sum / 1e3, 3), "wall_s": round(wall, 3),
        "served_equal_solo": mismatch[0] == 0,
        "mismatches": mismatch[0],
        "checked": "every served answer (saturation and timed runs) against the same (graph, k) served alone "
                   "in the warm-up",
        "server": srv.info(),
        "packing_max_vertices": args.serve_pack,
    }
    print(json.dumps(out), flush=True)
    srv.close()
    for d in dgs:
        d.free()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--variant", default="auto")
    ap.add_argument("--mode", default="hybrid",
                    help="plain | batched | hybrid | auto (autotune this graph and query first)")
    ap.add_argument("--autotune-ms", type=float, default=8000.0,
                    help="time budget of the autotuner that runs before the warm-up when --mode auto")
    ap.add_argument("--workload", default="ba1m")
    ap.add_argument("--cpu-seconds", type=float, default=40.0,
                    help="budget of the CPU oracle sample (its calibration overestimates, so it runs less)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--compare", default="plain,batched,hybrid",
                    help="modes timed once each (default knobs) beside the main run")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison runs")
    ap.add_argument("--tune", nargs="*", default=[],
                    help="context knobs for the main run, e.g. batch_width=128 blocks_per_cu=4")
    ap.add_argument("--plain-cap", type=int, default=20000,
                    help="search cap of every plain-mode comparison (never an uncapped plain run)")
    ap.add_argument("--configs", default="C1,C3,C4", help="other workloads measured into the same line")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one device copy of this size (for counter calibration)")
    ap.add_argument("--serve", action="store_true", help="run the serving-mix benchmark instead")
    ap.add_argument("--harmonic", action="store_true",
                    help="time top-k harmonic centrality on --workload instead")
    ap.add_argument("--reach-only", action="store_true",
                    help="time the reachability bounds of --workload (device and host paths) instead")
    ap.add_argument("--serve-graphs", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-pack", type=int, default=1 << 17,
                    help="pack graphs of at most this many vertices into shared launches (0: off)")
    ap.add_argument("--serve-sat", type=int, default=400, help="requests of the saturation run")
    ap.add_argument("--serve-load", type=float, default=0.7, help="arrival rate / saturation throughput")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=float, default=32.0)
    ap.add_argument("--serve-seed", type=int, default=7)
    ap.add_argument("--stats-from", default="",
                    help="print the kernel table of a rocprofv3 --stats folder and exit")
    ap.add_argument("--traffic-from", default="",
                    help="FETCH_DIR,WRITE_DIR of two rocprofv3 --pmc runs: store bytes per launch and exit")
    ap.add_argument("--traffic-kernel", default="k_batch")
    ap.add_argument("--traffic-last", type=int, default=3)
    ap.add_argument("--traffic-width", type=int, default=64, help="batch width of the profiled runs")
    ap.add_argument("--relabel", action="store_true",
                    help="upload the main line's graph with TKC_RELABEL (vertices by decreasing out-degree)")
    args = ap.parse_args()
    if args.stats_from:
        print(stats_table(args.stats_from))
        return
    if args.traffic_from:
        fd, wd = args.traffic_from.split(",")
        rec = traffic_from(fd, wd, args.workload, args.traffic_kernel, args.traffic_last,
                           args.calib_copy_mb << 20, args.k, args.mode, args.traffic_width, args.relabel)
        print(json.dumps(rec, indent=1))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the searches would shard by candidate ranges with a top-k merge)",
              file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_bench(args)
        return
    if args.reach_only:
        reach_bench(args)
        return
    if args.harmonic:
        harmonic_bench(args)
        return

    import torch
    import graphgen
    from paper_1704_01077_amd import tkc
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    print("bench: generating %s" % args.workload, file=sys.stderr, flush=True)
    g = graphgen.workload(args.workload)
    ctx = tkc.Context(0)
    dg = tkc.Graph.from_graphgen(ctx, g, relabel=args.relabel)
    torch.cuda.synchronize()

    if args.calib_copy_mb:
        a = torch.empty(args.calib_copy_mb << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    tuning = None
    if args.mode == "auto" and args.autotune_ms > 0:
        print("bench: autotune (budget %.0f ms)" % args.autotune_ms, file=sys.stderr, flush=True)
        tuning, tuned_ms = dg.autotune(args.k, args.variant, args.autotune_ms)
        print("bench: autotuned %s (%.3f ms)" % (tuning, tuned_ms), file=sys.stderr, flush=True)
    knobs = dict((kv.split("=")[0], int(kv.split("=")[1])) for kv in args.tune) or None
    if knobs:
        tuning = knobs
    m = measure(tkc, torch, ctx, g, dg, args.workload, args.k, args.variant, args.mode, args.steps, args.warmup,
                knobs, args.relabel)
    st = m.pop("_stats")

    compare = {}
    if not args.no_compare:
        for mode in [x for x in args.compare.split(",") if x]:
            print("bench: compare %s" % mode, file=sys.stderr, flush=True)
            compare[mode] = compare_once(tkc, torch, dg, args.k, args.variant, mode, m["_ids"], m["_S"],
                                         args.plain_cap)
    plain = compare.get("plain")
    useful = None
    if plain and plain.get("finished"):
        # the work a one-source-at-a-time engine needs for the same answer
        useful = round(plain["m_vis"] / (m["ms_per_step"] * 1e-3) / 1e9, 4)

    configs = {}
    if not args.no_configs:
        for cname in [x for x in args.configs.split(",") if x]:
            print("bench: config %s" % cname, file=sys.stderr, flush=True)
            configs[cname] = run_config(tkc, torch, graphgen, ctx, cname, args)

    cpu = None
    if not args.no_cpu:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(g, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": m["gteps"],
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "%s, top-k k=%d" % (WORKLOADS.get(args.workload, args.workload), args.k),
                   "k": args.k, "variant": args.variant, "variant_used": st["variant_used"],
                   "mode": args.mode, "mode_used": MODE_NAMES.get(st["mode_used"], st["mode_used"]),
                   "batch_width": st["batch_width"], "tuning": tuning, "relabel": bool(args.relabel), "n": g.n,
                   "arcs": int(g.arcs)},
        "wall_ms_p50": m["wall_ms_p50"],
        "wall_ms_p99": m["wall_ms_p99"],
        "m_vis": m["m_vis"],
        "useful_gteps": useful,
        "useful_note": "m_vis of the plain one-source-at-a-time engine on the same query over this run's "
                       "ms_per_step; value counts every lane's work, including searches the plain engine "
                       "would cut or skip",
        "improvement_factor": m["improvement_factor"],
        "phase_ms": m["phase_ms"],
        "searches": m["searches"],
        "roofline": m["roofline"],
        "compare": compare,
        "configs": configs,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    dg.free()
    ctx.close()


def measure(tkc, torch, ctx, g, dg, wname, k, variant, mode, steps, warmup, tune=None, relabel=False):
    """warmup untimed queries, then `steps` timed ones (each between device
    synchronisations); GTEPS, percentiles, phases and the dominant kernel's
    roofline."""
    keep = ctx.tuning()
    if tune:
        ctx.tune(**tune)
    try:
        for _ in range(warmup):
            tkc.topk_closeness(dg, k, variant, mode)
        torch.cuda.synchronize()
        walls, stats = [], []
        t_all0 = time.perf_counter()
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ids, S, r, f, st = tkc.topk_closeness(dg, k, variant, mode)
            torch.cuda.synchronize()
            walls.append((time.perf_counter() - t0) * 1e3)
            stats.append(st)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t_all0
    finally:
        ctx.tune(**keep)
    print("bench: %s timed %d steps" % (wname, steps), file=sys.stderr, flush=True)
    walls = np.array(walls)
    ms_per_step = t_all * 1e3 / steps
    st = stats[-1]
    mvis = st["m_vis"]
    # dominant kernel: library HIP events around its launches, over the timed steps
    kern_ms = float(np.mean([x["ms_kernel_main"] for x in stats]))
    launches = st["main_launches"]
    bytes_main = st["bytes_main"]
    per_launch_ms = kern_ms / max(1, launches)
    achieved = (bytes_main / max(1, launches)) / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
    kname = KERNEL_NAMES.get(st["main_kernel"], "?")
    mode_used = MODE_NAMES.get(st["mode_used"], "?")
    traffic = load_traffic(kname, wname, k, mode_used, st["batch_width"], relabel)
    undirected = not g.directed
    mn = (2 if undirected else 1) * (g.arcs // (2 if undirected else 1)) * g.n
    return {
        "_stats": st, "_ids": ids, "_S": S,
        "gteps": round(mvis / (ms_per_step * 1e-3) / 1e9, 4),
        "ms_per_step": round(ms_per_step, 4),
        "wall_ms_p50": round(float(np.percentile(walls, 50)), 4),
        "wall_ms_p99": round(float(np.percentile(walls, 99)), 4),
        "m_vis": int(mvis),
        "improvement_factor": mn / mvis if mvis else None,
        "phase_ms": {"reach": st["ms_reach"], "bounds": st["ms_bounds"], "traverse": st["ms_traverse"]},
        "searches": {"started": st["bfs_started"], "exact": st["bfs_exact"], "cut": st["bfs_cut"],
                     "skipped": st["skipped"], "deferred": st["deferred"], "max_level": st["max_level"]},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                     "launches_per_step": launches, "kernel_ms_per_step": round(kern_ms, 4),
                     "bytes_per_step": int(bytes_main)},
    }


def compare_once(tkc, torch, dg, k, variant, mode, ids, S, plain_cap):
    """One query in `mode` with the default knobs.  Plain mode always runs
    under a search cap: if it would need more searches it stops there and
    reports the work and time so far (finished = false), never an answer."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if mode == "plain":
        done, res, st = tkc.topk_closeness_budget(dg, k, variant, plain_cap)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        out = {"wall_ms": round(wall, 3), "m_vis": int(st["m_vis"]), "searches": int(st["bfs_started"]),
               "finished": bool(done), "search_cap": int(plain_cap)}
        if done:
            out["same_result"] = bool(np.array_equal(res[0], ids) and np.array_equal(res[1], S))
        else:
            out["note"] = ("stopped at the search cap: wall_ms and m_vis cover %d searches only, and the full "
                           "plain query takes longer" % st["bfs_started"])
        return out
    ids2, S2, r2, f2, st2 = tkc.topk_closeness(dg, k, variant, mode)
    torch.cuda.synchronize()
    return {"wall_ms": round((time.perf_counter() - t0) * 1e3, 3), "m_vis": int(st2["m_vis"]),
            "same_result": bool(np.array_equal(ids2, ids) and np.array_equal(S2, S))}


# the other workloads of the benchmark, each with its knobs fixed here: the
# BA n = 2,000 query (plain engine against batched), R-MAT scale 20 in its
# autotuned configuration (batched, W = 256, four workgroups per CU), the
# 2000^2 grid with the level-based variant
CONFIGS = {
    "C1": {"workload": "ba2k", "k": [1, 10], "variant": "auto", "mode": "plain", "steps": 30, "warmup": 3,
           "tune": None, "compare": ["batched", "hybrid"], "plain_cap": 20000},
    # C3's graph is uploaded with TKC_RELABEL (vertices by decreasing
    # out-degree): the skewed R-MAT degrees then pack the hubs' words together
    "C3": {"workload": "rmat20", "k": [10], "variant": "auto", "mode": "batched", "steps": 10, "warmup": 2,
           "tune": {"batch_width": 256, "blocks_per_cu": 4}, "compare": ["hybrid", "plain"], "plain_cap": 20000,
           "relabel": True},
    # a plain search on the grid is a whole-GPU search of ~430 levels (~8 ms):
    # the comparison stops after 300 of them
    "C4": {"workload": "grid2000", "k": [10], "variant": "nbbound", "mode": "batched", "steps": 2, "warmup": 1,
           "tune": {"batch_width": 128}, "compare": ["plain"], "plain_cap": 300},
}


def run_config(tkc, torch, graphgen, ctx, cname, args):
    cfg = CONFIGS[cname]
    g = graphgen.workload(cfg["workload"])
    relabel = bool(cfg.get("relabel"))
    dg = tkc.Graph.from_graphgen(ctx, g, relabel=relabel)
    out = {"workload": WORKLOADS.get(cfg["workload"], cfg["workload"]), "variant": cfg["variant"],
           "mode": cfg["mode"], "tuning": cfg["tune"], "relabel": relabel, "n": g.n, "arcs": int(g.arcs),
           "runs": {}}
    try:
        for k in cfg["k"]:
            m = measure(tkc, torch, ctx, g, dg, cfg["workload"], k, cfg["variant"], cfg["mode"], cfg["steps"],
                        cfg["warmup"], cfg["tune"], relabel)
            st = m.pop("_stats")
            ids, S = m.pop("_ids"), m.pop("_S")
            m["variant_used"] = st["variant_used"]
            m["mode_used"] = MODE_NAMES.get(st["mode_used"], st["mode_used"])
            m["compare"] = {}
            for mode in cfg["compare"]:
                print("bench: %s compare %s" % (cname, mode), file=sys.stderr, flush=True)
                m["compare"][mode] = compare_once(tkc, torch, dg, k, cfg["variant"], mode, ids, S,
                                                  min(args.plain_cap, cfg["plain_cap"]))
            plain = m["compare"].get("plain")
            m["useful_gteps"] = (round(plain["m_vis"] / (m["ms_per_step"] * 1e-3) / 1e9, 4)
                                 if plain and plain.get("finished") else None)
            out["runs"]["k=%d" % k] = m
        if g.directed:
            used, ms = dg.reach_info()
            out["reach_ms_once_per_graph"] = round(ms, 3)
            out["reach_note"] = ("directed reachability (SCCs + Alg. 6) runs once per graph and is cached; "
                                 "the timed queries reuse it")
    finally:
        dg.free()
    return out


if __name__ == "__main__":
    main()
