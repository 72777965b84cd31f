"""Benchmark: temporal edges traversed per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--mode batch|single] [--no-cpu] [--serve]

A step answers every query of the workload once.  By default that is the
largest workload: the bursty communication-style multigraph (R-MAT scale-22
pair structure, about 1.007e9 edges, bursty Pareto departure times, lambda
in [1, 100]) with its 32 earliest-arrival queries (t_alpha in the first half
of the span, t_omega = max), one query per call.  The graph and the queries
are synthetic and resident in HBM before timing starts.

value = sum over queries of the temporal edges each traverses (edges whose
tail is reached, departing no earlier than the tail's earliest arrival and
t_alpha, arriving by t_omega) times steps, divided by the wall time of the
timed steps.  The count per query comes from the CPU oracle's own result
(untimed) and must equal the GPU's count of the same query; with --no-cpu
(profiling runs) the GPU's count is used.

Printed as one JSON line.  The timed steps run without per-launch events;
the same steps then run again with every launch bracketed by HIP events on
its own stream, which give the dominant kernel's average launch duration
for the roofline figures (that pass's step time is reported beside them).
The CPU oracle is timed on a bounded sample of the same workload on this
host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bursty22-1b")
    ap.add_argument("--mode", choices=["batch", "single"], default=None,
                    help="default: the workload's own form (one query per call, or the batch)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--serve", action="store_true", help="also run the serving sweep")
    ap.add_argument("--extras", action="store_true", default=True,
                    help="also time the batch against one query per call, LD/F, paths, BFS (the default)")
    ap.add_argument("--no-extras", dest="extras", action="store_false", help="skip those timings")
    ap.add_argument("--tune", action="store_true", help="autotune before timing")
    ap.add_argument("--layout", type=int, choices=[0, 1, 2, 3], default=None,
                    help="batch layout to time (3: the sweep form); default: the library's")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_2401_02563_amd as K
    from workloads import CONFIGS, make_graph, make_queries

    torch.cuda.set_device(0)
    cfg = CONFIGS[args.workload]
    if args.mode is None:
        args.mode = cfg.get("bench_mode", "batch")
    t0 = time.time()
    g = make_graph(args.workload)
    srcs, ta, tw = make_queries(args.workload, g)
    log(f"generated {args.workload}: n={g.n} m={g.m} q={len(srcs)} in {time.time() - t0:.1f}s")
    dev = [K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)]
    torch.cuda.synchronize()
    tb = time.perf_counter()
    G = K.kairos_graph_build(*dev, g.n)
    build_s = time.perf_counter() - tb
    del dev
    log(f"index built in {build_s * 1e3:.1f} ms")
    q = len(srcs)
    out = torch.empty(q * g.n, dtype=torch.int32, device="cuda")
    one = torch.empty(g.n, dtype=torch.int32, device="cuda")

    tune_note = None
    if args.layout is not None:
        K.kairos_set_tuning(G, batch_layout=args.layout)
    if args.tune:
        # held-out queries of the workload's recipe (another seed), in the
        # timed work's shape: a batch as large as the timed one, or a few
        # queries answered one per call
        k = q if args.mode == "batch" else min(q, 4)
        form = K.KAIROS_TUNE_BATCH if args.mode == "batch" else K.KAIROS_TUNE_SINGLE
        hs, ha, hw = make_queries(args.workload, g, count=k, held_out=True)
        cache = os.environ.get("KAIROS_TUNING_CACHE")
        t0 = time.perf_counter()
        best = K.kairos_autotune_form(G, form, hs, ha, hw)
        tune_s = time.perf_counter() - t0
        tune_note = {"sample": f"{k} held-out queries of the workload's recipe (another seed), "
                               + ("as one batch" if args.mode == "batch" else "one per call"),
                     "seconds": round(tune_s, 2), "cache": cache}
        log(f"autotuned on {k} held-out queries in {tune_s:.1f} s: {best}")

    def step():
        if args.mode == "batch":
            K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
        else:
            for i in range(q):
                K.kairos_earliest_arrival(G, int(srcs[i]), int(ta[i]), int(tw[i]), out[i * g.n:(i + 1) * g.n])

    # traversed edges per query, from the GPU result (not timed); the
    # oracle's own count replaces it below when the CPU leg runs
    step()
    torch.cuda.synchronize()
    etrav = [K.kairos_traversed_edges(G, int(ta[i]), int(tw[i]), out[i * g.n:(i + 1) * g.n]) for i in range(q)]
    etrav_total = int(sum(etrav))
    log(f"traversed edges per step (GPU count): {etrav_total}")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed steps: `value` (no per-launch events, which cost host time on
    # short launches)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    ms_per_step = elapsed / args.steps * 1e3
    value = etrav_total * args.steps / elapsed
    # the same steps again with every launch bracketed by HIP events on its
    # own stream and device work counters on: the roofline figures
    K.kairos_profile_enable(G, True)
    K.kairos_profile_read(G)  # reset
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof_elapsed = time.perf_counter() - t2
    prof = K.kairos_profile_read(G)
    K.kairos_profile_enable(G, False)

    tuning = K.kairos_get_tuning(G)
    if os.environ.get("KAIROS_CALIBRATION_COPY"):
        # a plain 256 MiB copy: the counter-calibration kernel of bench_pmc.py
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    extra = {}
    if args.extras:
        extra.update(time_extras(K, torch, G, g, srcs, ta, tw, out, one, etrav))
    if args.serve:
        extra["serving"] = serve_sweep(K, torch, G, g, args.workload)

    cpu = None
    numerator = {"source": "gpu count (kairos_traversed_edges)", "queries": q}
    if not args.no_cpu:
        del out, one
        G.free()  # the oracle's sorted copy needs host memory, not the GPU; free device state first
        G = None
        cpu, oracle_etrav = cpu_baseline(g, srcs, ta, tw, args.cpu_seconds)
        bad = [i for i in range(q) if oracle_etrav[i] != etrav[i]]
        if bad:
            print(json.dumps({"error": "traversed-edge count differs between the GPU and the oracle",
                              "queries": bad[:8]}), flush=True)
            sys.exit(1)
        etrav_total = int(sum(oracle_etrav))
        value = etrav_total * args.steps / elapsed
        numerator = {"source": "oracle (C scan result, untimed), equal to the gpu count on every query",
                     "queries": q}
    roofline = roofline_from_profile(prof, args.mode, etrav_total * args.steps, args.workload, tuning)
    roofline["profiled_ms_per_step"] = round(prof_elapsed / args.steps * 1e3, 3)
    roofline["path"] = path_bytes(prof, etrav_total * args.steps, g.n * q * args.steps, elapsed)

    line = {
        "metric": "temporal edges traversed/s", "value": value, "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "queries_per_step": q,
                   "mode": args.mode, "window": cfg["window"]},
        "queries_per_s": q * args.steps / elapsed,
        "build_ms": round(build_s * 1e3, 2), "build_edges_per_s": g.m / build_s,
        "traversed_edges_per_step": etrav_total, "numerator": numerator,
        "rounds_per_step": prof["rounds"] / args.steps,
        "roofline": roofline, "cpu_baseline": cpu,
        "tuning": {"source": "autotuner" if args.tune else ("layout given" if args.layout is not None else "defaults"), **({"tuned": tune_note} if tune_note else {}),
                   **{k: tuning[k] for k in ("block", "batch_layout", "batch_persistent", "single_persistent",
                                             "rounds_per_sync", "tail_limit", "split", "chunk", "pull_alpha",
                                             "pull_beta", "dense_frontier", "arrival_filter", "run_dedupe",
                                             "sweep_group", "binned")}},
        **extra,
    }
    print(json.dumps(line), flush=True)
    if G is not None:
        G.free()


# Algorithmic bytes per unit of work (what the method must move, not what the
# caches do), for the per-(query, vertex) kernels -- single queries (push,
# chunk, tail, persist), the query-major batch and the lane-dense batch
# (hpush, hchunk, hpersist):
#   8 B per traversed edge (the record's head and arrival),
#   16 B per frontier entry expanded (two offsets, the tail's arrival, its
#        claim word),
#   4 B per successful relaxation (the new arrival),
#   8 B per (query, vertex) for the whole query (arrival init + result),
#        charged to the path figure, not to a traversal kernel.
# A kernel's traversed edges are the step's traversed edges (counted from
# the result) in proportion to the edges that kernel scanned.  The
# vertex-major batch (bpush, bchunk) reads each edge record once for the 64
# queries of a group: 8 B per edge record + 4 B per (edge, query) check of
# the head's arrival row + 12 B per (vertex, query) claim + 4 B per
# successful relaxation.
B_EDGE, B_ITEM, B_RELAX, B_VERTEX = 8, 16, 4, 8


def path_bytes(prof, traversed, vertex_queries, seconds):
    """Whole-step algorithmic bytes (all kernels) over the timed step time."""
    b = B_EDGE * traversed + B_ITEM * (prof["items"] + prof.get("tail_items", 0) + prof.get("binned_items", 0)) \
        + B_RELAX * prof["relaxations"] + B_VERTEX * vertex_queries
    gbs = b / seconds / 1e9 if seconds > 0 else 0.0
    return {"bytes": int(b), "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}


def kernel_names(mode, tuning):
    """Kernel names of the push, chunk and tail classes for this run."""
    if mode == "single":
        push = "persist_kernel" if tuning.get("single_persistent") else "push_kernel"
        # a binned round is timed as one unit: claim, scans, count, scatter, apply
        return {"push": push, "chunk": "chunk_kernel", "tail": "tail_kernel", "binned": "binned_round"}
    layout = tuning.get("batch_layout", 2)
    if layout == 3:
        # the sweep form: one cooperative launch per 64-query group
        return {"push": "sweep_kernel"}
    if layout == 2 and tuning.get("batch_persistent"):
        return {"push": "hpersist_kernel", "chunk": "hchunk_kernel"}
    return {0: {"push": "bpush_kernel", "chunk": "bchunk_kernel"},
            1: {"push": "push_kernel", "chunk": "chunk_kernel"},
            2: {"push": "hpush_kernel", "chunk": "hchunk_kernel"}}[layout]


def roofline_from_profile(prof, mode, pairs, workload, tuning):
    names = kernel_names(mode, tuning)
    classes = [c for c in ("push", "chunk", "tail", "binned") if c in names and prof.get(f"launches_{c}", 0) > 0]
    edges = {"push": prof["edges_scanned"], "chunk": prof["chunk_edges"], "tail": prof.get("tail_edges", 0),
             "binned": prof.get("binned_edges", 0)}
    items = {"push": prof["items"], "chunk": 0, "tail": prof.get("tail_items", 0), "binned": prof.get("binned_items", 0)}
    if names["push"] == "sweep_kernel":
        # the sweep relaxes every edge of the groups' windows; it keeps no
        # per-query counts, so its share is the whole traversal
        edges["push"], items["push"] = max(1, pairs), 0
    if names["push"] in ("hpersist_kernel", "persist_kernel") and prof.get("launches_chunk", 0) == 0:
        # one launch runs both phases: its edges are the push and chunk counts
        edges["push"] += edges["chunk"]
        edges["chunk"] = 0
    tot_edges = max(1, sum(edges[c] for c in classes))
    vertex_major = mode == "batch" and tuning.get("batch_layout") == 0
    res = {}
    for c in classes:
        share = edges[c] / tot_edges
        if vertex_major:
            b = 8 * edges[c] + 4 * pairs * share + 12 * items[c] + 4 * prof["relaxations"] * share
        else:
            b = B_EDGE * pairs * share + B_ITEM * items[c] + B_RELAX * prof["relaxations"] * share
        res[c] = {"bytes": b, "launches": max(1, prof[f"launches_{c}"]), "ms": prof[f"ms_{c}"]}
    kern = max(res, key=lambda c: res[c]["ms"])
    r = res[kern]
    avg_ms = r["ms"] / r["launches"]
    per_launch = r["bytes"] / r["launches"]
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    kname = names[kern]
    traffic = traffic_for(kname, workload, mode)
    # counted bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE per launch) over this
    # run's launch duration: what the kernel moves beyond L2, beside the
    # algorithmic figure above
    counted = traffic / (avg_ms * 1e-3) / 1e9 if traffic and avg_ms > 0 else None
    return {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_GBps": round(counted, 1) if counted else None,
            "traffic_frac": round(counted / HBM_PEAK_GBS, 4) if counted else None,
            "avg_launch_us": round(avg_ms * 1e3, 2), "launches": r["launches"],
            "alg_bytes_per_launch": int(per_launch),
            "per_kernel": {names[c]: {"ms": round(v["ms"], 3), "launches": v["launches"],
                                      "alg_GBps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)}
                           for c, v in res.items()}}


def traffic_for(kname, workload, mode):
    """HBM bytes per launch of `kname` from a stored rocprofv3 counter summary,
    or None when there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{mode}.json")
    if not os.path.exists(path):
        return None
    try:
        import bench_pmc
        doc = json.load(open(path))
        if doc.get("kernel_sources_sha") != bench_pmc.kernel_source_hash():
            return None
        k = doc["kernels"].get(kname)
        if not k or k.get("fetch_bytes_per_launch") is None or k.get("write_bytes_per_launch") is None:
            return None
        return int(k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"])
    except Exception:
        return None


def time_extras(K, torch, G, g, srcs, ta, tw, out, one, etrav):
    res = {}
    q = len(srcs)
    # one untimed call of each form first: it allocates that form's state
    K.kairos_earliest_arrival(G, int(srcs[0]), int(ta[0]), int(tw[0]), one)
    K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(q):
        K.kairos_earliest_arrival(G, int(srcs[i]), int(ta[i]), int(tw[i]), one)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    res["single_ea"] = {"queries_per_s": q / dt, "edges_per_s": sum(etrav) / dt, "ms_per_query": dt / q * 1e3}
    reps = 3
    t = time.perf_counter()
    for _ in range(reps):
        K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    res["batch_ea"] = {"queries_per_s": q / dt, "edges_per_s": sum(etrav) / dt, "ms_per_batch": dt * 1e3}
    k = min(4, q)
    for kind, fn in (("latest_departure", K.kairos_latest_departure), ("fastest", K.kairos_fastest)):
        fn(G, int(srcs[0]), int(ta[0]), int(tw[0]), one)  # first call allocates the sweep's scratch
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(k):
            fn(G, int(srcs[i]), int(ta[i]), int(tw[i]), one)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        res[kind] = {"ms_per_query": dt / k * 1e3, "queries": k}
    # earliest-arrival paths (predecessor pass), temporal BFS (level-
    # synchronous rounds) and single-target latest departure (reversed index,
    # built by the untimed first call), one query per call
    k = min(8, q)
    pt = torch.empty_like(one)
    pd = torch.empty_like(one)
    for kind, call in (("earliest_arrival_path",
                        lambda i: K.kairos_earliest_arrival_path(G, int(srcs[i]), int(ta[i]), int(tw[i]), one, pt, pd)),
                       ("temporal_bfs", lambda i: K.kairos_temporal_bfs(G, int(srcs[i]), int(ta[i]), int(tw[i]), one)),
                       ("latest_departure_to",
                        lambda i: K.kairos_latest_departure_to(G, int(srcs[i]), int(ta[i]), int(tw[i]), one))):
        call(0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(k):
            call(i)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        res[kind] = {"ms_per_query": dt / k * 1e3, "queries": k}
        if kind != "latest_departure_to":  # same traversed edges as earliest arrival
            res[kind]["edges_per_s"] = sum(etrav[:k]) / dt
    # shortest duration: the untimed first call builds the out-to-in edge map
    # and the per-in-edge labels
    k = min(4, q)
    K.kairos_shortest_duration(G, int(srcs[0]), int(ta[0]), int(tw[0]), one)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(k):
        K.kairos_shortest_duration(G, int(srcs[i]), int(ta[i]), int(tw[i]), one)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    # the same queries again with work counters on (untimed): out-edges
    # relaxed and vertices expanded
    K.kairos_profile_enable(G, True)
    K.kairos_profile_read(G)  # reset
    for i in range(k):
        K.kairos_shortest_duration(G, int(srcs[i]), int(ta[i]), int(tw[i]), one)
    p = K.kairos_profile_read(G)
    K.kairos_profile_enable(G, False)
    res["shortest_duration"] = {"ms_per_query": dt / k * 1e3, "queries": k,
                                "relaxed_edges_per_query": p["edges_scanned"] / k,
                                "expanded_vertices_per_query": p["items"] / k,
                                "rounds_per_query": p["rounds"] / k,
                                "relaxed_edges_per_s": p["edges_scanned"] / dt}
    return res


def serve_sweep(K, torch, G, g, name, rates=(1000, 2000, 5000, 10000, 20000, 50000), count=20000,
                warmup=1000, rounds_per_check=0, fifo=True, pool=4096, max_slots=256):
    """Open-loop Poisson arrivals: continuous-batching server versus a FIFO
    server answering one query at a time, on the same trace of `count`
    queries per rate.  The server first answers `warmup` other queries
    (closed loop, growing its slot pool).  Latency runs from the query's
    arrival time to its completion; queries wait on the client side while
    all `pool` output buffers are in flight.  A sample of the served results
    (every 500th query and the first of each kind) is copied out on
    completion and compared, after the timed run, with the same queries
    answered alone; a difference fails the run."""
    from workloads import make_queries, poisson_arrivals
    from workloads.configs import make_kinds
    total = count + warmup
    srcs, ta, tw = make_queries("serve-rmat20", g, total)
    kinds = make_kinds("serve-rmat20", total)
    pool = min(pool, total)
    outs = torch.empty((pool, g.n), dtype=torch.int32, device="cuda")
    fns = (K.kairos_earliest_arrival, K.kairos_latest_departure, K.kairos_fastest)
    for k in range(3):  # first call of each kind allocates its state
        fns[k](G, int(srcs[0]), int(ta[0]), int(tw[0]), outs[0])
    torch.cuda.synchronize()
    res = []
    for rate in rates:
        srv = K.kairos_server_create(G, max_slots=max_slots, queue_capacity=1 << 20,
                                     rounds_per_check=rounds_per_check)
        for j in range(warmup):
            K.kairos_server_submit(srv, int(kinds[j]), int(srcs[j]), int(ta[j]), int(tw[j]), outs[j % pool])
            if j % pool == pool - 1:
                _drain(K, srv, pool)
        _drain(K, srv, warmup % pool)
        arr = poisson_arrivals(rate, count, 105 + rate)
        free = list(range(pool))
        inflight = {}
        sample_at = set(range(0, count, 500))
        for kd in range(3):
            hits = np.nonzero(kinds[warmup:] == kd)[0]
            if len(hits):
                sample_at.add(int(hits[0]))
        samples = []
        lat = np.empty(count)
        done = 0
        i = 0
        start = time.monotonic_ns()
        last = start
        while done < count:
            now = (time.monotonic_ns() - start) * 1e-9
            while i < count and arr[i] <= now and free:
                b = free.pop()
                q = warmup + i
                tk = K.kairos_server_submit(srv, int(kinds[q]), int(srcs[q]), int(ta[q]), int(tw[q]), outs[b])
                inflight[tk] = (b, arr[i], i)
                i += 1
            for c in K.kairos_server_poll(srv, 4096):
                b, a, idx = inflight.pop(c["ticket"])
                if idx in sample_at:
                    samples.append((warmup + idx, outs[b].clone()))
                free.append(b)
                lat[done] = (c["t_done_ns"] - start) * 1e-9 - a
                last = max(last, c["t_done_ns"])
                done += 1
            time.sleep(0.0001)
        wall = (last - start) * 1e-9
        K.kairos_server_free(srv)
        # FIFO one-at-a-time on the same trace (virtual clock)
        fifo_lat = []
        clock = 0.0
        n_fifo = count if fifo else 0
        for j in range(n_fifo):
            q = warmup + j
            clock = max(clock, arr[j])
            t = time.perf_counter()
            fns[kinds[q]](G, int(srcs[q]), int(ta[q]), int(tw[q]), outs[0])
            clock += time.perf_counter() - t
            fifo_lat.append(clock - arr[j])
        # served results against the same queries alone (untimed)
        for q, got in samples:
            fns[kinds[q]](G, int(srcs[q]), int(ta[q]), int(tw[q]), outs[0])
            if not torch.equal(got, outs[0]):
                raise RuntimeError(f"served result of query {q} (kind {int(kinds[q])}) differs from the query alone")
        fl = np.array(fifo_lat) if fifo_lat else np.zeros(1)
        res.append({"rate": rate, "queries": count, "warmup": warmup, "served_qps": count / wall,
                    "checked_against_alone": len(samples),
                    "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                    "fifo_qps": float(n_fifo / clock) if clock > 0 else None,
                    "fifo_p50_ms": float(np.percentile(fl, 50) * 1e3) if n_fifo else None,
                    "fifo_p99_ms": float(np.percentile(fl, 99) * 1e3) if n_fifo else None})
        log(f"serve rate={rate}: {res[-1]}")
    return res


def _drain(K, srv, want):
    got = 0
    while got < want:
        got += len(K.kairos_server_poll(srv, 4096))
        time.sleep(0.0001)


def host_threads():
    """Threads the CPU leg may use: this process's CPU affinity, capped by
    OMP_NUM_THREADS when the host sets it (the host's share of cores)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def host_description():
    model, mem = "unknown", None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem = round(int(line.split()[1]) / 2**20, 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "mem_gib": mem}


def cpu_baseline(g, srcs, ta, tw, seconds):
    """The CPU oracle (one-pass scan over edges sorted by departure time),
    one query per host thread.  Timed on as many of the workload's queries
    as fit in about `seconds` of wall time (all of them when they fit);
    then, untimed, the oracle answers every query and counts the edges each
    traverses from its own result: the benchmark's numerator."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    cores = host_threads()
    q = len(srcs)
    t = time.perf_counter()
    se = oracle.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam, threads=cores)
    sort_s = time.perf_counter() - t
    # probe one query to size the timed sample
    t = time.perf_counter()
    oracle.earliest_arrival(se, srcs[0], ta[0], tw[0])
    per = max(time.perf_counter() - t, 1e-4)
    k = int(min(q, max(cores, seconds * cores / per)))
    k = max(1, min(k, q))
    results = {}

    def run(i):
        results[i] = oracle.earliest_arrival(se, srcs[i], ta[i], tw[i])

    t = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(run, range(k)))
    dt = time.perf_counter() - t

    def count(i):
        arr = results.pop(i) if i in results else oracle.earliest_arrival(se, srcs[i], ta[i], tw[i])
        return oracle.traversed_edges(se, ta[i], tw[i], arr)

    with ThreadPoolExecutor(cores) as ex:
        etrav = list(ex.map(count, range(q)))
    edges = float(sum(etrav[:k]))
    cpu = {"value": edges / dt, "unit": "edges/s", "cores": cores, "kind": "oracle",
           "queries_per_s": k / dt, "host": host_description(),
           "sample": f"first {k} of {q} queries of the workload, one per thread on {cores} threads; "
                     f"edges pre-sorted by departure once ({sort_s:.1f} s, not counted)"}
    return cpu, etrav


if __name__ == "__main__":
    main()
