"""HBM traffic of the benchmark's kernels from rocprofv3 counters.

    python bench_pmc.py run [bench args...]             # on the GPU host: three runs
    python bench_pmc.py summarize OUTDIR WORKLOAD MODE  # writes profiles/*.txt|json

`run` writes under $KAIROS_PROFILE_DIR (default profile_runs/) and
executes bench.py three times under rocprofv3: once with a kernel
trace and statistics, once collecting FETCH_SIZE and once WRITE_SIZE (each
counter in its own pass).  bench.py also copies a 256 MiB buffer with a
plain copy kernel in that process, which calibrates the counters: the copy
moves exactly 256 MiB each way, so the ratio of the counter reading to
256 MiB scales every other kernel's reading to HBM bytes.

`summarize` reads the rocpd databases and writes, per kernel, calls, mean
duration and the calibrated bytes per launch into
profiles/traffic_<workload>_<mode>.json (consumed by bench.py when the
kernel sources still hash the same) and a text summary
profiles/kernels_<workload>_<mode>.txt next to it.
"""
from __future__ import annotations

import collections
import glob
import hashlib
import json
import os
import re
import sqlite3
import subprocess
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
# the kernels the profiled workloads run (the small-graph kernel of tiny.hip
# serves graphs of at most 10,240 vertices, none of them)
KERNEL_SOURCES = ["paper_2401_02563_amd/csrc/traverse.hip", "paper_2401_02563_amd/csrc/batch.hip",
                  "paper_2401_02563_amd/csrc/build.hip", "paper_2401_02563_amd/csrc/stage.h",
                  "paper_2401_02563_amd/csrc/binned.h", "paper_2401_02563_amd/csrc/scan.h",
                  "paper_2401_02563_amd/csrc/sweep.h"]
COPY_BYTES = 256 << 20
# raw rocprofv3 output goes under this directory of the repository
OUT_ROOT = os.environ.get("KAIROS_PROFILE_DIR", "profile_runs")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(n: str) -> str:
    # template arguments (possibly several) are dropped: push_kernel<false, 256> -> push_kernel
    m = re.search(r"::(\w+)(<[^()]*>)?\(", n.replace("(anonymous namespace)", "anon"))
    if m:
        return m.group(1)
    return n.split("(")[0].strip()[-60:]


def run(argv):
    sys.path.insert(0, ROOT)
    from workloads import CONFIGS
    workload = argv[argv.index("--workload") + 1] if "--workload" in argv else "bursty22-1b"
    mode = argv[argv.index("--mode") + 1] if "--mode" in argv else CONFIGS[workload].get("bench_mode", "batch")
    out = os.path.join(ROOT, OUT_ROOT, f"pmc_{workload}_{mode}")
    os.makedirs(out, exist_ok=True)
    env = dict(os.environ, TMPDIR="/tmp", KAIROS_CALIBRATION_COPY="1")
    with open(os.path.join(out, "args.json"), "w") as f:
        json.dump(argv, f)  # the summary quotes the exact command
    # the timed earliest-arrival step only: the extra timings would mix other
    # query kinds into the per-kernel averages
    bench = [sys.executable, os.path.join(ROOT, "bench.py"), "--no-cpu", "--no-extras", *argv]
    passes = [("trace", ["--kernel-trace", "--stats"]), ("fetch", ["--pmc", "FETCH_SIZE"]),
              ("write", ["--pmc", "WRITE_SIZE"])]
    exits = {}
    for tag, opts in passes:
        cmd = ["timeout", "-s", "KILL", "240", "rocprofv3", *opts, "-d", os.path.join(out, tag), "-o", "run",
               "--", *bench]
        print("+", " ".join(cmd), flush=True)
        with open(os.path.join(out, f"{tag}.log"), "w") as log:
            rc = subprocess.call(cmd, stdout=log, stderr=subprocess.STDOUT, env=env)
        print(f"pass {tag} rc={rc}", flush=True)
        exits[tag] = rc
        with open(os.path.join(out, "exits.json"), "w") as f:
            json.dump(exits, f)  # the summary states every pass's exit status
        if rc in (-11, 139) and _bench_line_printed(os.path.join(out, f"{tag}.log")):
            # rocprofv3 can fault in its own exit handler after a cooperative
            # launch once the program has printed its last line; the results
            # are complete, and the summary records the fault
            print(f"pass {tag}: profiler faulted after the program finished (status {rc}); "
                  "results kept and the fault recorded in the summary", flush=True)
            continue
        if rc != 0:
            sys.exit(rc if rc > 0 else 1)


def _bench_line_printed(log_path):
    with open(log_path, errors="replace") as f:
        return any(line.startswith('{"metric"') for line in f)


def _db(path):
    dbs = glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True)
    if not dbs:
        raise FileNotFoundError(path)
    return sqlite3.connect(dbs[0])


def summarize(outdir, workload="bursty22-1b", mode="single"):
    trace = _db(os.path.join(outdir, "trace"))
    stats = collections.defaultdict(lambda: [0, 0.0])
    for name, dur in trace.execute("select name, duration from kernels"):
        s = stats[short_name(name)]
        s[0] += 1
        s[1] += dur
    counters = {}
    cal = {}
    for tag, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        agg = collections.defaultdict(lambda: [0, 0.0])
        best = None
        for name, val in _db(os.path.join(outdir, tag)).execute(
                "select name, counter_value from pmc_events where counter_name = ?", (ctr,)):
            k = short_name(name)
            a = agg[k]
            a[0] += 1
            a[1] += val
            # calibration: the one copy dispatch of COPY_BYTES (counters in KiB)
            if "copy" in k.lower():
                b = val * 1024.0
                if best is None or abs(b - COPY_BYTES) < abs(best - COPY_BYTES):
                    best = b
        counters[ctr] = agg
        cal[ctr] = (best / COPY_BYTES) if best else 1.0
    rows = {}
    for k, (n, dur) in stats.items():
        f = counters["FETCH_SIZE"].get(k)
        w = counters["WRITE_SIZE"].get(k)
        rows[k] = {
            "calls": n, "mean_us": dur / n / 1e3, "total_ms": dur / 1e6,
            "fetch_bytes_per_launch": (f[1] / f[0] * 1024.0 / cal["FETCH_SIZE"]) if f else None,
            "write_bytes_per_launch": (w[1] / w[0] * 1024.0 / cal["WRITE_SIZE"]) if w else None,
        }
    exits_path = os.path.join(outdir, "exits.json")
    exits = json.load(open(exits_path)) if os.path.exists(exits_path) else {}
    doc = {"workload": workload, "mode": mode, "kernel_sources_sha": kernel_source_hash(), "calibration": cal,
           "copy_bytes": COPY_BYTES, "profiler_exit_status": exits, "kernels": rows}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"traffic_{workload}_{mode}.json"), "w") as f:
        json.dump(doc, f, indent=1)
    argv = ["--workload", workload, "--mode", mode, "--steps", "3", "--warmup", "1"]
    if os.path.exists(os.path.join(outdir, "args.json")):
        argv = json.load(open(os.path.join(outdir, "args.json")))
    b = " ".join(["--no-cpu", "--no-extras", *argv])
    lines = [f"# rocprofv3 summary: bench.py workload {workload}, mode {mode}",
             "",
             "commands (from the repository root, on the GPU host; raw output under",
             f"$KAIROS_PROFILE_DIR, here {os.path.dirname(os.path.relpath(os.path.abspath(outdir), ROOT))}):",
             f"  python bench_pmc.py run {' '.join(argv)}",
             "  which makes three rocprofv3 passes, each its own process:",
             f"    rocprofv3 --kernel-trace --stats -- python bench.py {b}",
             f"    rocprofv3 --pmc FETCH_SIZE       -- python bench.py {b}",
             f"    rocprofv3 --pmc WRITE_SIZE       -- python bench.py {b}",
             f"  python bench_pmc.py summarize {os.path.relpath(os.path.abspath(outdir), ROOT)} {workload} {mode}",
             "",
             f"kernel sources sha256[:16]: {doc['kernel_sources_sha']}",
             "profiler exit status per pass: " + (", ".join(f"{k}={v}" for k, v in exits.items()) or "not recorded")
             + ("  (nonzero: rocprofv3 faulted in its own exit handler after the program printed its result line;"
                " the result files were complete)" if any(v != 0 for v in exits.values()) else ""),
             f"calibration (counter / true bytes of a {COPY_BYTES >> 20} MiB copy): "
             + ", ".join(f"{k}={v:.3f}" for k, v in cal.items()),
             "",
             f"{'kernel':34s} {'calls':>7s} {'mean_us':>10s} {'total_ms':>10s} {'fetch_MB/launch':>16s} {'write_MB/launch':>16s}"]
    for k, r in sorted(rows.items(), key=lambda kv: -kv[1]["total_ms"]):
        fb = f"{r['fetch_bytes_per_launch'] / 1e6:16.2f}" if r["fetch_bytes_per_launch"] is not None else f"{'-':>16s}"
        wb = f"{r['write_bytes_per_launch'] / 1e6:16.2f}" if r["write_bytes_per_launch"] is not None else f"{'-':>16s}"
        lines.append(f"{k[:34]:34s} {r['calls']:7d} {r['mean_us']:10.2f} {r['total_ms']:10.2f} {fb} {wb}")
    with open(os.path.join(ROOT, "profiles", f"kernels_{workload}_{mode}.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "run":
        run(sys.argv[2:])
    elif len(sys.argv) >= 3 and sys.argv[1] == "summarize":
        summarize(sys.argv[2], *(sys.argv[3:5]))
    else:
        print(__doc__)
        sys.exit(2)
