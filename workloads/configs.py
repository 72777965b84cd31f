"""Named synthetic workloads.

Each entry fixes the graph recipe, its seed and the query recipe.  The
graphs stand in for the paper's datasets (Table 3), which are not used:
they reproduce the traits the paper relies on (skewed degrees from R-MAT,
bursty per-pair times, uniform durations) and its "fraction of recent
edges" window sweeps (§6.2, §6.5) with log-uniform window widths.

  uniform-10k     10,000 vertices, 100,000 uniform edges, t in [0, 100000),
                  lam in [1, 10]; 16 sources, window [0, 99999].
  rmat20-32m      R-MAT scale 20, 2^25 edges, (a,b,c,d) = (.57,.19,.19,.05),
                  t uniform in [0, 2^30), lam = 1; 64 sources, t_alpha in the
                  first half of the span, t_omega = max.
  bursty22-1b     R-MAT scale-22 pairs (12 * 2^22 of them), each repeated
                  Geometric(mean 20) times, Pareto(1.5) bursts normalised to
                  uint32, lam in [1, 100]; 32 sources, windows as rmat20-32m.
  rmat22-256m     R-MAT scale 22, 2^28 edges, t uniform over uint32 (headroom
                  of 10 below the largest finite time), lam in [1, 10];
                  256 queries with log-uniform widths from 0.1% to 100%.
  serve-rmat20    the rmat20-32m graph, Poisson arrivals, kinds 60/20/20
                  EA/LD/F, log-uniform windows.
  rmat24-512m     R-MAT scale 24, 2^29 edges, otherwise like rmat20-32m.

``bench_mode`` is the form the benchmark times by default: one query per
call for the single-source workloads, one batched call for the batch.

``scale_shift`` shrinks an R-MAT recipe by that many powers of two in both
vertices and edges (same edge factor), for tests that must finish quickly.
"""
from __future__ import annotations

import numpy as np

from .gen import (TMAX, Graph, bursty_pair_graph, first_half_windows, log_uniform_windows,
                  query_kinds, rmat_graph, sample_sources, uniform_graph)

CONFIGS = {
    "uniform-10k": dict(kind="uniform", n=10_000, m=100_000, seed=1, t_lo=0, t_hi=99_999,
                        lam_lo=1, lam_hi=10, queries=16, qseed=101, window="fixed",
                        t_alpha=0, t_omega=99_999, bench_mode="single"),
    "rmat20-32m": dict(kind="rmat", scale=20, m=1 << 25, seed=2, t_lo=0, t_hi=(1 << 30) - 1,
                       lam_lo=1, lam_hi=1, queries=64, qseed=102, window="first_half",
                       bench_mode="single"),
    "bursty22-1b": dict(kind="bursty", scale=22, pairs=12 << 22, seed=3, lam_lo=1, lam_hi=100,
                        queries=32, qseed=103, window="first_half", bench_mode="single"),
    "rmat22-256m": dict(kind="rmat", scale=22, m=1 << 28, seed=4, t_lo=0, t_hi=TMAX - 10,
                        lam_lo=1, lam_hi=10, queries=256, qseed=104, window="log_uniform",
                        bench_mode="batch"),
    "serve-rmat20": dict(kind="rmat", scale=20, m=1 << 25, seed=2, t_lo=0, t_hi=(1 << 30) - 1,
                         lam_lo=1, lam_hi=1, queries=20_000, qseed=105, window="log_uniform",
                         rates=[1_000, 2_000, 5_000, 10_000, 20_000, 50_000], warmup=1_000),
    "rmat24-512m": dict(kind="rmat", scale=24, m=1 << 29, seed=24, t_lo=0, t_hi=(1 << 30) - 1,
                        lam_lo=1, lam_hi=1, queries=64, qseed=124, window="first_half",
                        bench_mode="single"),
}


def make_graph(name: str, scale_shift: int = 0) -> Graph:
    c = CONFIGS[name]
    if c["kind"] == "uniform":
        g = uniform_graph(c["n"], c["m"], c["seed"], c["t_lo"], c["t_hi"], c["lam_lo"], c["lam_hi"])
    elif c["kind"] == "rmat":
        g = rmat_graph(c["scale"] - scale_shift, c["m"] >> scale_shift, c["seed"], c["t_lo"],
                       c["t_hi"], c["lam_lo"], c["lam_hi"])
    elif c["kind"] == "bursty":
        g = bursty_pair_graph(c["scale"] - scale_shift, c["pairs"] >> scale_shift, c["seed"],
                              lam_lo=c["lam_lo"], lam_hi=c["lam_hi"])
    else:
        raise ValueError(c["kind"])
    g.meta["config"] = name
    g.meta["scale_shift"] = scale_shift
    return g


def _span(g: Graph, c: dict):
    if "t_lo" in c:
        return c["t_lo"], c["t_hi"]
    return int(g.t.min()), int(g.t.max())


def make_queries(name: str, g: Graph, count: int | None = None, held_out: bool = False):
    """Return (sources, t_alpha, t_omega) as uint32 arrays.

    ``held_out``: queries of the same recipe drawn from another seed, for
    tuning on a sample that is not the one timed."""
    c = CONFIGS[name]
    k = c["queries"] if count is None else count
    ss = np.random.SeedSequence([c["qseed"], 1] if held_out else c["qseed"]).spawn(2)
    src = sample_sources(g, k, int(ss[0].generate_state(1)[0]))
    lo, hi = _span(g, c)
    wseed = int(ss[1].generate_state(1)[0])
    if c["window"] == "fixed":
        ta = np.full(k, c["t_alpha"], np.uint32)
        tw = np.full(k, c["t_omega"], np.uint32)
    elif c["window"] == "first_half":
        ta, tw = first_half_windows(k, lo, hi, wseed)
    else:
        ta, tw = log_uniform_windows(k, lo, hi, wseed)
    return src, ta, tw


def make_kinds(name: str, count: int) -> np.ndarray:
    c = CONFIGS[name]
    return query_kinds(count, c["qseed"] + 7)
