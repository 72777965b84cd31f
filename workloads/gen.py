"""Seeded generators for temporal multigraphs, query sources, time windows
and arrival traces.

Every generator takes an explicit integer seed and uses numpy's PCG64 via
``numpy.random.SeedSequence``.  Large edge lists are produced in fixed-size
chunks whose child seeds come from ``SeedSequence.spawn``, so the output is
identical whatever number of worker threads fills the chunks.

Edge model (paper §2.1): a temporal edge joins ``src`` to ``dst`` and is
valid over a discrete interval; here that interval is written as a
departure time ``t`` and a duration ``lam`` >= 1, so the edge ends (arrives)
at ``t + lam``.  All arrays are ``uint32``.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

INF = 0xFFFFFFFF          # "no arrival" in every output
TMAX = 0xFFFFFFFE         # largest finite time value

_CHUNK = 1 << 22


def _workers() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


@dataclass
class Graph:
    """A temporal edge list plus the recipe that produced it."""
    n: int
    src: np.ndarray
    dst: np.ndarray
    t: np.ndarray
    lam: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def out_degree(self) -> np.ndarray:
        return np.bincount(self.src, minlength=self.n).astype(np.int64)


def _fill_chunks(m: int, seed: int, fn, workers: int | None = None) -> None:
    """Call ``fn(rng, lo, hi)`` for fixed chunks of [0, m) with spawned seeds."""
    nchunks = max(1, math.ceil(m / _CHUNK))
    children = np.random.SeedSequence(seed).spawn(nchunks)

    def run(i: int) -> None:
        lo = i * _CHUNK
        hi = min(m, lo + _CHUNK)
        if hi > lo:
            fn(np.random.Generator(np.random.PCG64(children[i])), lo, hi)

    w = workers or _workers()
    if w == 1 or nchunks == 1:
        for i in range(nchunks):
            run(i)
    else:
        with ThreadPoolExecutor(w) as ex:
            list(ex.map(run, range(nchunks)))


def _uniform_u32(rng, lo: int, hi: int, size: int) -> np.ndarray:
    """Uniform integers in the closed range [lo, hi] as uint32."""
    return rng.integers(lo, hi, size=size, endpoint=True, dtype=np.uint64).astype(np.uint32)


def _times(m: int, seed: int, t_lo: int, t_hi: int, lam_lo: int, lam_hi: int):
    t = np.empty(m, np.uint32)
    lam = np.empty(m, np.uint32)

    def fill(rng, lo, hi):
        t[lo:hi] = _uniform_u32(rng, t_lo, t_hi, hi - lo)
        lam[lo:hi] = _uniform_u32(rng, lam_lo, lam_hi, hi - lo)

    _fill_chunks(m, seed, fill)
    return t, lam


def uniform_graph(n: int, m: int, seed: int, t_lo: int, t_hi: int,
                  lam_lo: int, lam_hi: int) -> Graph:
    """Endpoints i.i.d. uniform over [0, n); t uniform in [t_lo, t_hi];
    lam uniform in [lam_lo, lam_hi]."""
    ss = np.random.SeedSequence(seed).spawn(2)
    src = np.empty(m, np.uint32)
    dst = np.empty(m, np.uint32)

    def fill(rng, lo, hi):
        src[lo:hi] = _uniform_u32(rng, 0, n - 1, hi - lo)
        dst[lo:hi] = _uniform_u32(rng, 0, n - 1, hi - lo)

    _fill_chunks(m, int(ss[0].generate_state(1)[0]), fill)
    t, lam = _times(m, int(ss[1].generate_state(1)[0]), t_lo, t_hi, lam_lo, lam_hi)
    return Graph(n, src, dst, t, lam, dict(kind="uniform", seed=seed, t_lo=t_lo, t_hi=t_hi,
                                          lam_lo=lam_lo, lam_hi=lam_hi))


def _rmat_pairs(scale: int, m: int, abcd, seed: int):
    """R-MAT endpoint pairs: at each of ``scale`` levels pick one of the four
    quadrants with probabilities (a, b, c, d), most significant bit first; no
    noise.  A seeded permutation relabels the vertices.  Duplicate pairs and
    self-loops are kept."""
    a, b, c, _d = abcd
    thr_a = np.uint64(round(a * 2 ** 32))
    thr_ab = np.uint64(round((a + b) * 2 ** 32))
    thr_abc = np.uint64(round((a + b + c) * 2 ** 32))
    n = 1 << scale
    ss = np.random.SeedSequence(seed).spawn(2)
    src = np.empty(m, np.uint32)
    dst = np.empty(m, np.uint32)

    def fill(rng, lo, hi):
        k = hi - lo
        s = np.zeros(k, np.uint32)
        d = np.zeros(k, np.uint32)
        for _ in range(scale):
            r = rng.integers(0, 1 << 32, size=k, dtype=np.uint64)
            sb = r >= thr_ab
            db = ((r >= thr_a) & (r < thr_ab)) | (r >= thr_abc)
            s = (s << np.uint32(1)) | sb.astype(np.uint32)
            d = (d << np.uint32(1)) | db.astype(np.uint32)
        src[lo:hi] = s
        dst[lo:hi] = d

    _fill_chunks(m, int(ss[0].generate_state(1)[0]), fill)
    perm = np.random.Generator(np.random.PCG64(ss[1])).permutation(n).astype(np.uint32)
    # relabel in chunks to bound temporaries
    for lo in range(0, m, _CHUNK):
        hi = min(m, lo + _CHUNK)
        src[lo:hi] = perm[src[lo:hi]]
        dst[lo:hi] = perm[dst[lo:hi]]
    return n, src, dst


def rmat_graph(scale: int, m: int, seed: int, t_lo: int, t_hi: int,
               lam_lo: int, lam_hi: int, abcd=(0.57, 0.19, 0.19, 0.05)) -> Graph:
    """R-MAT temporal graph with uniform departure times and durations."""
    ss = np.random.SeedSequence(seed).spawn(2)
    n, src, dst = _rmat_pairs(scale, m, abcd, int(ss[0].generate_state(1)[0]))
    t, lam = _times(m, int(ss[1].generate_state(1)[0]), t_lo, t_hi, lam_lo, lam_hi)
    return Graph(n, src, dst, t, lam, dict(kind="rmat", scale=scale, seed=seed, abcd=list(abcd),
                                          t_lo=t_lo, t_hi=t_hi, lam_lo=lam_lo, lam_hi=lam_hi))


def bursty_pair_graph(scale: int, pairs: int, seed: int, mean_repeat: float = 20.0,
                      pareto_alpha: float = 1.5, offset_width: float = 1e6,
                      lam_lo: int = 1, lam_hi: int = 100,
                      abcd=(0.57, 0.19, 0.19, 0.05)) -> Graph:
    """Communication-style multigraph: R-MAT endpoint pairs, each repeated a
    Geometric(p = 1/mean_repeat) number of times (support 1, 2, ...).  Within a
    pair the raw times are ``o + cumsum(gaps)`` with ``o ~ U[0,1) * W`` and
    gaps Pareto-I(alpha, x_m = 1).  Raw times are then floor-normalised onto
    [0, 2^32 - 2^8] over the whole graph, leaving headroom for lam."""
    ss = np.random.SeedSequence(seed).spawn(3)
    n, psrc, pdst = _rmat_pairs(scale, pairs, abcd, int(ss[0].generate_state(1)[0]))
    rep = np.empty(pairs, np.int64)
    off = np.empty(pairs, np.float64)

    def fill_pairs(rng, lo, hi):
        rep[lo:hi] = rng.geometric(1.0 / mean_repeat, size=hi - lo)
        off[lo:hi] = rng.random(hi - lo) * offset_width

    _fill_chunks(pairs, int(ss[1].generate_state(1)[0]), fill_pairs)
    starts = np.zeros(pairs + 1, np.int64)
    np.cumsum(rep, out=starts[1:])
    m = int(starts[-1])
    raw = np.empty(m, np.float64)
    # chunk over pairs so that a pair never straddles two chunks
    pchunk = _CHUNK // 32
    nch = max(1, math.ceil(pairs / pchunk))
    children = np.random.SeedSequence(int(ss[2].generate_state(1)[0])).spawn(nch)

    def fill_times(i):
        plo = i * pchunk
        phi = min(pairs, plo + pchunk)
        if phi <= plo:
            return
        rng = np.random.Generator(np.random.PCG64(children[i]))
        elo, ehi = int(starts[plo]), int(starts[phi])
        k = rep[plo:phi]
        gaps = 1.0 + rng.pareto(pareto_alpha, size=ehi - elo)
        cs = np.cumsum(gaps)
        first = (starts[plo:phi] - elo)
        base = np.repeat(cs[first] - gaps[first], k)
        raw[elo:ehi] = np.repeat(off[plo:phi], k) + (cs - base)

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(fill_times, range(nch)))
    rmin = float(raw.min())
    rmax = float(raw.max())
    top = float((1 << 32) - (1 << 8))
    scale_f = top / (rmax - rmin) if rmax > rmin else 0.0
    t = np.empty(m, np.uint32)
    for lo in range(0, m, _CHUNK):
        hi = min(m, lo + _CHUNK)
        t[lo:hi] = np.minimum(np.floor((raw[lo:hi] - rmin) * scale_f), top).astype(np.uint32)
    del raw
    src = np.repeat(psrc, rep)
    dst = np.repeat(pdst, rep)
    lam = np.empty(m, np.uint32)

    def fill_lam(rng, lo, hi):
        lam[lo:hi] = _uniform_u32(rng, lam_lo, lam_hi, hi - lo)

    _fill_chunks(m, int(ss[2].generate_state(2)[1]), fill_lam)
    return Graph(n, src, dst, t, lam, dict(kind="bursty", scale=scale, pairs=pairs, seed=seed,
                                          mean_repeat=mean_repeat, pareto_alpha=pareto_alpha,
                                          offset_width=offset_width, lam_lo=lam_lo, lam_hi=lam_hi))


def tiny_graph(seed: int, n: int = 7, m: int = 10, t_max: int = 8, lam_max: int = 3) -> Graph:
    """Small dense-tie multigraph for exhaustive checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    src = _uniform_u32(rng, 0, n - 1, m)
    dst = _uniform_u32(rng, 0, n - 1, m)
    t = _uniform_u32(rng, 0, t_max, m)
    lam = _uniform_u32(rng, 1, lam_max, m)
    return Graph(n, src, dst, t, lam, dict(kind="tiny", seed=seed))


def sample_sources(g: Graph, k: int, seed: int) -> np.ndarray:
    """Sources drawn uniformly among vertices with at least one out-edge
    (without replacement while enough exist)."""
    cand = np.nonzero(g.out_degree())[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    if cand.size == 0:
        return rng.integers(0, g.n, size=k).astype(np.uint32)
    replace = cand.size < k
    return rng.choice(cand, size=k, replace=replace).astype(np.uint32)


def first_half_windows(k: int, t_lo: int, t_hi: int, seed: int):
    """t_alpha uniform over the first half of [t_lo, t_hi]; t_omega = TMAX."""
    rng = np.random.Generator(np.random.PCG64(seed))
    half = (t_hi - t_lo + 1) // 2
    ta = _uniform_u32(rng, t_lo, t_lo + max(half, 1) - 1, k)
    tw = np.full(k, TMAX, np.uint32)
    return ta, tw


def log_uniform_windows(k: int, t_lo: int, t_hi: int, seed: int,
                        f_lo_exp: float = -3.0, f_hi_exp: float = 0.0):
    """Window width w = floor(f * T) with f = 10^U(f_lo_exp, f_hi_exp) and
    T = t_hi - t_lo; t_alpha uniform in [t_lo, t_lo + T - w]; t_omega = t_alpha + w."""
    rng = np.random.Generator(np.random.PCG64(seed))
    span = t_hi - t_lo
    f = 10.0 ** rng.uniform(f_lo_exp, f_hi_exp, size=k)
    w = np.floor(f * span).astype(np.uint64)
    ta = np.array([int(rng.integers(t_lo, t_lo + span - int(wi), endpoint=True)) for wi in w],
                  dtype=np.uint64)
    tw = ta + w
    return ta.astype(np.uint32), tw.astype(np.uint32)


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Open-loop arrival times in seconds (exponential inter-arrivals)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def query_kinds(count: int, seed: int, probs=(0.6, 0.2, 0.2)) -> np.ndarray:
    """Query kinds 0 = earliest arrival, 1 = latest departure, 2 = fastest."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.choice(3, size=count, p=list(probs)).astype(np.int32)
