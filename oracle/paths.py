"""Oracle for path-shaped outputs -- TEST INFRASTRUCTURE ONLY.

Plain numpy and Python, no code shared with the GPU library.  Both
functions write out a definition directly (no blocking, no reordering):

* ``ea_predecessors`` -- the last edge of an earliest-arrival path to every
  vertex (the path itself is Alg. 2's Ensure t[V] plus the edge that set
  each t[v]; §2.3 names earliest-arrival paths).  Several last edges can be
  optimal, so one is chosen by a fixed rule: among the usable edges
  (u, v, t, a) with a = EA[v] and EA[u] <= t, the latest departure t, then
  the smallest tail id u.  Edges with the same (u, v, t, a) are the same
  choice, so the rule leaves nothing open.
* ``min_hops`` -- temporal BFS (Table 4's T. BFS adapted to the query
  window, as §6.1 describes for BFS): the fewest edges on a time-respecting
  path from the source within [t_alpha, t_omega].  Computed level by level:
  EA_0 has only the source (at t_alpha); EA_{h+1}[v] is the least of
  EA_h[v] and every usable edge (u, v, t, a) with EA_h[u] <= t; hops[v] is
  the first h at which EA_h[v] is finite.  Usable: t >= t_alpha and
  a <= t_omega, consecutive edges non-strict (t >= arrival), as for every
  query here.

``brute_force_walks`` enumerates every time-respecting walk of a tiny graph
and returns, per vertex, the earliest arrival, the set of (tail, departure)
pairs that end a walk arriving at it, and the fewest edges of any walk; the
tests pin both functions above to it.

0xFFFFFFFF marks "none" (unreached vertices, and the source's predecessor).
"""
from __future__ import annotations

import numpy as np

INF = 0xFFFFFFFF


def _edges(src, dst, t, lam):
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    t = np.asarray(t, np.int64)
    a = t + np.asarray(lam, np.int64)
    return src, dst, t, a


def ea_predecessors(n, src, dst, t, lam, source, t_alpha, t_omega, ea):
    """(pred_tail, pred_departure) for the earliest-arrival array ``ea``."""
    src, dst, t, a = _edges(src, dst, t, lam)
    E = np.asarray(ea, np.int64)
    usable = (t >= t_alpha) & (a <= t_omega)
    reached_tail = E[src] != INF
    optimal = usable & reached_tail & (E[src] <= t) & (a == E[dst]) & (dst != source)
    pred_tail = np.full(n, INF, np.int64)
    pred_dep = np.full(n, INF, np.int64)
    # per head: the largest departure, then the smallest tail
    idx = np.nonzero(optimal)[0]
    order = np.lexsort((src[idx], -t[idx], dst[idx]))
    idx = idx[order]
    first = np.ones(idx.size, bool)
    first[1:] = dst[idx[1:]] != dst[idx[:-1]]
    pick = idx[first]
    pred_tail[dst[pick]] = src[pick]
    pred_dep[dst[pick]] = t[pick]
    return pred_tail.astype(np.uint32), pred_dep.astype(np.uint32)


def min_hops(n, src, dst, t, lam, source, t_alpha, t_omega):
    """(hops, ea): fewest edges of a time-respecting path from ``source``,
    and the earliest arrival, by levels EA_0, EA_1, ... as defined above."""
    src, dst, t, a = _edges(src, dst, t, lam)
    usable = (t >= t_alpha) & (a <= t_omega)
    src, dst, t, a = src[usable], dst[usable], t[usable], a[usable]
    cur = np.full(n, INF, np.int64)
    cur[source] = t_alpha
    hops = np.full(n, INF, np.int64)
    hops[source] = 0
    h = 0
    while True:
        h += 1
        ok = (cur[src] != INF) & (cur[src] <= t)
        nxt = cur.copy()
        np.minimum.at(nxt, dst[ok], a[ok])
        if np.array_equal(nxt, cur):
            break
        new = (cur == INF) & (nxt != INF)
        hops[new] = h
        cur = nxt
    return hops.astype(np.uint32), cur.astype(np.uint32)


def brute_force_walks(n, edges, source, t_alpha, t_omega):
    """Every time-respecting walk from ``source`` (tiny inputs only).

    ``edges`` is a list of (u, v, t, lam).  Returns (ea, last, hops): the
    earliest arrival per vertex, per vertex the set of (tail, departure)
    pairs of last edges of walks that arrive at ea[v], and the fewest edges
    of any walk reaching the vertex."""
    ea = [INF] * n
    hops = [INF] * n
    ends = [dict() for _ in range(n)]  # arrival -> set of (tail, departure)
    out = [[] for _ in range(n)]
    for (u, v, t, lam) in edges:
        if t >= t_alpha and t + lam <= t_omega:
            out[u].append((v, t, t + lam))

    def walk(u, now, k):
        for (v, t, a) in out[u]:
            if t < now:
                continue
            if a < ea[v]:
                ea[v] = a
            hops[v] = min(hops[v], k + 1)
            ends[v].setdefault(a, set()).add((u, t))
            walk(v, a, k + 1)

    walk(source, t_alpha, 0)
    ea[source] = t_alpha
    hops[source] = 0
    last = [set() if v == source or ea[v] == INF else ends[v][ea[v]] for v in range(n)]
    return ea, last, hops
