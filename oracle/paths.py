"""Oracle for path-shaped outputs -- TEST INFRASTRUCTURE ONLY.

Plain numpy and Python, no code shared with the GPU library.  Each
function writes out a definition directly (no blocking, no reordering):

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
  a <= t_omega; consecutive edges "Succeeds" (t >= arrival) by default or
  "Strictly succeeds" (t > arrival).  Its EA_h at the fixpoint is the
  earliest arrival under either predicate.
* ``strict_sweep`` -- latest departure and fastest under either succession
  predicate, by their cross-route definitions over the source's departure
  times S: LD[v] = max{s in S : v reachable when the source starts at s},
  F[v] = min over s in S of (EA_s[v] - s), with EA_s from ``min_hops``.

* ``latest_departure_to`` -- single-target latest departure (the
  single-target reading of the latest-departure path of §2.3): for every
  vertex u, the latest departure from u of a time-respecting path that ends
  at the target within [t_alpha, t_omega]; t_omega for the target itself.
  Computed level by level: L_0 has only the target (at t_omega);
  L_{h+1}[u] is the largest of L_h[u] and the departure t of every usable
  edge (u, v, t, a) whose arrival lets the path continue from v, a <= L_h[v]
  (a < L_h[v] strictly; the target itself accepts a <= t_omega under either
  predicate, as the end of a path has no successor).

Succession (§2.2): "Succeeds" lets the next edge leave at the previous
arrival (t >= arrival); "Strictly succeeds" needs t > arrival.  The first
edge of a path has no predecessor, so under either predicate it only needs
t >= the source's start (t_alpha, or s in a sweep).

``brute_force_walks`` enumerates every time-respecting walk of a tiny graph
and returns, per vertex, the earliest arrival, the set of (tail, departure)
pairs that end a walk arriving at it, the fewest edges of any walk, and the
latest departure and fastest duration; the tests pin the functions above to
it.

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


def min_hops(n, src, dst, t, lam, source, t_alpha, t_omega, strict=False):
    """(hops, ea): fewest edges of a time-respecting path from ``source``,
    and the earliest arrival, by levels EA_0, EA_1, ... as defined above
    (``strict``: consecutive edges follow "Strictly succeeds")."""
    src, dst, t, a = _edges(src, dst, t, lam)
    usable = (t >= t_alpha) & (a <= t_omega)
    src, dst, t, a = src[usable], dst[usable], t[usable], a[usable]
    cur = np.full(n, INF, np.int64)
    cur[source] = t_alpha
    hops = np.full(n, INF, np.int64)
    hops[source] = 0
    # the source's own edges only need t >= its start
    after = (src == source) | (not strict)
    h = 0
    while True:
        h += 1
        ok = (cur[src] != INF) & np.where(after, cur[src] <= t, cur[src] < t)
        nxt = cur.copy()
        np.minimum.at(nxt, dst[ok], a[ok])
        if np.array_equal(nxt, cur):
            break
        new = (cur == INF) & (nxt != INF)
        hops[new] = h
        cur = nxt
    return hops.astype(np.uint32), cur.astype(np.uint32)


def strict_sweep(n, src, dst, t, lam, source, t_alpha, t_omega, strict=False):
    """(ld, fastest) by the cross-route definitions above."""
    src_, dst_, t_, a_ = _edges(src, dst, t, lam)
    first = (src_ == source) & (t_ >= t_alpha) & (a_ <= t_omega)
    ld = np.full(n, INF, np.int64)
    fa = np.full(n, INF, np.int64)
    for s in sorted(set(t_[first].tolist())):
        _, ea_s = min_hops(n, src, dst, t, lam, source, s, t_omega, strict)
        ea_s = ea_s.astype(np.int64)
        r = ea_s != INF
        ld[r] = s  # ascending s: the last one that reaches v is the largest
        fa[r] = np.minimum(fa[r], ea_s[r] - s)
    ld[source] = t_omega
    fa[source] = 0
    return ld.astype(np.uint32), fa.astype(np.uint32)


def latest_departure_to(n, src, dst, t, lam, target, t_alpha, t_omega, strict=False):
    """Latest departure towards ``target`` by the level iteration above."""
    src, dst, t, a = _edges(src, dst, t, lam)
    usable = (t >= t_alpha) & (a <= t_omega)
    src, dst, t, a = src[usable], dst[usable], t[usable], a[usable]
    NONE = -1
    cur = np.full(n, NONE, np.int64)
    cur[target] = t_omega
    into_target = dst == target
    while True:
        lv = cur[dst]
        ok = (lv != NONE) & np.where(into_target | (not strict), a <= lv, a < lv)
        nxt = cur.copy()
        np.maximum.at(nxt, src[ok], t[ok])
        nxt[target] = t_omega
        if np.array_equal(nxt, cur):
            break
        cur = nxt
    cur[cur == NONE] = INF
    return cur.astype(np.uint32)


def brute_force_to(n, edges, target, t_alpha, t_omega, strict=False):
    """Latest departure towards ``target`` by enumerating every walk from
    every vertex (tiny inputs only)."""
    out = [[] for _ in range(n)]
    for (u, v, t, lam) in edges:
        if t >= t_alpha and t + lam <= t_omega:
            out[u].append((v, t, t + lam))
    best = [INF] * n
    best[target] = t_omega

    def walk(start, u, now, first):
        for (v, t, a) in out[u]:
            if first is not None and (t < now or (strict and t == now)):
                continue
            d = t if first is None else first
            if v == target and d != INF:
                if v != start and (best[start] == INF or d > best[start]):
                    best[start] = d
            walk(start, v, a, d)

    for s0 in range(n):
        if s0 != target:
            walk(s0, s0, t_alpha, None)
    return best


def brute_force_walks(n, edges, source, t_alpha, t_omega, strict=False):
    """Every time-respecting walk from ``source`` (tiny inputs only).

    ``edges`` is a list of (u, v, t, lam).  Returns (ea, last, hops, ld,
    fastest): the earliest arrival per vertex, per vertex the set of (tail,
    departure) pairs of last edges of walks that arrive at ea[v], the fewest
    edges of any walk reaching the vertex, the latest departure from the
    source of a walk reaching it and the least (arrival - departure)."""
    ea = [INF] * n
    hops = [INF] * n
    ld = [INF] * n
    fa = [INF] * n
    ends = [dict() for _ in range(n)]  # arrival -> set of (tail, departure)
    out = [[] for _ in range(n)]
    for (u, v, t, lam) in edges:
        if t >= t_alpha and t + lam <= t_omega:
            out[u].append((v, t, t + lam))

    def walk(u, now, k, dep):
        for (v, t, a) in out[u]:
            if t < now or (strict and k > 0 and t == now):
                continue
            d = t if k == 0 else dep
            if a < ea[v]:
                ea[v] = a
            hops[v] = min(hops[v], k + 1)
            ld[v] = d if ld[v] == INF else max(ld[v], d)
            fa[v] = min(fa[v], a - d)
            ends[v].setdefault(a, set()).add((u, t))
            walk(v, a, k + 1, d)

    walk(source, t_alpha, 0, None)
    ea[source] = t_alpha
    hops[source] = 0
    ld[source] = t_omega
    fa[source] = 0
    last = [set() if v == source or ea[v] == INF else ends[v][ea[v]] for v in range(n)]
    return ea, last, hops, ld, fa
