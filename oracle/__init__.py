"""CPU oracle for temporal minimal-path queries -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
use this package.  It shares no code with the GPU library: the C part
(``kairos_oracle.c``) is compiled separately with the host compiler, and
the Python part below uses numpy and the standard library only.

Contents (each function names the passage of the paper it follows):

* ``sort_by_departure``      -- edge list sorted by departure time (a plain
                                library sort), with a = t + lambda.
* ``earliest_arrival``       -- one-pass EA scan (C).
* ``profile``                -- EA / LD / F by Pareto profiles (C).
* ``traversed_edges``        -- temporal edges traversed by a query (C).
* ``shortest_duration``      -- least total duration by Pareto profiles of
                                (arrival, duration) (C).
* ``ea_certificate``         -- O(m) check that an array is exactly EA
                                (numpy; ``ea_certificate_scan``: the same
                                three conditions as one C loop, for 10^9
                                edges).
* ``brute_force``            -- enumeration of all time-respecting walks
                                (pure Python, tiny inputs only);
                                ``walk_facts`` adds, per walk, the edges it
                                uses and its total duration.
* ``temporal_csr``           -- expected out/in temporal CSR (numpy lexsort).
* ``paths.ea_predecessors``  -- last edge of an earliest-arrival path (numpy).
* ``paths.min_hops``         -- temporal BFS: fewest edges within the window.
* ``paths.brute_force_walks``-- enumeration pinning the two above.

Reading of the paper used throughout, where its text leaves a point open
or garbled:
  * a = t + lambda with lambda >= 1;
  * consecutive edges follow the non-strict "Succeeds" predicate of §2.2
    (next departure >= previous arrival), as the Update test of Alg. 2 does;
  * an edge is usable iff t >= t_alpha and a <= t_omega (closed window of
    Alg. 2's input interval);
  * the source starts at t_alpha, and a vertex is revisited whenever its
    arrival improves (Alg. 2's visit-once flag is not applied: it can miss
    an earlier arrival over a longer path);
  * latest departure is single-source (max departure from src of a path
    reaching v); fastest is min (arrival - departure from src);
  * 0xFFFFFFFF means unreachable.

Parity pins: brute force, the EA certificate, scipy shortest paths on
time-replicated static graphs, cross-routes and metamorphic relations; see
``tests/test_oracle.py``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

INF = 0xFFFFFFFF
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        lib.oracle_earliest_arrival.restype = u64
        lib.oracle_earliest_arrival.argtypes = [u64, p, p, p, p, u32, u32, u32, u32, p]
        lib.oracle_traversed_edges.restype = u64
        lib.oracle_traversed_edges.argtypes = [u64, p, p, p, u32, u32, p]
        lib.oracle_profile.restype = ctypes.c_int
        lib.oracle_profile.argtypes = [u64, p, p, p, p, u32, u32, u32, u32, p, p, p]
        lib.oracle_shortest_duration.restype = ctypes.c_int
        lib.oracle_shortest_duration.argtypes = [u64, p, p, p, p, u32, u32, u32, u32, ctypes.c_int, p]
        lib.oracle_ea_certificate.restype = ctypes.c_int
        lib.oracle_ea_certificate.argtypes = [u64, p, p, p, p, u32, u32, u32, u32, p, p]
        _LIB = lib
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class SortedEdges:
    """Edges sorted by departure time: parallel uint32 arrays src, dst, t, a."""

    def __init__(self, n, src, dst, t, a):
        self.n = int(n)
        self.src = np.ascontiguousarray(src, np.uint32)
        self.dst = np.ascontiguousarray(dst, np.uint32)
        self.t = np.ascontiguousarray(t, np.uint32)
        self.a = np.ascontiguousarray(a, np.uint32)

    @property
    def m(self):
        return int(self.src.shape[0])


def _threads() -> int:
    return max(1, os.cpu_count() or 1)


def _chunks(m: int, parts: int):
    step = -(-m // parts) if m else 1
    return [(lo, min(m, lo + step)) for lo in range(0, m, step)]


def departure_order(t, threads: int | None = None) -> np.ndarray:
    """The stable order of ``t`` (np.argsort(t, kind="stable")), as int64.

    A plain library sort of the packed keys (t << 32 | position), which are
    distinct, so sorting them is sorting by t with ties by position.  For
    large inputs the keys are sorted in P slices on P threads, split at
    common key bounds taken from the sorted slices, and each of the P key
    ranges sorted again on its own thread: range j holds exactly the keys
    between bound j-1 and bound j, so the ranges placed one after another
    are the whole sorted sequence."""
    t = np.asarray(t, np.uint32)
    m = int(t.size)
    P = threads or _threads()
    if m < (1 << 22) or P == 1:
        return np.argsort(t, kind="stable").astype(np.int64)
    from concurrent.futures import ThreadPoolExecutor
    keys = np.empty(m, np.uint64)
    parts = _chunks(m, P)

    def pack(c):
        lo, hi = c
        np.left_shift(t[lo:hi].astype(np.uint64), np.uint64(32), out=keys[lo:hi])
        keys[lo:hi] |= np.arange(lo, hi, dtype=np.uint64)
        keys[lo:hi].sort()

    with ThreadPoolExecutor(P) as ex:
        list(ex.map(pack, parts))
        # bounds: every (m/P)-th key of the union, estimated from the slices
        sample = np.sort(np.concatenate([keys[lo:hi][:: max(1, (hi - lo) // 256)] for lo, hi in parts]))
        bounds = sample[np.linspace(0, sample.size, P + 1).astype(np.int64)[1:-1]]
        cuts = [np.searchsorted(keys[lo:hi], bounds) + lo for lo, hi in parts]
        # range j: keys >= bounds[j-1] and < bounds[j] from every slice
        sizes = [sum(int((np.r_[c, hi][j]) - (np.r_[lo, c][j])) for c, (lo, hi) in zip(cuts, parts))
                 for j in range(P)]
        starts = np.concatenate([[0], np.cumsum(sizes)])
        order = np.empty(m, np.int64)

        def merge(j):
            pieces = [keys[(np.r_[lo, c][j]):(np.r_[c, hi][j])] for c, (lo, hi) in zip(cuts, parts)]
            r = np.concatenate(pieces) if pieces else np.empty(0, np.uint64)
            r.sort()
            order[starts[j]:starts[j + 1]] = (r & np.uint64(0xFFFFFFFF)).astype(np.int64)

        list(ex.map(merge, range(P)))
    return order


def _gather(x, order, threads):
    out = np.empty(order.size, x.dtype)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda c: np.take(x, order[c[0]:c[1]], out=out[c[0]:c[1]]), _chunks(order.size, threads)))
    return out


def sort_by_departure(n, src, dst, t, lam, threads: int | None = None) -> SortedEdges:
    """Sort edges by departure time (§2.1 data model; a = t + lambda)."""
    t = np.asarray(t, np.uint32)
    a64 = t.astype(np.uint64) + np.asarray(lam, np.uint64)
    if a64.size and int(a64.max()) > 0xFFFFFFFE:
        raise ValueError("t + lambda exceeds the largest finite time")
    a = a64.astype(np.uint32)
    del a64
    P = threads or _threads()
    order = departure_order(t, P)
    return SortedEdges(n, _gather(np.asarray(src, np.uint32), order, P),
                       _gather(np.asarray(dst, np.uint32), order, P), _gather(t, order, P),
                       _gather(a, order, P))


def earliest_arrival(se: SortedEdges, source: int, t_alpha: int, t_omega: int,
                     return_examined: bool = False):
    """EA from ``source`` within [t_alpha, t_omega] (Alg. 2's output t[V],
    computed by the one-pass scan in departure order)."""
    arr = np.empty(se.n, np.uint32)
    ex = _lib().oracle_earliest_arrival(se.m, _ptr(se.src), _ptr(se.dst), _ptr(se.t), _ptr(se.a),
                                        se.n, int(source), int(t_alpha), int(t_omega), _ptr(arr))
    return (arr, int(ex)) if return_examined else arr


def traversed_edges(se: SortedEdges, t_alpha: int, t_omega: int, arr: np.ndarray) -> int:
    """Number of temporal edges a query traverses: tail reached, departure in
    [max(EA[tail], t_alpha), t_omega) and arrival <= t_omega."""
    arr = np.ascontiguousarray(arr, np.uint32)
    return int(_lib().oracle_traversed_edges(se.m, _ptr(se.src), _ptr(se.t), _ptr(se.a),
                                             int(t_alpha), int(t_omega), _ptr(arr)))


def profile(se: SortedEdges, source: int, t_alpha: int, t_omega: int):
    """(EA, LD, F) by per-vertex Pareto profiles of (arrival, departure)."""
    ea = np.empty(se.n, np.uint32)
    ld = np.empty(se.n, np.uint32)
    fa = np.empty(se.n, np.uint32)
    rc = _lib().oracle_profile(se.m, _ptr(se.src), _ptr(se.dst), _ptr(se.t), _ptr(se.a), se.n,
                               int(source), int(t_alpha), int(t_omega), _ptr(ea), _ptr(ld), _ptr(fa))
    if rc != 0:
        raise MemoryError("oracle_profile")
    return ea, ld, fa


def shortest_duration(se: SortedEdges, source: int, t_alpha: int, t_omega: int,
                      strict: bool = False) -> np.ndarray:
    """SD[v]: least total duration (sum of lambda) of a time-respecting path
    from ``source`` to v within [t_alpha, t_omega] (Table 4's shortest
    duration), by per-vertex Pareto profiles of (arrival, duration).
    ``strict``: consecutive edges follow "Strictly succeeds" (§2.2)."""
    sd = np.empty(se.n, np.uint32)
    rc = _lib().oracle_shortest_duration(se.m, _ptr(se.src), _ptr(se.dst), _ptr(se.t), _ptr(se.a), se.n,
                                         int(source), int(t_alpha), int(t_omega), 1 if strict else 0, _ptr(sd))
    if rc != 0:
        raise MemoryError("oracle_shortest_duration")
    return sd


def ea_certificate_scan(n, src, dst, t, a, source, t_alpha, t_omega, A) -> bool:
    """``ea_certificate``'s three conditions checked by one C loop over the
    edges (any order; ``a`` = t + lambda as uint32)."""
    arrs = [np.ascontiguousarray(x, np.uint32) for x in (src, dst, t, a)]
    A = np.ascontiguousarray(A, np.uint32)
    if A.shape != (n,):
        return False
    scratch = np.empty(n, np.uint8)
    return bool(_lib().oracle_ea_certificate(arrs[0].size, *[_ptr(x) for x in arrs], int(n), int(source),
                                             int(t_alpha), int(t_omega), _ptr(A), _ptr(scratch)))


def ea_certificate(n, src, dst, t, lam, source, t_alpha, t_omega, A) -> bool:
    """True iff ``A`` is exactly the earliest-arrival array.

    (i)   A[source] == t_alpha;
    (ii)  every finite A[v], v != source, is the arrival of a usable edge
          (u, v, t, a) with A[u] <= t (a witness predecessor);
    (iii) no usable edge with A[u] <= t arrives before A[v].
    (ii) makes A an upper bound walked back along strictly decreasing
    witnesses to the source; (iii) makes it a lower bound by induction along
    any time-respecting path.  Usable: t >= t_alpha and a <= t_omega.
    """
    A = np.asarray(A, np.uint64)
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    t = np.asarray(t, np.uint64)
    a = t + np.asarray(lam, np.uint64)
    if A.shape != (n,) or A[source] != t_alpha:
        return False
    # values of a reached vertex lie in the window
    fin = A != INF
    if np.any(A[fin] < t_alpha) or np.any(A[fin] > t_omega):
        return False
    ok = (t >= t_alpha) & (a <= t_omega) & (A[src] != INF) & (A[src] <= t)
    # (iii)
    if np.any(a[ok] < A[dst[ok]]):
        return False
    # (ii)
    witnessed = np.zeros(n, bool)
    w = ok & (a == A[dst])
    witnessed[dst[w]] = True
    need = fin.copy()
    need[source] = False
    return bool(np.all(witnessed[need]))


def brute_force(n, edges, source, t_alpha, t_omega):
    """Enumerate every time-respecting walk from ``source`` (tiny inputs).

    ``edges`` is a list of (u, v, t, lam).  Returns (EA, LD, F) as lists
    following the definitions of temporal minimal paths (§2.3)."""
    ea = [INF] * n
    ld = [INF] * n
    fa = [INF] * n
    out = [[] for _ in range(n)]
    for (u, v, t, lam) in edges:
        if t >= t_alpha and t + lam <= t_omega:
            out[u].append((v, t, t + lam))

    def walk(u, now, dep):
        for (v, t, a) in out[u]:
            if t < now:
                continue
            d = t if dep is None else dep
            if ea[v] == INF or a < ea[v]:
                ea[v] = a
            if ld[v] == INF or d > ld[v]:
                ld[v] = d
            if fa[v] == INF or a - d < fa[v]:
                fa[v] = a - d
            walk(v, a, d)

    walk(source, t_alpha, None)
    ea[source] = t_alpha
    ld[source] = t_omega
    fa[source] = 0
    return ea, ld, fa


def walk_facts(n, edges, source, t_alpha, t_omega, strict=False):
    """Enumerate every time-respecting walk from ``source`` (tiny inputs).

    ``edges`` is a list of (u, v, t, lam).  Returns (used, sd): the set of
    indices of the edges that lie on at least one walk, and per vertex the
    least total duration (sum of lambda) of a walk reaching it (0 for the
    source, INF if none).  ``strict``: consecutive edges follow "Strictly
    succeeds" (§2.2); the first edge needs only t >= t_alpha."""
    sd = [INF] * n
    used = set()
    out = [[] for _ in range(n)]
    for i, (u, v, t, lam) in enumerate(edges):
        if t >= t_alpha and t + lam <= t_omega:
            out[u].append((i, v, t, t + lam, lam))

    def walk(u, now, total, first):
        for (i, v, t, a, lam) in out[u]:
            if t < now or (strict and not first and t == now):
                continue
            used.add(i)
            if total + lam < sd[v]:
                sd[v] = total + lam
            walk(v, a, total + lam, False)

    walk(source, t_alpha, 0, True)
    sd[source] = 0
    return used, sd


def temporal_csr(n, src, dst, t, lam):
    """Expected temporal CSR (§4.2): out-edges grouped by tail and ordered by
    (tail, t, a, head); in-edges grouped by head and ordered by
    (head, a, t, tail).  Returns dict of uint32 arrays (offsets uint64)."""
    src = np.asarray(src, np.uint32)
    dst = np.asarray(dst, np.uint32)
    t = np.asarray(t, np.uint32)
    a = (t.astype(np.uint64) + np.asarray(lam, np.uint64)).astype(np.uint32)
    o = np.lexsort((dst, a, t, src))
    i = np.lexsort((src, t, a, dst))
    off_out = np.zeros(n + 1, np.uint64)
    off_in = np.zeros(n + 1, np.uint64)
    np.cumsum(np.bincount(src, minlength=n), out=off_out[1:])
    np.cumsum(np.bincount(dst, minlength=n), out=off_in[1:])
    return dict(off_out=off_out, dst_out=dst[o], t_out=t[o], a_out=a[o],
                off_in=off_in, src_in=src[i], t_in=t[i], a_in=a[i])
