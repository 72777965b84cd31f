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
* ``ea_certificate``         -- O(m) check that an array is exactly EA.
* ``brute_force``            -- enumeration of all time-respecting walks
                                (pure Python, tiny inputs only).
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


def sort_by_departure(n, src, dst, t, lam) -> SortedEdges:
    """Sort edges by departure time (§2.1 data model; a = t + lambda)."""
    t = np.asarray(t, np.uint32)
    a64 = t.astype(np.uint64) + np.asarray(lam, np.uint64)
    if a64.size and int(a64.max()) > 0xFFFFFFFE:
        raise ValueError("t + lambda exceeds the largest finite time")
    order = np.argsort(t, kind="stable")
    return SortedEdges(n, np.asarray(src, np.uint32)[order], np.asarray(dst, np.uint32)[order],
                       t[order], a64[order].astype(np.uint32))


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
