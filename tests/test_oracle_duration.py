"""Pins for the oracle's traversed-edge count, its shortest-duration scan,
its C earliest-arrival certificate and its parallel departure sort, each
against something other than the oracle itself: enumeration of every
time-respecting walk, hand-worked cases, scipy shortest paths on
time-replicated static graphs, the numpy certificate, numpy's stable sort,
and planted mutations of the C source that these pins must catch."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle as O
from workloads import make_graph, make_queries, tiny_graph

INF = O.INF


def arrays(edges):
    src = np.array([e[0] for e in edges], np.uint32)
    dst = np.array([e[1] for e in edges], np.uint32)
    t = np.array([e[2] for e in edges], np.uint32)
    lam = np.array([e[3] for e in edges], np.uint32)
    return src, dst, t, lam


@st.composite
def tiny_cases(draw):
    n = draw(st.integers(1, 7))
    m = draw(st.integers(0, 10))
    edges = [(draw(st.integers(0, n - 1)), draw(st.integers(0, n - 1)), draw(st.integers(0, 8)),
              draw(st.integers(1, 3))) for _ in range(m)]
    s = draw(st.integers(0, n - 1))
    ta = draw(st.integers(0, 9))
    tw = draw(st.integers(ta, 13))
    return n, edges, s, ta, tw


@settings(max_examples=1500, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_cases())
def test_walk_enumeration_pins_traversed_edges_and_duration(case):
    """The traversed-edge count is the number of distinct edges lying on at
    least one time-respecting walk from the source (an edge lies on one iff
    its tail can be reached by its departure); the shortest duration is the
    least sum of lambda over the walks reaching a vertex."""
    n, edges, s, ta, tw = case
    used, bsd = O.walk_facts(n, edges, s, ta, tw)
    src, dst, t, lam = arrays(edges)
    se = O.sort_by_departure(n, src, dst, t, lam)
    ea = O.earliest_arrival(se, s, ta, tw)
    assert O.traversed_edges(se, ta, tw, ea) == len(used)
    assert list(O.shortest_duration(se, s, ta, tw)) == bsd
    # "Strictly succeeds" (§2.2): enumeration with departures after arrivals
    _, bsd_strict = O.walk_facts(n, edges, s, ta, tw, strict=True)
    assert list(O.shortest_duration(se, s, ta, tw, strict=True)) == bsd_strict
    # the C certificate accepts exactly what the numpy one accepts
    a = t + lam
    assert O.ea_certificate_scan(n, src, dst, t, a, s, ta, tw, ea)


def test_duration_hand_worked():
    # 0 -(t=0, lam=10)-> 1 arrives at 10; 0 -(0, 1)-> 2 -(20, 1)-> 1 arrives
    # at 21 with total 2.  From 1: an edge at 15 only the direct arrival can
    # take (total 10 + 1), an edge at 25 takes the later, shorter one
    # (2 + 1).  Earliest arrival and fastest follow other paths.
    n = 5
    edges = [(0, 1, 0, 10), (0, 2, 0, 1), (2, 1, 20, 1), (1, 3, 15, 1), (1, 4, 25, 1)]
    src, dst, t, lam = arrays(edges)
    se = O.sort_by_departure(n, src, dst, t, lam)
    assert list(O.shortest_duration(se, 0, 0, 100)) == [0, 2, 1, 11, 3]
    ea = O.earliest_arrival(se, 0, 0, 100)
    assert list(ea) == [0, 10, 1, 16, 26]
    _, ld, fa = O.profile(se, 0, 0, 100)
    assert list(fa) == [0, 10, 1, 16, 26]
    # the window cuts the late, short path: 1 keeps the direct edge only
    assert list(O.shortest_duration(se, 0, 0, 20)) == [0, 10, 1, 11, INF]
    # a walk back into the source never lowers its 0
    se2 = O.sort_by_departure(2, *arrays([(0, 1, 0, 1), (1, 0, 1, 1)]))
    assert list(O.shortest_duration(se2, 0, 0, 9)) == [0, 1]
    # non-strict succession: leaving at the arrival time is allowed
    se3 = O.sort_by_departure(3, *arrays([(0, 1, 0, 2), (1, 2, 2, 3)]))
    assert list(O.shortest_duration(se3, 0, 0, 9)) == [0, 2, 5]
    se4 = O.sort_by_departure(3, *arrays([(0, 1, 0, 2), (1, 2, 1, 3)]))
    assert list(O.shortest_duration(se4, 0, 0, 9)) == [0, 2, INF]
    # empty graph
    se5 = O.sort_by_departure(3, *arrays([]))
    assert list(O.shortest_duration(se5, 1, 0, 9)) == [INF, 0, INF]


@pytest.mark.parametrize("seed", range(6))
def test_duration_scipy_special_case(seed):
    """A static graph replicated at every integer time with lambda = weight:
    the shortest duration is the static shortest-path distance (scipy
    dijkstra), as long as the window holds it."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    rng = np.random.default_rng(100 + seed)
    n, k = 12, 26
    best = {}
    for u, v, w in zip(rng.integers(0, n, k), rng.integers(0, n, k), rng.integers(1, 4, k)):
        if u != v:
            best[(int(u), int(v))] = min(best.get((int(u), int(v)), 99), int(w))
    static = [(u, v, w) for (u, v), w in best.items()]
    ta, tw = 2, 2 + 9
    edges = [(u, v, tt, w) for (u, v, w) in static for tt in range(tw + 1)]
    s = int(rng.integers(0, n))
    M = csr_matrix(([w for *_, w in static], ([u for u, *_ in static], [v for _, v, _ in static])), shape=(n, n))
    dist = dijkstra(M, indices=s)
    se = O.sort_by_departure(n, *arrays(edges))
    sd = O.shortest_duration(se, s, ta, tw)
    for v in range(n):
        if np.isfinite(dist[v]) and dist[v] <= tw - ta:
            assert sd[v] == int(dist[v]), v
        else:
            assert sd[v] == INF, v


@pytest.mark.parametrize("seed", range(8))
def test_duration_invariants_on_generated_graphs(seed):
    """On larger graphs: reached exactly where earliest arrival is finite,
    never above the fastest duration (a path's total duration is at most its
    arrival minus its departure), at least the lightest usable in-edge, and
    monotone in the window."""
    g = tiny_graph(seed, n=60, m=900, t_max=300, lam_max=9)
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    s = int(g.src[seed])
    ta, tw = 20, 280
    sd = O.shortest_duration(se, s, ta, tw).astype(np.int64)
    ea, ld, fa = O.profile(se, s, ta, tw)
    assert np.array_equal(sd != INF, ea != INF)
    fin = sd != INF
    assert np.all(sd[fin] <= fa[fin].astype(np.int64))
    minin = np.full(g.n, INF, np.int64)
    ok = (g.t >= ta) & (g.t.astype(np.int64) + g.lam <= tw)
    np.minimum.at(minin, g.dst[ok].astype(np.int64), g.lam[ok].astype(np.int64))
    fin[s] = False
    assert np.all(sd[fin] >= minin[fin])
    narrow = O.shortest_duration(se, s, ta + 30, tw - 30).astype(np.int64)
    assert np.all(narrow >= sd)


def test_certificate_scan_matches_numpy_certificate():
    g = make_graph("uniform-10k")
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    srcs, ta, tw = make_queries("uniform-10k", g)
    a = g.t + g.lam
    rng = np.random.default_rng(7)
    for q in range(3):
        s, w0, w1 = int(srcs[q]), int(ta[q]), int(tw[q])
        ea = O.earliest_arrival(se, s, w0, w1)
        assert O.ea_certificate_scan(g.n, g.src, g.dst, g.t, a, s, w0, w1, ea)
        fin = np.nonzero((ea != INF) & (np.arange(g.n) != s))[0]
        for kind in range(5):
            bad = ea.copy()
            v = int(rng.choice(fin))
            if kind == 0:
                bad[v] -= 1            # below the true arrival: no witness
            elif kind == 1:
                bad[v] += 1            # above it: an edge undercuts it
            elif kind == 2:
                bad[v] = INF           # a reached vertex dropped
            elif kind == 3:
                bad[s] = w0 + 1        # wrong source start
            else:
                bad[int(np.nonzero(ea == INF)[0][0])] = w1  # a spurious arrival
            want = O.ea_certificate(g.n, g.src, g.dst, g.t, g.lam, s, w0, w1, bad)
            assert not want
            assert O.ea_certificate_scan(g.n, g.src, g.dst, g.t, a, s, w0, w1, bad) == want


def test_departure_order_is_the_stable_sort():
    rng = np.random.default_rng(3)
    for m, hi in ((0, 5), (7, 3), (5_000_000, 1000), (6_000_001, 0xFFFFFFFE), (4_194_304, 1)):
        t = rng.integers(0, hi, size=m, endpoint=True, dtype=np.uint64).astype(np.uint32)
        for threads in (1, 3, 8):
            assert np.array_equal(O.departure_order(t, threads), np.argsort(t, kind="stable")), (m, hi, threads)


MUTANTS = [  # (original text, planted text, harmless?)
    ("if (t[e] >= lo && a[e] <= t_omega)", "if (t[e] > lo && a[e] <= t_omega)", False),
    ("if (t[e] >= lo && a[e] <= t_omega)", "if (t[e] >= lo && a[e] < t_omega)", False),
    # an unreached tail's INF already fails t >= lo, so the test is redundant
    ("if (r == ORACLE_INF)\n            continue;", "if (0)\n            continue;", True),
    # reached tails always have arr >= t_alpha, so the max is redundant
    ("uint32_t lo = r > t_alpha ? r : t_alpha;", "uint32_t lo = r;", True),
    ("if (t[e] >= lo && a[e] <= t_omega)", "if (t[e] >= t_alpha && a[e] <= t_omega)", False),
    ("d = P[u].dur[k] + lam;", "d = P[u].dur[0] + lam;", False),
    ("dprofile_last_by(&P[u], strict ? t[e] - 1 : t[e]);", "dprofile_last_by(&P[u], t[e] - 1);", False),
    # strict succession read as the non-strict one: only the strict pin sees it
    ("dprofile_last_by(&P[u], strict ? t[e] - 1 : t[e]);", "dprofile_last_by(&P[u], t[e]);", False),
    ("if (strict && t[e] == 0)\n                continue;", "if (0)\n                continue;", False),
    ("            d = lam;\n", "            d = 0;\n", False),
    ("s_v = P[v].dur[P[v].len - 1];", "s_v = P[v].dur[0];", False),
    ("if (k >= 0 && p->dur[k] <= d)", "if (k >= 0 && p->dur[k] < d)", True),
    ("while (last < p->len && p->dur[last] >= d)", "while (last < p->len && p->dur[last] > d)", True),
    ("if (a[e] > t_omega || v == source)\n            continue;\n        uint32_t lam",
     "if (v == source)\n            continue;\n        uint32_t lam", False),
]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_planted_mutations_are_caught(tmp_path):
    """Each planted mistake in a copy of the C oracle's traversed-edge count
    or shortest-duration scan must fail the walk-enumeration pin; the
    harmless rewrites (a redundant bound, tie handling that keeps the same
    minimum) must not."""
    src_c = open(os.path.join(os.path.dirname(O.__file__), "kairos_oracle.c")).read()
    rng = np.random.default_rng(11)
    # the hand-worked case above first, then drawn ones
    cases = [(5, [(0, 1, 0, 10), (0, 2, 0, 1), (2, 1, 20, 1), (1, 3, 15, 1), (1, 4, 25, 1)], 0, 0, 100),
             # departures at time 0 after an arrival listed first: under strict
             # succession nothing arrives before 0
             (3, [(0, 1, 0, 1), (1, 2, 0, 1)], 0, 0, 10)]
    for _ in range(600):
        n = int(rng.integers(1, 7))
        m = int(rng.integers(0, 12))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n)), int(rng.integers(0, 10)),
                  int(rng.integers(1, 6))) for _ in range(m)]
        ta = int(rng.integers(0, 6))
        cases.append((n, edges, int(rng.integers(0, n)), ta, int(rng.integers(ta, 16))))
    for i, (old, new, harmless) in enumerate(MUTANTS):
        assert old in src_c, old
        cpath = tmp_path / f"m{i}.c"
        lpath = tmp_path / f"m{i}.so"
        cpath.write_text(src_c.replace(old, new, 1))
        subprocess.run(["gcc", "-O1", "-shared", "-fPIC", str(cpath), "-o", str(lpath)], check=True)
        lib = ctypes.CDLL(str(lpath))
        u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        lib.oracle_traversed_edges.restype = u64
        lib.oracle_traversed_edges.argtypes = [u64, p, p, p, u32, u32, p]
        lib.oracle_shortest_duration.argtypes = [u64, p, p, p, p, u32, u32, u32, u32, ctypes.c_int, p]
        caught = False
        for (n, edges, s, ta, tw) in cases:
            se = O.sort_by_departure(n, *arrays(edges))
            ea = O.earliest_arrival(se, s, ta, tw)
            used, bsd = O.walk_facts(n, edges, s, ta, tw)
            cnt = lib.oracle_traversed_edges(se.m, O._ptr(se.src), O._ptr(se.t), O._ptr(se.a), ta, tw, O._ptr(ea))
            sd = np.empty(n, np.uint32)
            lib.oracle_shortest_duration(se.m, O._ptr(se.src), O._ptr(se.dst), O._ptr(se.t), O._ptr(se.a),
                                         n, s, ta, tw, 0, O._ptr(sd))
            _, bsd_strict = O.walk_facts(n, edges, s, ta, tw, strict=True)
            sds = np.empty(n, np.uint32)
            lib.oracle_shortest_duration(se.m, O._ptr(se.src), O._ptr(se.dst), O._ptr(se.t), O._ptr(se.a),
                                         n, s, ta, tw, 1, O._ptr(sds))
            if cnt != len(used) or list(sd) != bsd or list(sds) != bsd_strict:
                caught = True
                break
        assert caught != harmless, (old, new, caught)
