"""Pins for the CPU oracle, each against something other than the oracle
itself: exhaustive enumeration, hand-worked cases, scipy shortest paths on
time-replicated static graphs, the O(m) EA certificate, cross-routes between
independent oracle routines, metamorphic relations, and planted mutations
of the oracle source that these pins must catch."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle as O
from workloads import tiny_graph, make_graph, make_queries

INF = O.INF


def run_all(n, edges, s, ta, tw):
    src = np.array([e[0] for e in edges], np.uint32)
    dst = np.array([e[1] for e in edges], np.uint32)
    t = np.array([e[2] for e in edges], np.uint32)
    lam = np.array([e[3] for e in edges], np.uint32)
    se = O.sort_by_departure(n, src, dst, t, lam)
    ea = O.earliest_arrival(se, s, ta, tw)
    pea, pld, pf = O.profile(se, s, ta, tw)
    return (src, dst, t, lam, se), ea, pea, pld, pf


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
def test_brute_force_matches_scan_and_profile(case):
    n, edges, s, ta, tw = case
    bea, bld, bf = O.brute_force(n, edges, s, ta, tw)
    (src, dst, t, lam, se), ea, pea, pld, pf = run_all(n, edges, s, ta, tw)
    assert list(ea) == bea
    assert list(pea) == bea
    assert list(pld) == bld
    assert list(pf) == bf
    assert O.ea_certificate(n, src, dst, t, lam, s, ta, tw, ea)


def test_hand_worked_cases(oracle_mod):
    # 0 -(t=1,a=9)-> 2 directly, and 0 -(1,2)-> 1 -(3,4)-> 2 over two hops.
    # The two-hop path reaches 2 at 4; a visit-once traversal that admits 2
    # from the first round keeps 9.  Window [0, 20].
    n, edges = 3, [(0, 2, 1, 8), (0, 1, 1, 1), (1, 2, 3, 1)]
    _, ea, pea, pld, pf = run_all(n, edges, 0, 0, 20)
    assert list(ea) == [0, 2, 4]
    assert list(pld) == [20, 1, 1]
    assert list(pf) == [0, 1, 3]
    # non-strict succession: 1 is reached at 2 and an edge departs 1 at 2
    _, ea, *_ = run_all(3, [(0, 1, 0, 2), (1, 2, 2, 1)], 0, 0, 10)
    assert list(ea) == [0, 2, 3]
    # departure one unit before arrival is not usable
    _, ea, *_ = run_all(3, [(0, 1, 0, 2), (1, 2, 1, 1)], 0, 0, 10)
    assert list(ea) == [0, 2, INF]
    # closed window: arrival exactly t_omega is kept, one past it is not
    _, ea, *_ = run_all(3, [(0, 1, 0, 5), (0, 2, 0, 6)], 0, 0, 5)
    assert list(ea) == [0, 5, INF]
    # departure exactly t_alpha is kept, one before it is not
    _, ea, *_ = run_all(3, [(0, 1, 3, 1), (0, 2, 2, 1)], 0, 3, 10)
    assert list(ea) == [3, 4, INF]
    # fastest may use a later departure than the earliest arrival path:
    # leave at 0 arrive 10 (duration 10) vs leave at 7 arrive 11 (duration 4)
    _, ea, pea, pld, pf = run_all(2, [(0, 1, 0, 10), (0, 1, 7, 4)], 0, 0, 20)
    assert list(ea) == [0, 10] and list(pld) == [20, 7] and list(pf) == [0, 4]
    # self-loop and empty graph
    _, ea, *_ = run_all(2, [(0, 0, 0, 1)], 0, 0, 10)
    assert list(ea) == [0, INF]
    _, ea, pea, pld, pf = run_all(4, [], 2, 5, 9)
    assert list(ea) == [INF, INF, 5, INF] and list(pld) == [INF, INF, 9, INF]
    assert list(pf) == [INF, INF, 0, INF]


def _replicated(static_edges, L):
    out = []
    for (u, v, w) in static_edges:
        for tt in range(L):
            out.append((u, v, tt, w))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_scipy_special_case(seed, oracle_mod):
    """Static graph replicated at every integer time: EA = t_alpha + dist,
    F = dist, LD = t_omega - dist (scipy dijkstra; w = 1 is BFS)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    rng = np.random.default_rng(seed)
    n = 12
    k = 26
    us = rng.integers(0, n, k)
    vs = rng.integers(0, n, k)
    ws = rng.integers(1, 4, k) if seed % 2 else np.ones(k, int)
    # keep the lightest parallel edge for scipy (it sums duplicates)
    best = {}
    for u, v, w in zip(us, vs, ws):
        if u != v:
            best[(u, v)] = min(best.get((u, v), 99), int(w))
    static = [(u, v, w) for (u, v), w in best.items()]
    ta, tw = 3, 3 + 9
    L = tw + 1
    s = int(rng.integers(0, n))
    M = csr_matrix(([w for *_, w in static], ([u for u, *_ in static], [v for _, v, _ in static])),
                   shape=(n, n))
    dist = dijkstra(M, indices=s)
    _, ea, pea, pld, pf = run_all(n, _replicated(static, L), s, ta, tw)
    for v in range(n):
        if v == s:
            assert (ea[v], pld[v], pf[v]) == (ta, tw, 0)
        elif np.isfinite(dist[v]) and dist[v] <= tw - ta:
            d = int(dist[v])
            assert ea[v] == ta + d and pea[v] == ta + d
            assert pf[v] == d
            assert pld[v] == tw - d
        else:
            assert ea[v] == INF and pld[v] == INF and pf[v] == INF


@pytest.mark.parametrize("seed", range(40))
def test_cross_route_profile_vs_repeated_scans(seed, oracle_mod):
    """LD[v] = max{s in S : EA_s[v] finite}; F[v] = min_s EA_s[v] - s, with
    S the departure times of the source's usable out-edges and EA_s the
    one-pass scan over the window [s, t_omega]."""
    g = tiny_graph(seed, n=30, m=200, t_max=60, lam_max=6)
    s = int(g.src[seed % g.m])
    ta, tw = 5, 55
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    pea, pld, pf = O.profile(se, s, ta, tw)
    ea = O.earliest_arrival(se, s, ta, tw)
    assert np.array_equal(pea, ea)
    a = g.t.astype(np.int64) + g.lam
    S = sorted({int(x) for x in g.t[(g.src == s) & (g.t >= ta) & (a <= tw)]}, reverse=True)
    ld = np.full(g.n, INF, np.uint64)
    fa = np.full(g.n, INF, np.uint64)
    for sd in S:
        e = O.earliest_arrival(se, s, sd, tw).astype(np.uint64)
        fin = e != INF
        ld[fin & (ld == INF)] = sd
        fa[fin] = np.minimum(fa[fin], e[fin] - sd)
    ld[s], fa[s] = tw, 0
    assert np.array_equal(ld, pld.astype(np.uint64))
    assert np.array_equal(fa, pf.astype(np.uint64))


def test_certificate_rejects_perturbations(oracle_mod):
    g = tiny_graph(7, n=600, m=1500, t_max=500, lam_max=10)
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    s, ta, tw = int(g.src[0]), 10, 480
    ea = O.earliest_arrival(se, s, ta, tw)
    args = (g.n, g.src, g.dst, g.t, g.lam, s, ta, tw)
    assert O.ea_certificate(*args, ea)
    reached = [v for v in range(g.n) if ea[v] != INF and v != s]
    unreached = [v for v in range(g.n) if ea[v] == INF]
    assert reached and unreached
    rng = np.random.default_rng(0)
    for v in rng.choice(reached, 10):
        for delta in (-1, +1):
            bad = ea.copy()
            bad[v] = int(ea[v]) + delta
            assert not O.ea_certificate(*args, bad)
        bad = ea.copy()
        bad[v] = INF
        assert not O.ea_certificate(*args, bad)
    for v in rng.choice(unreached, min(5, len(unreached))):
        bad = ea.copy()
        bad[v] = tw
        assert not O.ea_certificate(*args, bad)
    bad = ea.copy()
    bad[s] = ta + 1
    assert not O.ea_certificate(*args, bad)


@pytest.mark.parametrize("seed", range(8))
def test_metamorphic(seed, oracle_mod):
    g = tiny_graph(100 + seed, n=60, m=600, t_max=300, lam_max=8)
    s = int(g.src[0])
    ta, tw = 20, 280
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    ea = O.earliest_arrival(se, s, ta, tw).astype(np.int64)
    ea[ea == INF] = 1 << 40
    # shrinking the window never lowers an arrival
    for (a2, w2) in [(ta + 30, tw), (ta, tw - 60), (ta + 10, tw - 10)]:
        e2 = O.earliest_arrival(se, s, a2, w2).astype(np.int64)
        e2[e2 == INF] = 1 << 40
        mask = np.arange(g.n) != s
        assert np.all(e2[mask] >= ea[mask])
    # adding edges never raises an arrival
    g2 = tiny_graph(900 + seed, n=60, m=200, t_max=300, lam_max=8)
    se3 = O.sort_by_departure(g.n, np.r_[g.src, g2.src], np.r_[g.dst, g2.dst], np.r_[g.t, g2.t],
                              np.r_[g.lam, g2.lam])
    e3 = O.earliest_arrival(se3, s, ta, tw).astype(np.int64)
    e3[e3 == INF] = 1 << 40
    assert np.all(e3 <= ea)
    # input order does not matter
    p = np.random.default_rng(seed).permutation(g.m)
    sep = O.sort_by_departure(g.n, g.src[p], g.dst[p], g.t[p], g.lam[p])
    assert np.array_equal(O.profile(sep, s, ta, tw)[1], O.profile(se, s, ta, tw)[1])
    assert np.array_equal(O.earliest_arrival(sep, s, ta, tw), O.earliest_arrival(se, s, ta, tw))
    # relabelling vertices permutes the output
    rl = np.random.default_rng(seed + 1).permutation(g.n).astype(np.uint32)
    ser = O.sort_by_departure(g.n, rl[g.src], rl[g.dst], g.t, g.lam)
    for base, rel in zip(O.profile(se, s, ta, tw), O.profile(ser, int(rl[s]), ta, tw)):
        assert np.array_equal(rel[rl], base)
    # shifting every time by c: EA + c, LD + c, F unchanged
    c = 1000
    ses = O.sort_by_departure(g.n, g.src, g.dst, g.t + c, g.lam)
    b_ea, b_ld, b_f = O.profile(se, s, ta, tw)
    s_ea, s_ld, s_f = O.profile(ses, s, ta + c, tw + c)
    fin = b_ea != INF
    assert np.array_equal(s_ea[fin], b_ea[fin] + c) and np.all(s_ea[~fin] == INF)
    assert np.array_equal(s_ld[fin], b_ld[fin] + c)
    assert np.array_equal(s_f, b_f)


def test_traversed_edges_definition(oracle_mod):
    g = tiny_graph(3, n=40, m=400, t_max=100, lam_max=5)
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    s, ta, tw = int(g.src[1]), 10, 90
    ea = O.earliest_arrival(se, s, ta, tw)
    want = 0
    for u, t, lam in zip(g.src, g.t, g.lam):
        r = int(ea[u])
        if r != INF and t >= max(r, ta) and t + lam <= tw:
            want += 1
    assert O.traversed_edges(se, ta, tw, ea) == want
    assert want > 0


def test_temporal_csr_reference(oracle_mod):
    g = tiny_graph(5, n=9, m=60, t_max=6, lam_max=2)
    ix = O.temporal_csr(g.n, g.src, g.dst, g.t, g.lam)
    a = [int(x) + int(y) for x, y in zip(g.t, g.lam)]
    rows = sorted(zip(g.src.tolist(), g.t.tolist(), a, g.dst.tolist()))
    assert ix["dst_out"].tolist() == [r[3] for r in rows]
    assert ix["t_out"].tolist() == [r[1] for r in rows]
    assert ix["a_out"].tolist() == [r[2] for r in rows]
    rows = sorted(zip(g.dst.tolist(), a, g.t.tolist(), g.src.tolist()))
    assert ix["src_in"].tolist() == [r[3] for r in rows]
    assert ix["a_in"].tolist() == [r[1] for r in rows]
    for v in range(g.n):
        assert ix["off_out"][v + 1] - ix["off_out"][v] == int((g.src == v).sum())
        assert ix["off_in"][v + 1] - ix["off_in"][v] == int((g.dst == v).sum())


def test_certificate_on_generated_workload(oracle_mod):
    g = make_graph("uniform-10k")
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    srcs, ta, tw = make_queries("uniform-10k", g)
    for q in range(4):
        ea = O.earliest_arrival(se, srcs[q], ta[q], tw[q])
        assert O.ea_certificate(g.n, g.src, g.dst, g.t, g.lam, int(srcs[q]), int(ta[q]), int(tw[q]), ea)
        pea, pld, pf = O.profile(se, srcs[q], ta[q], tw[q])
        assert np.array_equal(pea, ea)
        fin = ea != INF
        fin[srcs[q]] = False
        assert np.all(pld[fin] >= ta[q]) and np.all(pld[fin] < tw[q])
        assert np.all(pf[fin] >= 1) and np.all(pf[fin] <= ea[fin] - ta[q])
        assert np.array_equal(pld != INF, ea != INF) and np.array_equal(pf != INF, ea != INF)


MUTANTS = [  # (original text, planted text, harmless?)
    ("arr[u] <= t[e]", "arr[u] < t[e]", False),                       # strict succession
    ("a[e] <= t_omega && arr[u]", "a[e] < t_omega && arr[u]", False),  # open window end
    ("a[e] <= t_omega && arr[u]", "arr[u]", False),                     # arrival bound dropped
    ("arr[source] = t_alpha;", "arr[source] = 0;", False),             # wrong source start
    ("a[e] < arr[v])", "a[e] <= arr[v] && v != u)", True),             # equivalent rewrite
    ("s = profile_best_by(&P[u], t[e]);", "s = profile_best_by(&P[u], t[e] - 1);", False),
    ("if (d < f_v)", "if (d > f_v || f_v == ORACLE_INF)", False),
    ("e_v = P[v].arr[0];", "e_v = P[v].arr[P[v].len - 1];", False),
    ("l_v = P[v].dep[P[v].len - 1];", "l_v = P[v].dep[0];", False),
]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_planted_mutations_are_caught(tmp_path, oracle_mod):
    """Each planted mistake in a copy of the C oracle must fail a pin
    (brute force on tiny graphs); the one harmless rewrite must not."""
    import ctypes
    src_c = open(os.path.join(os.path.dirname(O.__file__), "kairos_oracle.c")).read()
    rng = np.random.default_rng(1)
    cases = []
    for _ in range(400):
        n = int(rng.integers(1, 7))
        m = int(rng.integers(0, 10))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n)), int(rng.integers(0, 8)),
                  int(rng.integers(1, 4))) for _ in range(m)]
        ta = int(rng.integers(0, 6))
        cases.append((n, edges, int(rng.integers(0, n)), ta, int(rng.integers(ta, 12))))
    for i, (old, new, harmless) in enumerate(MUTANTS):
        assert old in src_c, old
        cpath = tmp_path / f"m{i}.c"
        lpath = tmp_path / f"m{i}.so"
        cpath.write_text(src_c.replace(old, new, 1))
        subprocess.run(["gcc", "-O1", "-shared", "-fPIC", str(cpath), "-o", str(lpath)], check=True)
        lib = ctypes.CDLL(str(lpath))
        u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        lib.oracle_earliest_arrival.argtypes = [u64, p, p, p, p, u32, u32, u32, u32, p]
        lib.oracle_profile.argtypes = [u64, p, p, p, p, u32, u32, u32, u32, p, p, p]
        caught = False
        for (n, edges, s, ta, tw) in cases:
            (src, dst, t, lam, se), *_ = run_all(n, edges, s, ta, tw)
            ea = np.empty(n, np.uint32)
            lib.oracle_earliest_arrival(se.m, O._ptr(se.src), O._ptr(se.dst), O._ptr(se.t),
                                        O._ptr(se.a), n, s, ta, tw, O._ptr(ea))
            pe, pl, pf = (np.empty(n, np.uint32) for _ in range(3))
            lib.oracle_profile(se.m, O._ptr(se.src), O._ptr(se.dst), O._ptr(se.t), O._ptr(se.a),
                               n, s, ta, tw, O._ptr(pe), O._ptr(pl), O._ptr(pf))
            b = O.brute_force(n, edges, s, ta, tw)
            if list(ea) != b[0] or list(pe) != b[0] or list(pl) != b[1] or list(pf) != b[2]:
                caught = True
                break
        assert caught != harmless, (old, new, caught)
