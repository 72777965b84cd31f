"""Pins for the path oracles (``oracle.paths``): earliest-arrival
predecessors and temporal BFS hop counts, each against exhaustive walk
enumeration, hand-worked cases and a library routine on a special case."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle as O
from oracle import paths as P

INF = O.INF


def arrays(edges):
    cols = list(zip(*edges)) if edges else [(), (), (), ()]
    return [np.array(c, np.uint32) for c in cols]


@st.composite
def tiny_cases(draw):
    n = draw(st.integers(1, 7))
    m = draw(st.integers(0, 12))
    edges = [(draw(st.integers(0, n - 1)), draw(st.integers(0, n - 1)), draw(st.integers(0, 8)),
              draw(st.integers(1, 3))) for _ in range(m)]
    s = draw(st.integers(0, n - 1))
    ta = draw(st.integers(0, 9))
    tw = draw(st.integers(ta, 13))
    return n, edges, s, ta, tw


def rule_pick(pairs):
    """The documented choice among optimal last edges: latest departure,
    then smallest tail."""
    if not pairs:
        return INF, INF
    best_t = max(t for _, t in pairs)
    return min(u for u, t in pairs if t == best_t), best_t


@settings(max_examples=1500, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_cases())
def test_predecessors_and_hops_match_enumeration(case):
    n, edges, s, ta, tw = case
    bea, last, bhops, _, _ = P.brute_force_walks(n, edges, s, ta, tw)
    src, dst, t, lam = arrays(edges)
    se = O.sort_by_departure(n, src, dst, t, lam)
    ea = O.earliest_arrival(se, s, ta, tw)
    assert list(ea) == bea
    pt, pd = P.ea_predecessors(n, src, dst, t, lam, s, ta, tw, ea)
    for v in range(n):
        assert (int(pt[v]), int(pd[v])) == rule_pick(last[v]), v
    hops, hea = P.min_hops(n, src, dst, t, lam, s, ta, tw)
    assert list(hops) == bhops
    assert list(hea) == bea


def test_hand_worked():
    # 0 -(t=1,a=9)-> 2 directly; 0 -(1,2)-> 1 -(3,4)-> 2.  Window [0, 20].
    # EA[2] = 4 over two edges, but 2 is one edge away: hops and the
    # earliest-arrival path length differ.
    n, edges = 3, [(0, 2, 1, 8), (0, 1, 1, 1), (1, 2, 3, 1)]
    src, dst, t, lam = arrays(edges)
    ea = np.array([0, 2, 4], np.uint32)
    pt, pd = P.ea_predecessors(n, src, dst, t, lam, 0, 0, 20, ea)
    assert pt.tolist() == [INF, 0, 1] and pd.tolist() == [INF, 1, 3]
    hops, hea = P.min_hops(n, src, dst, t, lam, 0, 0, 20)
    assert hops.tolist() == [0, 1, 1] and hea.tolist() == [0, 2, 4]
    # window ending at 8: the direct edge (arrival 9) is no longer usable
    hops, hea = P.min_hops(n, src, dst, t, lam, 0, 0, 8)
    assert hops.tolist() == [0, 1, 2] and hea.tolist() == [0, 2, 4]


def test_predecessor_tie_rule():
    # three optimal last edges into 3 (arrival 10): (1, t=7), (2, t=8), (0, t=8);
    # the rule takes departure 8, then tail 0
    n = 4
    edges = [(0, 1, 0, 1), (0, 2, 0, 1), (1, 3, 7, 3), (2, 3, 8, 2), (0, 3, 8, 2), (1, 3, 9, 5)]
    src, dst, t, lam = arrays(edges)
    se = O.sort_by_departure(n, src, dst, t, lam)
    ea = O.earliest_arrival(se, 0, 0, 30)
    assert ea.tolist() == [0, 1, 1, 10]
    pt, pd = P.ea_predecessors(n, src, dst, t, lam, 0, 0, 30, ea)
    assert (int(pt[3]), int(pd[3])) == (0, 8)
    # a tail that is reached too late for its edge is not a predecessor
    edges2 = [(0, 1, 5, 1), (1, 2, 3, 1), (0, 2, 3, 1)]
    src, dst, t, lam = arrays(edges2)
    ea = O.earliest_arrival(O.sort_by_departure(3, src, dst, t, lam), 0, 0, 30)
    pt, pd = P.ea_predecessors(3, src, dst, t, lam, 0, 0, 30, ea)
    assert ea.tolist() == [0, 6, 4] and (int(pt[2]), int(pd[2])) == (0, 3)


@pytest.mark.parametrize("seed", range(4))
def test_hops_equal_bfs_on_replicated_static_graph(seed):
    """A static graph whose edges exist at every integer time with duration
    1: within a long enough window the fewest edges is the BFS distance."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    rng = np.random.default_rng(seed)
    n, me, L = 12, 20, 30
    u = rng.integers(0, n, me)
    v = rng.integers(0, n, me)
    edges = [(int(a), int(b), tt, 1) for a, b in zip(u, v) for tt in range(L)]
    src, dst, t, lam = arrays(edges)
    dist = shortest_path(csr_matrix((np.ones(me), (u, v)), shape=(n, n)), unweighted=True, indices=0)
    hops, hea = P.min_hops(n, src, dst, t, lam, 0, 0, L)
    want = [0 if i == 0 else (INF if not np.isfinite(dist[i]) else int(dist[i])) for i in range(n)]
    assert hops.tolist() == want
    # earliest arrival there is t_alpha + distance
    assert hea.tolist() == [INF if w == INF else w for w in want]


def test_hops_monotone_in_window():
    rng = np.random.default_rng(5)
    n, m = 40, 300
    src = rng.integers(0, n, m).astype(np.uint32)
    dst = rng.integers(0, n, m).astype(np.uint32)
    t = rng.integers(0, 100, m).astype(np.uint32)
    lam = rng.integers(1, 6, m).astype(np.uint32)
    wide, _ = P.min_hops(n, src, dst, t, lam, 3, 0, 120)
    narrow, _ = P.min_hops(n, src, dst, t, lam, 3, 10, 80)
    assert np.all(wide.astype(np.int64) <= narrow.astype(np.int64))


MUTATIONS = [
    ("(E[src] <= t)", "(E[src] < t)"),                                  # strict succession
    ("np.lexsort((src[idx], -t[idx], dst[idx]))", "np.lexsort((src[idx], t[idx], dst[idx]))"),  # earliest departure
    ("np.lexsort((src[idx], -t[idx], dst[idx]))", "np.lexsort((-src[idx], -t[idx], dst[idx]))"),  # largest tail
    ("nxt = cur.copy()\n        np.minimum.at(nxt, dst[ok], a[ok])",
     "nxt = cur\n        np.minimum.at(nxt, dst[ok], a[ok])\n        cur = cur.copy()"),  # same-level chaining
    ("hops[new] = h", "hops[new] = h + 1"),                              # off by one
    ("(a <= t_omega)", "(a < t_omega)"),                                  # open window end
    ("(src == source) | (not strict)", "(not strict)"),                   # strict first edge
    ("cur[src] <= t, cur[src] < t)", "cur[src] <= t, cur[src] <= t)"),    # strictness ignored
    ("ld[r] = s", "ld[r] = np.maximum(ld[r], s)"),                        # INF taken as a departure
    ("into_target | (not strict)", "(not strict)"),                       # strict at the path's end
    ("np.maximum.at(nxt, src[ok], t[ok])", "np.maximum.at(nxt, src[ok], a[ok])"),  # arrival for departure
    ("a <= lv, a < lv)", "a < lv, a < lv)"),                              # strictness everywhere
]


@pytest.mark.parametrize("old,new", MUTATIONS)
def test_planted_mutations_are_caught(old, new):
    """Each plausible slip in the path oracle fails the enumeration pin on a
    fixed sample of tiny cases."""
    import os
    import types
    path = os.path.join(os.path.dirname(O.__file__), "paths.py")
    text = open(path).read()
    assert old in text
    mod = types.ModuleType("mutant_paths")
    exec(compile(text.replace(old, new, 1), "mutant_paths", "exec"), mod.__dict__)
    rng = np.random.default_rng(123)
    caught = False
    for _ in range(400):
        n = int(rng.integers(2, 7))
        m = int(rng.integers(1, 12))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n)), int(rng.integers(0, 9)),
                  int(rng.integers(1, 4))) for _ in range(m)]
        s, ta = int(rng.integers(0, n)), int(rng.integers(0, 4))
        tw = int(rng.integers(ta, 14))
        bea, last, bhops, _, _ = P.brute_force_walks(n, edges, s, ta, tw)
        sea, _, shops, sld, sfa = P.brute_force_walks(n, edges, s, ta, tw, strict=True)
        src, dst, t, lam = arrays(edges)
        ea = np.array(bea, np.uint32)
        pt, pd = mod.ea_predecessors(n, src, dst, t, lam, s, ta, tw, ea)
        hops, hea = mod.min_hops(n, src, dst, t, lam, s, ta, tw)
        h2, e2 = mod.min_hops(n, src, dst, t, lam, s, ta, tw, True)
        l2, f2 = mod.strict_sweep(n, src, dst, t, lam, s, ta, tw, True)
        to = mod.latest_departure_to(n, src, dst, t, lam, s, ta, tw)
        to2 = mod.latest_departure_to(n, src, dst, t, lam, s, ta, tw, True)
        if any((int(pt[v]), int(pd[v])) != rule_pick(last[v]) for v in range(n)) or \
                list(hops) != bhops or list(hea) != bea or list(h2) != shops or list(e2) != sea or \
                list(l2) != sld or list(f2) != sfa or \
                list(to) != P.brute_force_to(n, edges, s, ta, tw) or \
                list(to2) != P.brute_force_to(n, edges, s, ta, tw, True):
            caught = True
            break
    assert caught


@settings(max_examples=1000, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_cases(), st.booleans())
def test_succession_predicates_match_enumeration(case, strict):
    """Both predicates of §2.2: earliest arrival and hops from the level
    iteration, latest departure and fastest from the cross-route sweep, all
    against walk enumeration; without strictness also against the C profile
    scan (an independent route)."""
    n, edges, s, ta, tw = case
    bea, _, bhops, bld, bfa = P.brute_force_walks(n, edges, s, ta, tw, strict)
    src, dst, t, lam = arrays(edges)
    hops, ea = P.min_hops(n, src, dst, t, lam, s, ta, tw, strict)
    assert list(ea) == bea and list(hops) == bhops
    ld, fa = P.strict_sweep(n, src, dst, t, lam, s, ta, tw, strict)
    assert list(ld) == bld and list(fa) == bfa
    if not strict:
        pea, pld, pf = O.profile(O.sort_by_departure(n, src, dst, t, lam), s, ta, tw)
        assert list(pld) == bld and list(pf) == bfa


def test_strict_hand_worked():
    # 0 -(t=1, a=2)-> 1 -(t=2, a=3)-> 2 and 1 -(t=3, a=5)-> 2; window [1, 10].
    # Succeeds: 2 at 3 over the edge leaving at 1's arrival.  Strictly
    # succeeds: that edge is too early, 2 at 5.  The source's edge leaving at
    # t_alpha = 1 is usable under both.
    n, edges = 3, [(0, 1, 1, 1), (1, 2, 2, 1), (1, 2, 3, 2)]
    src, dst, t, lam = arrays(edges)
    assert P.min_hops(n, src, dst, t, lam, 0, 1, 10)[1].tolist() == [1, 2, 3]
    assert P.min_hops(n, src, dst, t, lam, 0, 1, 10, strict=True)[1].tolist() == [1, 2, 5]
    ld, fa = P.strict_sweep(n, src, dst, t, lam, 0, 1, 10, strict=True)
    assert ld.tolist() == [10, 1, 1] and fa.tolist() == [0, 1, 4]


TMAX = 0xFFFFFFFE


def reversed_edges(src, dst, t, lam):
    """Each edge (u, v, t, lam) becomes (v, u, TMAX - (t + lam), lam): the
    time axis read backwards."""
    a = t.astype(np.int64) + lam
    return dst, src, (TMAX - a).astype(np.uint32), lam


@settings(max_examples=800, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_cases(), st.booleans())
def test_latest_departure_to_matches_enumeration(case, strict):
    n, edges, target, ta, tw = case
    want = P.brute_force_to(n, edges, target, ta, tw, strict)
    src, dst, t, lam = arrays(edges)
    got = P.latest_departure_to(n, src, dst, t, lam, target, ta, tw, strict)
    assert list(got) == want


@settings(max_examples=500, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_cases(), st.booleans())
def test_latest_departure_to_is_earliest_arrival_backwards(case, strict):
    """Latest departure towards a target equals TMAX minus the earliest
    arrival from that target on the time-reversed graph, with the window
    reversed too: an independent route (the C scan without strictness)."""
    n, edges, target, ta, tw = case
    src, dst, t, lam = arrays(edges)
    got = P.latest_departure_to(n, src, dst, t, lam, target, ta, tw, strict)
    rs, rd, rt, rl = reversed_edges(src, dst, t, lam)
    if strict:
        _, ea = P.min_hops(n, rs, rd, rt, rl, target, TMAX - tw, TMAX - ta, True)
    else:
        ea = O.earliest_arrival(O.sort_by_departure(n, rs, rd, rt, rl), target, TMAX - tw, TMAX - ta)
    back = np.where(ea == INF, INF, TMAX - ea.astype(np.int64))
    assert got.tolist() == back.tolist()


def test_latest_departure_to_hand_worked():
    # 0 -(t=1,a=2)-> 1 -(t=2,a=3)-> 2 (target) and 0 -(t=4,a=9)-> 2; window [0, 10].
    # From 0 the latest departure that still reaches 2 is 4 (direct edge);
    # from 1 it is 2.  With the window ending at 8 the direct edge is gone.
    n, edges = 3, [(0, 1, 1, 1), (1, 2, 2, 1), (0, 2, 4, 5)]
    src, dst, t, lam = arrays(edges)
    assert P.latest_departure_to(n, src, dst, t, lam, 2, 0, 10).tolist() == [4, 2, 10]
    assert P.latest_departure_to(n, src, dst, t, lam, 2, 0, 8).tolist() == [1, 2, 8]
    # strictly succeeds: 0 -> 1 arrives at 2 and 1 leaves at 2, too early
    assert P.latest_departure_to(n, src, dst, t, lam, 2, 0, 8, strict=True).tolist() == [INF, 2, 8]
