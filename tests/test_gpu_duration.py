"""Shortest duration (Table 4's "S. Duration" row) on the GPU, bit-exact
against the oracle's Pareto scan over (arrival, duration) and against walk
enumeration, under both succession predicates of §2.2."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle as O  # noqa: E402
import paper_2401_02563_amd as K  # noqa: E402
from workloads import Graph, make_graph, make_queries, tiny_graph  # noqa: E402

INF = 0xFFFFFFFF
SD = K.KAIROS_SHORTEST_DURATION
_CACHE = {}


def built(key, factory):
    if key not in _CACHE:
        g = factory()
        G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)
        se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
        _CACHE[key] = (g, G, se)
    return _CACHE[key]


def sd(G, s, a, w, strict=False):
    out = torch.full((G.n,), 7, dtype=torch.int32, device="cuda")
    if strict:
        K.kairos_query(G, SD, s, a, w, out, strict=True)
    else:
        K.kairos_shortest_duration(G, s, a, w, out)
    return K.as_u32(out)


@pytest.mark.parametrize("seed", range(20))
def test_tiny_every_source_against_enumeration(seed):
    g = tiny_graph(seed + 300, n=7, m=14, t_max=6, lam_max=3)
    G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)
    edges = list(zip(g.src.tolist(), g.dst.tolist(), g.t.tolist(), g.lam.tolist()))
    for s in range(g.n):
        for strict in (False, True):
            a, w = seed % 3, 6 + seed % 6
            print("case: tiny", seed, s, strict, flush=True)
            _, want = O.walk_facts(g.n, edges, s, a, w, strict=strict)
            assert sd(G, s, a, w, strict).tolist() == want
    G.free()


@pytest.mark.parametrize("strict", [False, True])
def test_uniform_all_sources(strict):
    g, G, se = built("uniform", lambda: make_graph("uniform-10k"))
    srcs, ta, tw = make_queries("uniform-10k", g)
    for i in range(len(srcs)):
        s, a, w = int(srcs[i]), int(ta[i]), int(tw[i])
        print("case: uniform", i, strict, flush=True)
        got = sd(G, s, a, w, strict)
        assert np.array_equal(got, O.shortest_duration(se, s, a, w, strict=strict)), i
    # durations are a different quantity from fastest: waiting is free
    _, _, fa = O.profile(se, int(srcs[0]), int(ta[0]), int(tw[0]))
    assert not np.array_equal(sd(G, int(srcs[0]), int(ta[0]), int(tw[0])), fa)


@pytest.mark.parametrize("which", ["rmat14", "rmat16", "bursty14", "bursty16", "rmat22-log"])
def test_skewed(which):
    name, shift, count = {"rmat14": ("rmat20-32m", 6, 6), "rmat16": ("rmat20-32m", 4, 4),
                          "bursty14": ("bursty22-1b", 8, 6), "bursty16": ("bursty22-1b", 6, 3),
                          "rmat22-log": ("rmat22-256m", 8, 8)}[which]
    g, G, se = built(which, lambda: make_graph(name, scale_shift=shift))
    srcs, ta, tw = make_queries(name, g, count=count)
    reached = 0
    for i in range(len(srcs)):
        s, a, w = int(srcs[i]), int(ta[i]), int(tw[i])
        for strict in (False, True):
            print("case:", which, i, strict, flush=True)
            got = sd(G, s, a, w, strict)
            assert np.array_equal(got, O.shortest_duration(se, s, a, w, strict=strict)), (i, strict)
            reached = max(reached, int((got != INF).sum()))
    assert reached > 100


def test_ties_near_top_of_range():
    """Times and durations on a grid of 8 near 2^32, so departures equal
    arrivals everywhere and the two predicates differ."""
    rng = np.random.Generator(np.random.PCG64(23))
    n, m = 150, 3000
    src = rng.integers(0, n, m, dtype=np.uint32)
    dst = rng.integers(0, n, m, dtype=np.uint32)
    t = (0xFFFFFFFE - 400 + rng.integers(0, 40, m) * 8).astype(np.uint32)
    lam = rng.integers(1, 4, m, dtype=np.uint32) * 8
    g = Graph(n, src, dst, t, lam, dict(kind="ties"))
    G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)
    se = O.sort_by_departure(n, src, dst, t, lam)
    differs = False
    for s in range(0, n, 29):
        for (a, w) in ((0, 0xFFFFFFFE), (0xFFFFFFFE - 300, 0xFFFFFFFE - 100)):
            got = {}
            for strict in (False, True):
                print("case: ties", s, a, w, strict, flush=True)
                got[strict] = sd(G, s, a, w, strict)
                assert np.array_equal(got[strict], O.shortest_duration(se, s, a, w, strict=strict))
            differs |= not np.array_equal(got[False], got[True])
    assert differs
    G.free()


def test_edge_cases_and_errors():
    # no edges; a source without out-edges; one vertex
    g = Graph(4, np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.uint32), {})
    G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)
    assert sd(G, 2, 0, 10).tolist() == [INF, INF, 0, INF]
    G.free()
    src = np.array([0, 1, 1], np.uint32)
    dst = np.array([1, 2, 0], np.uint32)
    t = np.array([5, 7, 9], np.uint32)
    lam = np.array([2, 3, 1], np.uint32)
    G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (src, dst, t, lam)], 4)
    assert sd(G, 0, 0, 100).tolist() == [0, 2, 5, INF]
    assert sd(G, 0, 0, 9).tolist() == [0, 2, INF, INF]   # 1 -> 2 arrives at 10
    assert sd(G, 0, 6, 100).tolist() == [0, INF, INF, INF]
    assert sd(G, 3, 0, 100).tolist() == [INF, INF, INF, 0]
    assert sd(G, 0, 5, 7, strict=True).tolist() == [0, 2, INF, INF]
    out = torch.empty(4, dtype=torch.int32, device="cuda")
    with pytest.raises(K.KairosError) as e:
        K.kairos_shortest_duration(G, 4, 0, 10, out)
    assert e.value.status == 2
    with pytest.raises(K.KairosError) as e:
        K.kairos_shortest_duration(G, 0, 11, 10, out)
    assert e.value.status == 2
    # the two out-edge to in-index maps (4 B per edge each) are counted with
    # the index
    _, _, bytes_after = K.kairos_graph_stats(G)
    G.free()
    G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (src, dst, t, lam)], 4)
    _, _, bytes_before = K.kairos_graph_stats(G)
    assert bytes_after == bytes_before + 8 * 3
    G.free()


def test_full_size_scale20_queries():
    """Two queries of the scale-20 workload at full size (2^25 edges)."""
    g, G, se = built("rmat20-full", lambda: make_graph("rmat20-32m"))
    srcs, ta, tw = make_queries("rmat20-32m", g)
    for q in (0, 7):
        s, a, w = int(srcs[q]), int(ta[q]), int(tw[q])
        print("case: rmat20-32m full", q, flush=True)
        got = sd(G, s, a, w)
        assert np.array_equal(got, O.shortest_duration(se, s, a, w)), q
        assert int((got != INF).sum()) > 10000


def _hub_graph(T=12000, seed=5):
    """A hub h whose in-list is lowered across T positions in one round (a
    dirty range longer than one wavefront expands, spanning two tiles of the
    workgroup expansion), later in-edges that the first expansion fills, an
    early arrival of small total that refills the whole list, a sink without
    out-edges with more than 32 in-edges, and exact copies of edges."""
    rng = np.random.default_rng(seed)
    s, y, w1, c1, h, z = 0, 1, 2, 3, 4, 5
    u = 6 + np.arange(T)                    # reached from s in round 0
    up = 6 + T + np.arange(64)              # reached two rounds later
    x = 6 + T + 64 + np.arange(32)          # the hub's successors
    n = int(x[-1]) + 1
    E = []
    E += [(s, int(u[i]), 10 + i, int(rng.integers(1, 1000))) for i in range(T)]
    times = rng.permutation(T)
    E += [(int(u[i]), h, 20000 + int(times[i]), int(rng.integers(1, 50))) for i in range(T)]
    E += [(int(u[i]), z, 20000 + i, int(rng.integers(1, 50))) for i in range(100)]
    E += [(s, y, 1, 1), (y, w1, 2, 1), (w1, h, 3, 1)]           # early, total 3
    E += [(s, c1, 5, 2)] + [(c1, int(up[k]), 6 + k, 3) for k in range(64)]
    E += [(int(up[k]), h, 50000 + k, int(rng.integers(1, 9))) for k in range(64)]
    E += [(h, int(x[j]), int(t), int(rng.integers(1, 20))) for j in range(32) for t in (4 + j, 30000 + 97 * j, 60000 + j)]
    # exact copies of edges (each copy keeps a label of its own)
    E += E[:40] + E[T:T + 40] + [(w1, h, 3, 1)] * 2 + E[-10:]
    src, dst, t, lam = (np.array([e[k] for e in E], dtype=np.uint32) for k in range(4))
    return Graph(n, src, dst, t, lam, dict(kind="hub", seed=seed))


@pytest.mark.parametrize("strict", [False, True])
def test_long_dirty_ranges_and_sinks(strict):
    """Dirty ranges expanded by a workgroup, long fills past the dirty end,
    and the minimum over a long in-list of a vertex without out-edges."""
    g, G, se = built("hub", _hub_graph)
    for s, a, w in ((0, 0, 70000), (0, 0, 40000), (0, 2, 70000), (0, 9, 25000)):
        print("case: hub", s, a, w, strict, flush=True)
        got = sd(G, s, a, w, strict)
        assert np.array_equal(got, O.shortest_duration(se, s, a, w, strict=strict)), (s, a, w)
    assert int((sd(G, 0, 0, 70000, strict) != INF).sum()) > 12000


@pytest.mark.parametrize("rps", [1, 3])
def test_rounds_per_check_and_counters(rps):
    """Rounds checked one at a time or queued three per host check, with
    work counters off and on (on: every round is checked), give the same
    labels."""
    g, G, se = built("bursty16", lambda: make_graph("bursty22-1b", scale_shift=6))
    srcs, ta, tw = make_queries("bursty22-1b", g, count=3)
    old = K.kairos_get_tuning(G)
    K.kairos_set_tuning(G, rounds_per_sync=rps)
    try:
        for i in range(len(srcs)):
            s, a, w = int(srcs[i]), int(ta[i]), int(tw[i])
            want = O.shortest_duration(se, s, a, w)
            print("case: rounds per check", rps, i, flush=True)
            assert np.array_equal(sd(G, s, a, w), want), i
            K.kairos_profile_enable(G, True)
            K.kairos_profile_read(G)
            got = sd(G, s, a, w)
            prof = K.kairos_profile_read(G)
            K.kairos_profile_enable(G, False)
            assert np.array_equal(got, want), i
            if int((want != INF).sum()) > 1:
                assert prof["rounds"] > 0 and prof["items"] > 0 and prof["edges_scanned"] > 0, prof
    finally:
        K.kairos_set_tuning(G, **old)
