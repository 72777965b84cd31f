"""GPU parity of earliest-arrival predecessors and temporal BFS hop counts
against the path oracle (``oracle.paths``), through the C interface.
Integer results, unique by definition: bit-exact."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from oracle import paths as P  # noqa: E402
import paper_2401_02563_amd as K  # noqa: E402
from workloads import make_graph, make_queries, tiny_graph, Graph  # noqa: E402

INF = 0xFFFFFFFF
_CACHE = {}


def built(key, factory):
    if key not in _CACHE:
        g = factory()
        G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)
        se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
        _CACHE[key] = (g, G, se)
    return _CACHE[key]


GRAPHS = {
    "uniform": lambda: built("uniform", lambda: make_graph("uniform-10k")),
    "rmat16": lambda: built("rmat16", lambda: make_graph("rmat20-32m", scale_shift=4)),
    "bursty16": lambda: built("bursty16", lambda: make_graph("bursty22-1b", scale_shift=6)),
    "rmat_wide": lambda: built("rmat_wide", lambda: make_graph("rmat22-256m", scale_shift=8)),
}
QUERIES = {"uniform": "uniform-10k", "rmat16": "rmat20-32m", "bursty16": "bursty22-1b",
           "rmat_wide": "rmat22-256m"}


def path_gpu(G, s, a, w):
    out, pt, pd = (torch.full((G.n,), 7, dtype=torch.int32, device="cuda") for _ in range(3))
    K.kairos_earliest_arrival_path(G, s, a, w, out, pt, pd)
    return K.as_u32(out), K.as_u32(pt), K.as_u32(pd)


def hops_gpu(G, s, a, w):
    out = torch.full((G.n,), 7, dtype=torch.int32, device="cuda")
    K.kairos_temporal_bfs(G, s, a, w, out)
    return K.as_u32(out)


def check_query(g, G, se, s, a, w):
    print("case:", g.meta.get("kind"), g.n, g.m, s, a, w, flush=True)
    ea, pt, pd = path_gpu(G, s, a, w)
    want = O.earliest_arrival(se, s, a, w)
    assert np.array_equal(ea, want)
    wt, wd = P.ea_predecessors(g.n, g.src, g.dst, g.t, g.lam, s, a, w, want)
    assert np.array_equal(pt, wt)
    assert np.array_equal(pd, wd)
    hops = hops_gpu(G, s, a, w)
    wh, _ = P.min_hops(g.n, g.src, g.dst, g.t, g.lam, s, a, w)
    assert np.array_equal(hops, wh)


@pytest.mark.parametrize("which", list(GRAPHS))
def test_paths_and_hops(which):
    g, G, se = GRAPHS[which]()
    srcs, ta, tw = make_queries(QUERIES[which], g, count=6)
    for q in range(len(srcs)):
        check_query(g, G, se, int(srcs[q]), int(ta[q]), int(tw[q]))


@pytest.mark.parametrize("seed", range(20))
def test_tiny_every_source(seed):
    g = tiny_graph(seed, n=7, m=12, t_max=8, lam_max=3)
    G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    for s in range(g.n):
        check_query(g, G, se, s, seed % 4, 6 + seed % 7)
    G.free()


@pytest.mark.parametrize("tuning", [dict(tail_limit=0), dict(tail_limit=0, rounds_per_sync=1),
                                    dict(tail_limit=100000), dict(split=64, chunk=64, tail_limit=0),
                                    dict(arrival_filter=2, tail_limit=0), dict(dense_frontier=1, tail_limit=0),
                                    dict(single_persistent=1, tail_limit=0), dict(pull_alpha=1, tail_limit=0)])
def test_hops_independent_of_tuning(tuning):
    """Level-synchronous rounds must give the same hop counts whatever kernel
    path (one-workgroup loop, multi-block rounds) runs them."""
    g, G, se = GRAPHS["rmat16"]()
    old = K.kairos_get_tuning(G)
    try:
        K.kairos_set_tuning(G, **tuning)
        srcs, ta, tw = make_queries("rmat20-32m", g, count=3)
        for q in range(len(srcs)):
            print("case: tuning", tuning, q, flush=True)
            hops = hops_gpu(G, int(srcs[q]), int(ta[q]), int(tw[q]))
            wh, _ = P.min_hops(g.n, g.src, g.dst, g.t, g.lam, int(srcs[q]), int(ta[q]), int(tw[q]))
            assert np.array_equal(hops, wh)
    finally:
        K.kairos_set_tuning(G, **old)


def test_late_timestamps_and_ties():
    """Times near the top of the u32 range, many equal arrivals (bursts of
    identical departures): the predecessor tie rule and the hop levels."""
    rng = np.random.Generator(np.random.PCG64(91))
    n, m = 200, 6000
    src = rng.integers(0, n, m, dtype=np.uint32)
    dst = rng.integers(0, n, m, dtype=np.uint32)
    t = (0xFFFFFFFE - 400 + rng.integers(0, 40, m) * 8).astype(np.uint32)
    lam = rng.integers(1, 4, m, dtype=np.uint32) * 8
    g = Graph(n, src, dst, t, lam, dict(kind="late"))
    G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    for s in range(0, n, 23):
        for a, w in ((0, 0xFFFFFFFE), (0xFFFFFFFE - 300, 0xFFFFFFFE - 100)):
            check_query(g, G, se, s, a, w)
    G.free()


def test_argument_errors():
    g, G, se = GRAPHS["uniform"]()
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(K.KairosError) as ei:
        K.kairos_temporal_bfs(G, g.n, 0, 5, out)
    assert ei.value.status == 2
    with pytest.raises(K.KairosError) as ei:
        K.kairos_earliest_arrival_path(G, 0, 9, 5, out, out, out)
    assert ei.value.status == 2
