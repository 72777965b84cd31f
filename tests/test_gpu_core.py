"""GPU parity of the index builder and single / batched queries against the
CPU oracle, through the C interface.  Integer results: bit-exact."""
import json
import glob
import os
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle as O  # noqa: E402
import paper_2401_02563_amd as K  # noqa: E402
from workloads import make_graph, make_queries, tiny_graph, Graph  # noqa: E402

INF = 0xFFFFFFFF
_CACHE = {}


def dev(g):
    return [K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)]


def built(key, factory):
    if key not in _CACHE:
        g = factory()
        G = K.kairos_graph_build(*dev(g), g.n)
        se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
        _CACHE[key] = (g, G, se)
    return _CACHE[key]


def uniform():
    return built("uniform", lambda: make_graph("uniform-10k"))


def rmat16():
    return built("rmat16", lambda: make_graph("rmat20-32m", scale_shift=4))


def bursty16():
    return built("bursty16", lambda: make_graph("bursty22-1b", scale_shift=6))


def rmat_wide():
    return built("rmat_wide", lambda: make_graph("rmat22-256m", scale_shift=8))


def gappy():
    """Long blocks of vertices without in-edges and without out-edges in the
    middle of the internal id order: 3,000 vertices reach only the first 100,
    1,000 more are isolated, 2,000 are targets only."""
    def make():
        rng = np.random.default_rng(17)
        m = 40_000
        src = rng.integers(0, 3_000, m).astype(np.uint32)
        dst = np.where(rng.random(m) < 0.5, rng.integers(0, 100, m), rng.integers(4_000, 6_000, m)).astype(np.uint32)
        t = rng.integers(0, 50_000, m).astype(np.uint32)
        lam = rng.integers(1, 20, m).astype(np.uint32)
        return Graph(6_000, src, dst, t, lam, dict(kind="gappy"))
    return built("gappy", make)


def ea_gpu(G, s, a, w):
    out = torch.empty(G.n, dtype=torch.int32, device="cuda")
    K.kairos_earliest_arrival(G, s, a, w, out)
    return K.as_u32(out)


def print_case(*a):
    print("case:", *a, flush=True)


@pytest.mark.parametrize("which", ["uniform", "rmat16", "bursty16", "rmat_wide", "gappy"])
def test_index_matches_lexsort(which):
    g, G, _ = {"uniform": uniform, "rmat16": rmat16, "bursty16": bursty16, "rmat_wide": rmat_wide,
               "gappy": gappy}[which]()
    print_case("index", which, g.n, g.m)
    view = K.kairos_graph_index(G)
    ix = {k: K.as_u32(v) for k, v in view.items() if k != "n_live"}
    # internal ids: vertices with out-edges first, then the others; within
    # each part decreasing in-degree (clamped to 31 bits), ties by caller id
    perm = ix["perm"]
    assert np.array_equal(np.sort(perm), np.arange(g.n, dtype=np.uint32))
    indeg = np.minimum(np.bincount(g.dst, minlength=g.n), (1 << 31) - 1)
    sink = np.bincount(g.src, minlength=g.n) == 0
    order = np.lexsort((np.arange(g.n), -indeg, sink))
    assert np.array_equal(perm[order], np.arange(g.n, dtype=np.uint32))
    assert view["n_live"] == int((~sink).sum())
    want = O.temporal_csr(g.n, perm[g.src], perm[g.dst], g.t, g.lam)
    assert np.array_equal(ix["off_out"], want["off_out"].astype(np.uint32))
    assert np.array_equal(ix["off_in"], want["off_in"].astype(np.uint32))
    assert np.array_equal(ix["t_out"], want["t_out"])
    da = ix["dst_a_out"].reshape(-1, 2)
    assert np.array_equal(da[:, 0], want["dst_out"]) and np.array_equal(da[:, 1], want["a_out"])
    assert np.array_equal(ix["a_in"], want["a_in"])
    st = ix["src_t_in"].reshape(-1, 2)
    assert np.array_equal(st[:, 0], want["src_in"]) and np.array_equal(st[:, 1], want["t_in"])


def test_ea_uniform_all_sources():
    g, G, se = uniform()
    srcs, ta, tw = make_queries("uniform-10k", g)
    for q in range(len(srcs)):
        print_case("ea uniform", q)
        got = ea_gpu(G, int(srcs[q]), int(ta[q]), int(tw[q]))
        want = O.earliest_arrival(se, srcs[q], ta[q], tw[q])
        assert np.array_equal(got, want), q
        assert O.ea_certificate(g.n, g.src, g.dst, g.t, g.lam, int(srcs[q]), int(ta[q]), int(tw[q]), got)


@pytest.mark.parametrize("which", ["rmat16", "bursty16", "rmat_wide"])
def test_ea_skewed(which):
    g, G, se = {"rmat16": rmat16, "bursty16": bursty16, "rmat_wide": rmat_wide}[which]()
    name = {"rmat16": "rmat20-32m", "bursty16": "bursty22-1b", "rmat_wide": "rmat22-256m"}[which]
    srcs, ta, tw = make_queries(name, g, count=8)
    for q in range(len(srcs)):
        print_case("ea", which, q)
        got = ea_gpu(G, int(srcs[q]), int(ta[q]), int(tw[q]))
        want = O.earliest_arrival(se, srcs[q], ta[q], tw[q])
        assert np.array_equal(got, want), q
        tg = K.kairos_traversed_edges(G, int(ta[q]), int(tw[q]), torch.from_numpy(got.view(np.int32)).cuda())
        assert tg == O.traversed_edges(se, ta[q], tw[q], want)


@pytest.mark.parametrize("tuning", [dict(split=64, chunk=64), dict(split=100000, chunk=4096),
                                    dict(rounds_per_sync=4), dict(rounds_per_sync=1), dict(pull_alpha=1, pull_beta=1000000),
                                    dict(pull_alpha=8, pull_beta=24), dict(arrival_filter=0),
                                    dict(arrival_filter=0, tail_limit=0), dict(arrival_filter=2),
                                    dict(arrival_filter=4), dict(arrival_filter=8, tail_limit=0),
                                    dict(arrival_filter=2, tail_limit=0, dense_frontier=4),
                                    dict(single_persistent=0), dict(run_dedupe=1),
                                    dict(single_persistent=1, tail_limit=0),
                                    dict(single_persistent=1, tail_limit=0, dense_frontier=4),
                                    dict(block=512), dict(block=512, tail_limit=0),
                                    dict(block=512, tail_limit=0, split=64, chunk=64),
                                    dict(block=512, tail_limit=0, dense_frontier=4, pull_alpha=8, pull_beta=24)])
def test_ea_independent_of_tuning(tuning):
    """Results are unique, so every launch configuration must agree bit for bit."""
    g, G, se = rmat16()
    old = K.kairos_get_tuning(G)
    try:
        K.kairos_set_tuning(G, **tuning)
        srcs, ta, tw = make_queries("rmat20-32m", g, count=4)
        for q in range(len(srcs)):
            print_case("tuning", tuning, q)
            got = ea_gpu(G, int(srcs[q]), int(ta[q]), int(tw[q]))
            assert np.array_equal(got, O.earliest_arrival(se, srcs[q], ta[q], tw[q]))
    finally:
        K.kairos_set_tuning(G, **old)


GOLD = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "*.json")))


@pytest.mark.parametrize("path", GOLD, ids=[os.path.basename(p) for p in GOLD])
def test_golden_on_gpu(path):
    d = json.load(open(path))
    e = np.array(d["edges"], np.uint32).reshape(-1, 4)
    G = K.kairos_graph_build(*[K.to_u32_tensor(e[:, i]) for i in range(4)], d["n"])
    out = torch.empty(d["n"], dtype=torch.int32, device="cuda")
    args = (d["source"], d["t_alpha"], d["t_omega"], out)
    K.kairos_earliest_arrival(G, *args)
    assert K.as_u32(out).tolist() == d["ea"]
    K.kairos_latest_departure(G, *args)
    assert K.as_u32(out).tolist() == d["ld"]
    K.kairos_fastest(G, *args)
    assert K.as_u32(out).tolist() == d["fastest"]
    G.free()


@pytest.mark.parametrize("seed", range(30))
def test_tiny_all_kinds(seed):
    g = tiny_graph(seed, n=7, m=12, t_max=8, lam_max=3)
    G = K.kairos_graph_build(*dev(g), g.n)
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for s in range(g.n):
        ta, tw = seed % 4, 6 + seed % 7
        pea, pld, pf = O.profile(se, s, ta, tw)
        K.kairos_earliest_arrival(G, s, ta, tw, out)
        assert np.array_equal(K.as_u32(out), pea)
        K.kairos_latest_departure(G, s, ta, tw, out)
        assert np.array_equal(K.as_u32(out), pld)
        K.kairos_fastest(G, s, ta, tw, out)
        assert np.array_equal(K.as_u32(out), pf)
    G.free()


@pytest.mark.parametrize("filt", [0, 2, 4, 8])
def test_late_timestamps_all_kinds(filt):
    """Departures near the top of the u32 range and windows up to the whole
    range: the arrival codes then use their widest parts (up to 2^31), where
    a code's bound comes closest to overflowing 32 bits."""
    rng = np.random.Generator(np.random.PCG64(77))
    n, m = 300, 4000
    src = rng.integers(0, n, m, dtype=np.uint32)
    dst = rng.integers(0, n, m, dtype=np.uint32)
    t = rng.integers(0xFFFFFFFE - (1 << 26), 0xFFFFFFFE - 200, m, dtype=np.uint64).astype(np.uint32)
    lam = rng.integers(1, 150, m, dtype=np.uint32)
    g = Graph(n, src, dst, t, lam, dict(kind="late"))
    G = K.kairos_graph_build(*dev(g), g.n)
    K.kairos_set_tuning(G, arrival_filter=filt, tail_limit=0 if filt else 4096)
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    lo = int(t.min())
    for s in range(0, n, 37):
        for ta, tw in ((0, 0xFFFFFFFE), (lo + (1 << 24), 0xFFFFFFFE - (1 << 20))):
            print_case("late", filt, s, ta, tw)
            pea, pld, pf = O.profile(se, s, ta, tw)
            K.kairos_earliest_arrival(G, s, ta, tw, out)
            assert np.array_equal(K.as_u32(out), pea), (s, ta, tw)
            K.kairos_latest_departure(G, s, ta, tw, out)
            assert np.array_equal(K.as_u32(out), pld), (s, ta, tw)
            K.kairos_fastest(G, s, ta, tw, out)
            assert np.array_equal(K.as_u32(out), pf), (s, ta, tw)
    G.free()


def test_ld_fastest_uniform():
    g, G, se = uniform()
    srcs, ta, tw = make_queries("uniform-10k", g)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for q in range(4):
        print_case("ldf uniform", q)
        pea, pld, pf = O.profile(se, srcs[q], ta[q], tw[q])
        K.kairos_latest_departure(G, int(srcs[q]), int(ta[q]), int(tw[q]), out)
        assert np.array_equal(K.as_u32(out), pld), q
        K.kairos_fastest(G, int(srcs[q]), int(ta[q]), int(tw[q]), out)
        assert np.array_equal(K.as_u32(out), pf), q


@pytest.mark.parametrize("persistent,tail", [(0, 4096), (1, 0), (1, 64)])
def test_ld_fastest_launch_modes(persistent, tail):
    """Sweeps give the same answers with rounds in one cooperative launch,
    in per-round launches, and with small frontiers in one workgroup."""
    g, G, se = rmat16()
    srcs, ta, tw = make_queries("rmat20-32m", g, count=3)
    old = K.kairos_get_tuning(G)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    try:
        K.kairos_set_tuning(G, single_persistent=persistent, tail_limit=tail)
        for q in range(3):
            print_case("ldf modes", persistent, tail, q)
            pea, pld, pf = O.profile(se, srcs[q], ta[q], tw[q])
            K.kairos_earliest_arrival(G, int(srcs[q]), int(ta[q]), int(tw[q]), out)
            assert np.array_equal(K.as_u32(out), pea), q
            K.kairos_latest_departure(G, int(srcs[q]), int(ta[q]), int(tw[q]), out)
            assert np.array_equal(K.as_u32(out), pld), q
            K.kairos_fastest(G, int(srcs[q]), int(ta[q]), int(tw[q]), out)
            assert np.array_equal(K.as_u32(out), pf), q
    finally:
        K.kairos_set_tuning(G, **old)


def test_ld_fastest_bursty():
    g, G, se = bursty16()
    srcs, ta, tw = make_queries("bursty22-1b", g, count=3)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for q in range(3):
        print_case("ldf bursty", q)
        pea, pld, pf = O.profile(se, srcs[q], ta[q], tw[q])
        K.kairos_latest_departure(G, int(srcs[q]), int(ta[q]), int(tw[q]), out)
        assert np.array_equal(K.as_u32(out), pld), q
        K.kairos_fastest(G, int(srcs[q]), int(ta[q]), int(tw[q]), out)
        assert np.array_equal(K.as_u32(out), pf), q


@pytest.mark.parametrize("which", ["uniform", "rmat_wide"])
def test_batch_rows_equal_single(which):
    g, G, se = {"uniform": uniform, "rmat_wide": rmat_wide}[which]()
    name = {"uniform": "uniform-10k", "rmat_wide": "rmat22-256m"}[which]
    srcs, ta, tw = make_queries(name, g, count=16)
    out = torch.empty(len(srcs) * g.n, dtype=torch.int32, device="cuda")
    print_case("batch", which)
    K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
    rows = K.as_u32(out).reshape(len(srcs), g.n)
    for q in range(len(srcs)):
        assert np.array_equal(rows[q], O.earliest_arrival(se, srcs[q], ta[q], tw[q])), q


@pytest.mark.parametrize("layout,persistent,dedupe", [(1, 0, 1), (2, 0, 1), (2, 1, 1), (2, 1, 0), (0, 0, 1), (3, 0, 1)])
def test_batch_bursty_runs(layout, persistent, dedupe):
    """Bursty pairs put runs of edges into one head next to each other: the
    batch kernels with and without one atomic per run agree with the oracle."""
    g, G, se = bursty16()
    assert K.kairos_get_tuning(G)["run_dedupe"] == 1  # default from the index statistics
    srcs, ta, tw = make_queries("bursty22-1b", g, count=70)
    old = K.kairos_get_tuning(G)
    try:
        K.kairos_set_tuning(G, batch_layout=layout, batch_persistent=persistent, run_dedupe=dedupe)
        out = torch.empty(len(srcs) * g.n, dtype=torch.int32, device="cuda")
        print_case("bursty batch", layout, persistent, dedupe)
        K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
        rows = K.as_u32(out).reshape(len(srcs), g.n)
        for qi in list(range(0, 70, 9)) + [63, 64, 69]:
            assert np.array_equal(rows[qi], O.earliest_arrival(se, srcs[qi], ta[qi], tw[qi])), qi
    finally:
        K.kairos_set_tuning(G, **old)


def test_edge_cases():
    # empty graph
    g = Graph(5, *(np.zeros(0, np.uint32) for _ in range(4)))
    G = K.kairos_graph_build(*dev(g), g.n)
    assert ea_gpu(G, 3, 7, 9).tolist() == [INF, INF, INF, 7, INF]
    out = torch.empty(5, dtype=torch.int32, device="cuda")
    K.kairos_latest_departure(G, 3, 7, 9, out)
    assert K.as_u32(out).tolist() == [INF, INF, INF, 9, INF]
    G.free()
    # one vertex with a self-loop; window of width zero
    g = Graph(1, np.array([0], np.uint32), np.array([0], np.uint32), np.array([5], np.uint32),
              np.array([1], np.uint32))
    G = K.kairos_graph_build(*dev(g), 1)
    assert ea_gpu(G, 0, 5, 5).tolist() == [5]
    G.free()
    # times at the top of the range, arrival exactly TMAX
    T = 0xFFFFFFFE
    g = Graph(3, np.array([0, 1], np.uint32), np.array([1, 2], np.uint32),
              np.array([T - 3, T - 1], np.uint32), np.array([2, 1], np.uint32))
    G = K.kairos_graph_build(*dev(g), 3)
    assert ea_gpu(G, 0, 0, T).tolist() == [0, T - 1, T]
    G.free()


def test_build_rejects_bad_edges():
    ok = tiny_graph(1)
    for field, val, status in (("src", 7, 2), ("dst", 99, 2), ("lam", 0, 2)):
        g = tiny_graph(1)
        getattr(g, field)[3] = val
        with pytest.raises(K.KairosError) as ei:
            K.kairos_graph_build(*dev(g), g.n)
        assert ei.value.status == status
    g = tiny_graph(1)
    g.t[0] = 0xFFFFFFFE
    with pytest.raises(K.KairosError):
        K.kairos_graph_build(*dev(g), g.n)
    G = K.kairos_graph_build(*dev(ok), ok.n)
    out = torch.full((ok.n,), 123, dtype=torch.int32, device="cuda")
    for args in ((ok.n, 0, 5), (0, 6, 5), (0, 0, 0xFFFFFFFF)):
        with pytest.raises(K.KairosError) as ei:
            K.kairos_earliest_arrival(G, *args, out)
        assert ei.value.status == 2
    assert (out == 123).all()
    G.free()


@pytest.mark.parametrize("layout,persistent", [(0, 0), (1, 0), (2, 0), (2, 1), (3, 0)])
def test_batch_layouts_ragged_groups(layout, persistent):
    """100 queries = one full and one ragged group of 64 lanes."""
    g, G, se = rmat16()
    srcs, ta, tw = make_queries("rmat22-256m", g, count=100)  # log-uniform windows on this graph
    ta = (ta.astype(np.uint64) * ((1 << 30) - 1) // 0xFFFFFFF4).astype(np.uint32)
    tw = np.maximum(ta, (tw.astype(np.uint64) * ((1 << 30) - 1) // 0xFFFFFFF4).astype(np.uint32))
    old = K.kairos_get_tuning(G)
    try:
        K.kairos_set_tuning(G, batch_layout=layout, batch_persistent=persistent)
        out = torch.empty(len(srcs) * g.n, dtype=torch.int32, device="cuda")
        print_case("batch layout", layout, "persistent", persistent)
        K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
        rows = K.as_u32(out).reshape(len(srcs), g.n)
        for qi in list(range(0, 100, 7)) + [63, 64, 99]:
            assert np.array_equal(rows[qi], O.earliest_arrival(se, srcs[qi], ta[qi], tw[qi])), qi
    finally:
        K.kairos_set_tuning(G, **old)


@pytest.mark.parametrize("q", [1, 64, 130])
def test_batch_persistent_matches_per_round(q):
    """One persistent launch for all rounds equals one launch per phase, bit
    for bit, and the oracle on sampled rows; repeated calls reuse the state."""
    g, G, se = uniform()
    srcs, ta, tw = make_queries("uniform-10k", g, count=q)
    old = K.kairos_get_tuning(G)
    outs = []
    try:
        for persistent in (0, 1, 1):
            K.kairos_set_tuning(G, batch_layout=2, batch_persistent=persistent)
            out = torch.full((q * g.n,), 5, dtype=torch.int32, device="cuda")
            print_case("persistent", q, persistent)
            K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
            outs.append(K.as_u32(out).reshape(q, g.n))
    finally:
        K.kairos_set_tuning(G, **old)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])
    for qi in sorted({0, q // 2, q - 1}):
        assert np.array_equal(outs[1][qi], O.earliest_arrival(se, srcs[qi], ta[qi], tw[qi])), qi


def test_batch_duplicate_sources():
    g, G, se = uniform()
    s = int(make_queries("uniform-10k", g)[0][0])
    k = 70
    ta = np.arange(k, dtype=np.uint32) * 1000
    tw = np.full(k, 99_999, np.uint32)
    tw[::3] = ta[::3] + 20_000
    srcs = np.full(k, s, np.uint32)
    out = torch.empty(k * g.n, dtype=torch.int32, device="cuda")
    K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
    rows = K.as_u32(out).reshape(k, g.n)
    for qi in range(k):
        assert np.array_equal(rows[qi], O.earliest_arrival(se, s, ta[qi], tw[qi])), qi


def test_chunk_list_overflow_paths():
    """A chunk list of 3 entries forces the in-kernel fallback walks."""
    os.environ["KAIROS_TEST_CHUNK_CAP"] = "3"
    try:
        g = make_graph("rmat20-32m", scale_shift=6)
        G = K.kairos_graph_build(*dev(g), g.n)
        K.kairos_set_tuning(G, split=64, chunk=64)
        se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
        srcs, ta, tw = make_queries("rmat20-32m", g, count=70)
        for qi in range(3):
            assert np.array_equal(ea_gpu(G, int(srcs[qi]), int(ta[qi]), int(tw[qi])),
                                  O.earliest_arrival(se, srcs[qi], ta[qi], tw[qi]))
        out = torch.empty(len(srcs) * g.n, dtype=torch.int32, device="cuda")
        for layout in (0, 1, 2, 3):
            K.kairos_set_tuning(G, batch_layout=layout)
            K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
            rows = K.as_u32(out).reshape(len(srcs), g.n)
            for qi in (0, 5, 64, 69):
                assert np.array_equal(rows[qi], O.earliest_arrival(se, srcs[qi], ta[qi], tw[qi])), (layout, qi)
        G.free()
    finally:
        del os.environ["KAIROS_TEST_CHUNK_CAP"]


def test_autotune_keeps_results(tmp_path):
    """The tuner keeps results exact, stores its choice under the graph's key
    in the cache file, and takes it from there the next time without
    measuring; the tuning sample is held out from the timed queries."""
    g, G, se = rmat16()
    srcs, ta, tw = make_queries("rmat20-32m", g, count=8)
    hs, ha, hw = make_queries("rmat20-32m", g, count=8, held_out=True)
    assert not set(zip(srcs.tolist(), ta.tolist())) & set(zip(hs.tolist(), ha.tolist()))
    old = K.kairos_get_tuning(G)
    cache = tmp_path / "tuning.txt"
    os.environ["KAIROS_TUNING_CACHE"] = str(cache)
    try:
        best = K.kairos_autotune(G, hs, ha, hw)
        assert best == K.kairos_get_tuning(G)
        lines = cache.read_text().splitlines()
        assert len(lines) == 1 and lines[0].split()[0].endswith("/batch")
        assert [int(x) for x in lines[0].split()[1:]] == list(best.values())
        K.kairos_set_tuning(G, **old)
        t0 = time.perf_counter()
        again = K.kairos_autotune(G, hs, ha, hw)
        assert again == best and time.perf_counter() - t0 < 0.5
        one = K.kairos_autotune(G, hs[:1], ha[:1], hw[:1])  # another key: one-query form
        assert len(cache.read_text().splitlines()) == 2
        K.kairos_set_tuning(G, **one)
        assert np.array_equal(ea_gpu(G, int(srcs[1]), int(ta[1]), int(tw[1])),
                              O.earliest_arrival(se, srcs[1], ta[1], tw[1]))
        K.kairos_set_tuning(G, **best)
        out = torch.empty(len(srcs) * g.n, dtype=torch.int32, device="cuda")
        K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
        rows = K.as_u32(out).reshape(len(srcs), g.n)
        for q in range(len(srcs)):
            assert np.array_equal(rows[q], O.earliest_arrival(se, srcs[q], ta[q], tw[q])), q
        assert np.array_equal(ea_gpu(G, int(srcs[0]), int(ta[0]), int(tw[0])),
                              O.earliest_arrival(se, srcs[0], ta[0], tw[0]))
    finally:
        del os.environ["KAIROS_TUNING_CACHE"]
        K.kairos_set_tuning(G, **old)


@pytest.mark.parametrize("dense", [0, 1, 4, 1000000])
def test_dense_frontier_walk(dense):
    """Dense rounds (every vertex walked, members found by their stamp) give
    the same bits as queue rounds, also right after pull rounds."""
    g, G, se = rmat16()
    old = K.kairos_get_tuning(G)
    try:
        K.kairos_set_tuning(G, dense_frontier=dense, tail_limit=0 if dense == 1000000 else 4096)
        srcs, ta, tw = make_queries("rmat20-32m", g, count=3)
        for q in range(len(srcs)):
            assert np.array_equal(ea_gpu(G, int(srcs[q]), int(ta[q]), int(tw[q])),
                                  O.earliest_arrival(se, srcs[q], ta[q], tw[q]))
        K.kairos_set_tuning(G, pull_alpha=8)
        assert np.array_equal(ea_gpu(G, int(srcs[0]), int(ta[0]), int(tw[0])),
                              O.earliest_arrival(se, srcs[0], ta[0], tw[0]))
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        pea, pld, pf = O.profile(se, srcs[1], ta[1], tw[1])
        K.kairos_latest_departure(G, int(srcs[1]), int(ta[1]), int(tw[1]), out)
        assert np.array_equal(K.as_u32(out), pld)
    finally:
        K.kairos_set_tuning(G, **old)


@pytest.mark.parametrize("layout,persistent", [(1, 0), (2, 0), (2, 1), (0, 0), (3, 0)])
def test_gappy_single_and_batch(layout, persistent):
    """Vertices without out-edges are never enqueued and vertices without
    in-edges sit in one block of ids: every query kind and batch layout still
    matches the oracle, including sources without out-edges."""
    g, G, se = gappy()
    old = K.kairos_get_tuning(G)
    K.kairos_set_tuning(G, batch_layout=layout, batch_persistent=persistent)
    try:
        rng = np.random.default_rng(5)
        srcs = np.concatenate([rng.integers(0, 3_000, 12), [3_500, 4_100, 5_999, 50]]).astype(np.uint32)
        ta = rng.integers(0, 20_000, len(srcs)).astype(np.uint32)
        tw = (ta + rng.integers(1_000, 60_000, len(srcs))).astype(np.uint32)
        print_case("gappy", layout, persistent)
        out = torch.empty(len(srcs) * g.n, dtype=torch.int32, device="cuda")
        K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
        rows = K.as_u32(out).reshape(len(srcs), g.n)
        one = torch.empty(g.n, dtype=torch.int32, device="cuda")
        for q in range(len(srcs)):
            s, a, w = int(srcs[q]), int(ta[q]), int(tw[q])
            pea, pld, pf = O.profile(se, s, a, w)
            assert np.array_equal(rows[q], pea), q
            assert np.array_equal(ea_gpu(G, s, a, w), pea), q
            if q % 4 == 0:
                K.kairos_latest_departure(G, s, a, w, one)
                assert np.array_equal(K.as_u32(one), pld), q
                K.kairos_fastest(G, s, a, w, one)
                assert np.array_equal(K.as_u32(one), pf), q
    finally:
        K.kairos_set_tuning(G, **old)


@pytest.mark.parametrize("which", ["uniform", "rmat16", "bursty16", "rmat_wide", "gappy"])
@pytest.mark.parametrize("tuning", [dict(binned=256), dict(binned=256, tail_limit=0),
                                    dict(binned=4096, tail_limit=0, rounds_per_sync=2)])
def test_binned_rounds(which, tuning):
    """Destination-binned rounds (claims, count, scatter, apply through LDS)
    give the same bits as push rounds, under both succession predicates and
    with paths; the rounds really ran (binned edges counted)."""
    from oracle import paths as P
    g, G, se = {"uniform": uniform, "rmat16": rmat16, "bursty16": bursty16, "rmat_wide": rmat_wide,
                "gappy": gappy}[which]()
    name = {"uniform": "uniform-10k", "rmat16": "rmat20-32m", "bursty16": "bursty22-1b",
            "rmat_wide": "rmat22-256m", "gappy": "uniform-10k"}[which]
    old = K.kairos_get_tuning(G)
    try:
        K.kairos_set_tuning(G, **tuning)
        srcs, ta, tw = make_queries(name, g, count=4)
        binned = 0
        for q in range(len(srcs)):
            s, a, w = int(srcs[q]), int(ta[q]), int(tw[q])
            print_case("binned", which, tuning, q)
            K.kairos_profile_enable(G, True)
            K.kairos_profile_read(G)
            got = ea_gpu(G, s, a, w)
            binned += K.kairos_profile_read(G)["binned_edges"]
            K.kairos_profile_enable(G, False)
            want = O.earliest_arrival(se, s, a, w)
            assert np.array_equal(got, want), q
            assert K.kairos_traversed_edges(G, a, w, torch.from_numpy(got.view(np.int32)).cuda()) == \
                O.traversed_edges(se, a, w, want)
            if q == 0:
                _, sea = P.min_hops(g.n, g.src, g.dst, g.t, g.lam, s, a, w, True)
                out = torch.empty(g.n, dtype=torch.int32, device="cuda")
                K.kairos_query(G, K.KAIROS_EARLIEST_ARRIVAL, s, a, w, out, strict=True)
                assert np.array_equal(K.as_u32(out), sea)
                pt, pd = (torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(2))
                K.kairos_earliest_arrival_path(G, s, a, w, out, pt, pd)
                wt, wd = P.ea_predecessors(g.n, g.src, g.dst, g.t, g.lam, s, a, w, want)
                assert np.array_equal(K.as_u32(pt), wt) and np.array_equal(K.as_u32(pd), wd)
        if tuning == dict(binned=256, tail_limit=0) and which in ("uniform", "rmat16", "bursty16"):
            assert binned > 0  # wide windows: large frontiers (the narrow-window graphs may have none)
    finally:
        K.kairos_set_tuning(G, **old)


def test_binned_rounds_scale20_full():
    """All 2^20 vertices (64 bins) with binned rounds from 4096 entries, in
    the benchmark's one-query-per-call form."""
    g, G, se = built("rmat20-full", lambda: make_graph("rmat20-32m"))
    old = K.kairos_get_tuning(G)
    try:
        K.kairos_set_tuning(G, binned=4096)
        srcs, ta, tw = make_queries("rmat20-32m", g)
        for q in range(0, 64, 9):
            print_case("binned full", q)
            assert np.array_equal(ea_gpu(G, int(srcs[q]), int(ta[q]), int(tw[q])),
                                  O.earliest_arrival(se, srcs[q], ta[q], tw[q])), q
    finally:
        K.kairos_set_tuning(G, **old)


@pytest.mark.parametrize("which,count", [("uniform", 16), ("uniform", 130), ("rmat16", 64), ("bursty16", 40),
                                         ("rmat_wide", 100)])
def test_batch_sweep_form(which, count):
    """The sweep form (every edge of the group's windows in departure order,
    a lane per query, slabs fixed up by stamped passes) gives every row of
    the batch bit for bit, on full and ragged groups, first-half and
    log-uniform windows, duplicate sources; repeated calls reuse its state."""
    g, G, se = {"uniform": uniform, "rmat16": rmat16, "bursty16": bursty16, "rmat_wide": rmat_wide}[which]()
    name = {"uniform": "uniform-10k", "rmat16": "rmat20-32m", "bursty16": "bursty22-1b",
            "rmat_wide": "rmat22-256m"}[which]
    srcs, ta, tw = make_queries(name, g, count=count)
    srcs[1] = srcs[0]  # a duplicate source with its own window
    old = K.kairos_get_tuning(G)
    try:
        K.kairos_set_tuning(G, batch_layout=3)
        out = torch.full((count * g.n,), 5, dtype=torch.int32, device="cuda")
        for rep in range(2):
            print_case("sweep batch", which, count, rep)
            K.kairos_profile_enable(G, True)
            K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
            prof = K.kairos_profile_read(G)
            K.kairos_profile_enable(G, False)
            # the sweep itself answered (no hand-over to the lane-dense rounds)
            assert prof["sweep_slabs"] > 0 and prof["sweep_fallbacks"] == 0, prof
            rows = K.as_u32(out).reshape(count, g.n)
            for qi in range(count):
                assert np.array_equal(rows[qi], O.earliest_arrival(se, srcs[qi], ta[qi], tw[qi])), (rep, qi)
    finally:
        K.kairos_set_tuning(G, **old)


def test_batch_sweep_form_small_slabs_settle():
    """Many fix-up passes: on the scale-16 R-MAT graph every slab of the
    sweep form holds 2^20 records, i.e. the whole window in one slab, so
    its chains are settled by fix-up passes alone (the profile shows more
    passes than slabs) and the rows stay exact."""
    g, G, se = rmat16()
    srcs, ta, tw = make_queries("rmat20-32m", g, count=64)
    old = K.kairos_get_tuning(G)
    try:
        K.kairos_set_tuning(G, batch_layout=3)
        out = torch.empty(64 * g.n, dtype=torch.int32, device="cuda")
        K.kairos_profile_enable(G, True)
        K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
        prof = K.kairos_profile_read(G)
        K.kairos_profile_enable(G, False)
        assert prof["sweep_fallbacks"] == 0 and prof["sweep_passes"] > 2 * prof["sweep_slabs"], prof
        rows = K.as_u32(out).reshape(64, g.n)
        for qi in range(0, 64, 7):
            assert np.array_equal(rows[qi], O.earliest_arrival(se, srcs[qi], ta[qi], tw[qi])), qi
    finally:
        K.kairos_set_tuning(G, **old)


@pytest.mark.parametrize("n", [10240, 10241])
def test_small_graph_kernel(n):
    """Graphs of at most 10,240 vertices answer a single earliest-arrival
    query in one workgroup with the query state in LDS (one launch, no
    push / chunk rounds); one vertex more takes the general rounds.  Both
    give the oracle's rows, with and without "Strictly succeeds", and the
    LDS kernel equals the general one-workgroup rounds (tail_limit 0 turns
    it off) on the same graph."""
    from workloads.gen import uniform_graph
    g = uniform_graph(n, 6 * n, 77, 0, 20000, 1, 10)
    G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    rng = np.random.default_rng(n)
    srcs = rng.integers(0, n, 6)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    old = K.kairos_get_tuning(G)
    try:
        for i, s in enumerate(srcs.tolist()):
            a, w = int(rng.integers(0, 5000)), int(rng.integers(10000, 20001))
            print_case("small graph kernel", n, s, a, w)
            K.kairos_profile_enable(G, True)
            K.kairos_earliest_arrival(G, s, a, w, out)
            prof = K.kairos_profile_read(G)
            K.kairos_profile_enable(G, False)
            got = K.as_u32(out).copy()
            assert np.array_equal(got, O.earliest_arrival(se, s, a, w)), (s, a, w)
            if n <= 10240:
                assert prof["launches_tail"] == 1 and prof["launches_push"] == 0, prof
            K.kairos_set_tuning(G, tail_limit=0)
            assert np.array_equal(ea_gpu(G, s, a, w), got)
            K.kairos_set_tuning(G, **old)
            strict = K.as_u32(K.kairos_query(G, 0, s, a, w, out, strict=True)).copy()
            K.kairos_set_tuning(G, tail_limit=0)
            assert np.array_equal(K.as_u32(K.kairos_query(G, 0, s, a, w, out, strict=True)), strict)
            K.kairos_set_tuning(G, **old)
    finally:
        K.kairos_set_tuning(G, **old)
        G.free()
