"""Parity at the benchmark's full sizes and launch configurations.

* rmat20-32m (2^25 edges): every row of the 64-query batch, single queries,
  latest departure / fastest samples, predecessors, hop counts and
  traversed-edge counts, all bit-exact against the oracle.
* bursty22-1b (about 10^9 edges; the largest workload, and the one the
  benchmark times one query per call): earliest arrival of five of its 32
  queries checked by the exact EA certificate, two of them also against the
  oracle's one-pass scan with their traversed-edge counts, and latest
  departure / fastest / shortest duration of one query against the
  oracle's profile scans.
* rmat22-256m (256-query batch) and rmat24-512m (single queries): eight rows
  each by the EA certificate, two of them also against the oracle's scan;
  the scale-24 batch of 64 also in the sweep form, whose rows must equal
  the checked single-query rows.

The certificate (source at t_alpha, a witness edge for every reached
vertex, no usable edge arriving earlier) is exact and needs no sorted copy
of the edges; it runs as one C loop over the edge list."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle as O  # noqa: E402
import paper_2401_02563_amd as K  # noqa: E402
from workloads import make_graph, make_queries  # noqa: E402

_C = {}


def load(name):
    if name not in _C:
        _C.clear()  # keep one large workload in memory at a time
        print(f"case: generating {name}", flush=True)
        g = make_graph(name)
        G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)
        print(f"case: index built for {name} (m={g.m})", flush=True)
        se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
        _C[name] = (g, G, se)
    return _C[name]


def test_rmat20_batch_all_rows_bit_exact():
    g, G, se = load("rmat20-32m")
    srcs, ta, tw = make_queries("rmat20-32m", g)
    out = torch.empty(len(srcs) * g.n, dtype=torch.int32, device="cuda")
    K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
    rows = K.as_u32(out).reshape(len(srcs), g.n)
    for q in range(len(srcs)):
        want = O.earliest_arrival(se, srcs[q], ta[q], tw[q])
        assert np.array_equal(rows[q], want), q
        if q % 16 == 0:
            ec = K.kairos_traversed_edges(G, int(ta[q]), int(tw[q]), out[q * g.n:(q + 1) * g.n])
            assert ec == O.traversed_edges(se, ta[q], tw[q], want)


def test_rmat20_single_and_sweeps():
    g, G, se = load("rmat20-32m")
    srcs, ta, tw = make_queries("rmat20-32m", g)
    one = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for q in range(0, 64, 8):
        print("case: single", q, flush=True)
        K.kairos_earliest_arrival(G, int(srcs[q]), int(ta[q]), int(tw[q]), one)
        assert np.array_equal(K.as_u32(one), O.earliest_arrival(se, srcs[q], ta[q], tw[q])), q
    for q in (1, 2):
        print("case: sweep", q, flush=True)
        pea, pld, pf = O.profile(se, srcs[q], ta[q], tw[q])
        K.kairos_latest_departure(G, int(srcs[q]), int(ta[q]), int(tw[q]), one)
        assert np.array_equal(K.as_u32(one), pld), q
        K.kairos_fastest(G, int(srcs[q]), int(ta[q]), int(tw[q]), one)
        assert np.array_equal(K.as_u32(one), pf), q


def test_rmat20_paths_and_hops():
    """Predecessors and temporal BFS hop counts on the full scale-20 graph
    (two queries; the level-by-level hop oracle takes seconds per query)."""
    from oracle import paths as P
    g, G, se = load("rmat20-32m")
    srcs, ta, tw = make_queries("rmat20-32m", g)
    out, pt, pd = (torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(3))
    for q in (0, 5):
        s, a, w = int(srcs[q]), int(ta[q]), int(tw[q])
        print("case: paths", q, flush=True)
        K.kairos_earliest_arrival_path(G, s, a, w, out, pt, pd)
        want = O.earliest_arrival(se, s, a, w)
        assert np.array_equal(K.as_u32(out), want)
        wt, wd = P.ea_predecessors(g.n, g.src, g.dst, g.t, g.lam, s, a, w, want)
        assert np.array_equal(K.as_u32(pt), wt) and np.array_equal(K.as_u32(pd), wd)
        print("case: hops", q, flush=True)
        K.kairos_temporal_bfs(G, s, a, w, out)
        wh, _ = P.min_hops(g.n, g.src, g.dst, g.t, g.lam, s, a, w)
        assert np.array_equal(K.as_u32(out), wh)


def _spread(k, count):
    """`count` query indices spread over 0..k-1, first and last included."""
    return sorted(set(np.linspace(0, k - 1, count).round().astype(int).tolist()))


@pytest.mark.parametrize("name,kind,cert_rows,scan_rows,sweep_rows,sweep_form", [
    ("bursty22-1b", "single", 5, 2, 1, False),
    ("rmat24-512m", "single", 8, 2, 0, True),
    ("rmat22-256m", "batch", 8, 2, 0, False)])
def test_large_full_size(name, kind, cert_rows, scan_rows, sweep_rows, sweep_form):
    """Earliest arrival at full size in the launch configuration the
    benchmark times (one query per call, or the whole batch in one call):
    `cert_rows` rows by the exact certificate, the first and the middle of
    them (`scan_rows`) also element by element against the oracle's scan
    with their traversed-edge counts; latest departure / fastest / shortest
    duration of `sweep_rows` queries against the oracle's profile scans.
    With `sweep_form`, the whole batch also runs in the sweep form (the
    form the autotuner picks for it) and those rows must equal the checked
    one-query rows bit for bit."""
    _C.clear()
    print(f"case: generating {name}", flush=True)
    g = make_graph(name)
    G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)
    torch.cuda.synchronize()
    srcs, ta, tw = make_queries(name, g)
    rows = _spread(len(srcs), cert_rows)
    scan = [rows[0], rows[len(rows) // 2]][:scan_rows]
    got, counts = {}, {}
    one = torch.empty(g.n, dtype=torch.int32, device="cuda")
    if kind == "batch":
        out = torch.empty(len(srcs) * g.n, dtype=torch.int32, device="cuda")
        print(f"case: {name} batch of {len(srcs)}", flush=True)
        K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
        view = out.view(len(srcs), g.n)
        for q in rows:
            got[q] = K.as_u32(view[q])
            if q in scan:
                counts[q] = K.kairos_traversed_edges(G, int(ta[q]), int(tw[q]), view[q])
        del out, view
    else:
        for q in rows:
            print(f"case: {name} single query {q}", flush=True)
            K.kairos_earliest_arrival(G, int(srcs[q]), int(ta[q]), int(tw[q]), one)
            got[q] = K.as_u32(one)
            if q in scan:
                counts[q] = K.kairos_traversed_edges(G, int(ta[q]), int(tw[q]), one)
    if sweep_form:
        print(f"case: {name} batch of {len(srcs)} in the sweep form", flush=True)
        old = K.kairos_get_tuning(G)
        K.kairos_set_tuning(G, batch_layout=3)
        out = torch.empty(len(srcs) * g.n, dtype=torch.int32, device="cuda")
        K.kairos_profile_enable(G, True)
        K.kairos_earliest_arrival_batch(G, srcs, ta, tw, out)
        prof = K.kairos_profile_read(G)
        K.kairos_profile_enable(G, False)
        K.kairos_set_tuning(G, **old)
        assert prof["sweep_slabs"] > 0 and prof["sweep_fallbacks"] == 0, prof
        view = out.view(len(srcs), g.n)
        for q in rows:
            assert np.array_equal(K.as_u32(view[q]), got[q]), q
        del out, view
    sweeps = {}
    for q in range(1, 1 + sweep_rows):
        print(f"case: {name} latest departure / fastest of query {q}", flush=True)
        K.kairos_latest_departure(G, int(srcs[q]), int(ta[q]), int(tw[q]), one)
        ld = K.as_u32(one)
        K.kairos_fastest(G, int(srcs[q]), int(ta[q]), int(tw[q]), one)
        fa = K.as_u32(one)
        K.kairos_shortest_duration(G, int(srcs[q]), int(ta[q]), int(tw[q]), one)
        sweeps[q] = (ld, fa, K.as_u32(one))
    del one
    G.free()
    torch.cuda.empty_cache()
    a = (g.t.astype(np.uint64) + g.lam).astype(np.uint32)
    for q in rows:
        print(f"case: {name} certificate of query {q}", flush=True)
        assert O.ea_certificate_scan(g.n, g.src, g.dst, g.t, a, int(srcs[q]), int(ta[q]), int(tw[q]), got[q]), q
    del a
    assert max(int((got[q] != 0xFFFFFFFF).sum()) for q in rows) > 1000  # real traversals, not trivial ones
    print(f"case: {name} sorting edges by departure for the oracle", flush=True)
    se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
    for q in scan:
        print(f"case: {name} oracle scan of query {q}", flush=True)
        want = O.earliest_arrival(se, srcs[q], ta[q], tw[q])
        assert np.array_equal(got[q], want), q
        assert counts[q] == O.traversed_edges(se, ta[q], tw[q], want), q
    for q, (ld, fa, sd) in sweeps.items():
        print(f"case: {name} oracle profile of query {q}", flush=True)
        pea, pld, pf = O.profile(se, srcs[q], ta[q], tw[q])
        assert np.array_equal(ld, pld), q
        assert np.array_equal(fa, pf), q
        print(f"case: {name} oracle shortest duration of query {q}", flush=True)
        assert np.array_equal(sd, O.shortest_duration(se, srcs[q], ta[q], tw[q])), q
