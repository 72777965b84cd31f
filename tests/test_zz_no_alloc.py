"""The allocation-free earliest-arrival entry point against the ordinary
one, bit for bit, through the C interface: two calls in a row on a larger
and then a smaller graph (the fixed scratch array keeps the first call's
contents), several sources and windows, a tuning that forces every round
through the multi-block kernels and the chunk list, overlapping calls from
two host threads, and the size limit."""
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2401_02563_amd as K  # noqa: E402
from workloads import Graph, make_graph, make_queries  # noqa: E402


def build(g):
    return K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)


def both(G, s, a, w):
    ref = torch.full((G.n,), 3, dtype=torch.int32, device="cuda")
    got = torch.full((G.n,), 5, dtype=torch.int32, device="cuda")
    K.kairos_earliest_arrival(G, s, a, w, ref)
    K.kairos_earliest_arrival_noalloc(G, s, a, w, got)
    return K.as_u32(ref), K.as_u32(got)


def test_larger_then_smaller_graph():
    big = make_graph("rmat20-32m", scale_shift=4)      # 2^16 vertices, 2^21 edges
    small = make_graph("uniform-10k")                  # 10^4 vertices
    for g, name in ((big, "rmat20-32m"), (small, "uniform-10k")):
        G = build(g)
        srcs, ta, tw = make_queries(name, g, count=6)
        for i in range(len(srcs)):
            print("case: noalloc", name, i, flush=True)
            ref, got = both(G, int(srcs[i]), int(ta[i]), int(tw[i]))
            assert np.array_equal(ref, got), (name, i)
        # the multi-block kernels and the chunk list on every round
        old = K.kairos_get_tuning(G)
        K.kairos_set_tuning(G, tail_limit=0, split=16, chunk=16)
        try:
            ref, got = both(G, int(srcs[0]), int(ta[0]), int(tw[0]))
            assert np.array_equal(ref, got), name
        finally:
            K.kairos_set_tuning(G, **old)
        G.free()


def test_overlapping_calls_from_two_threads():
    g = make_graph("rmat20-32m", scale_shift=6)
    G = build(g)
    srcs, ta, tw = make_queries("rmat20-32m", g, count=8)
    want = []
    for i in range(len(srcs)):
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        K.kairos_earliest_arrival(G, int(srcs[i]), int(ta[i]), int(tw[i]), out)
        want.append(K.as_u32(out))
    outs = [torch.full((g.n,), 9, dtype=torch.int32, device="cuda") for _ in srcs]
    torch.cuda.synchronize()
    errors = []

    def worker(ids):
        try:
            for i in ids:
                K.kairos_earliest_arrival_noalloc(G, int(srcs[i]), int(ta[i]), int(tw[i]), outs[i])
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)

    th = [threading.Thread(target=worker, args=(range(k, len(srcs), 2),)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for i in range(len(srcs)):
        assert np.array_equal(K.as_u32(outs[i]), want[i]), i
    G.free()


def test_size_limit_and_arguments():
    # more vertices than the fixed array holds: a clear error, nothing written
    n = 16 << 20
    g = Graph(n, np.array([0], np.uint32), np.array([1], np.uint32), np.array([5], np.uint32),
              np.array([1], np.uint32), {})
    G = build(g)
    out = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    with pytest.raises(K.KairosError) as e:
        K.kairos_earliest_arrival_noalloc(G, 0, 0, 10, out)
    assert e.value.status == 6
    assert int((out != 7).sum()) == 0
    G.free()
    del out
    g = make_graph("uniform-10k")
    G = build(g)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(K.KairosError) as e:
        K.kairos_earliest_arrival_noalloc(G, g.n, 0, 10, out)
    assert e.value.status == 2
    with pytest.raises(K.KairosError) as e:
        K.kairos_earliest_arrival_noalloc(G, 0, 11, 10, out)
    assert e.value.status == 2
    G.free()
