"""Host-side checks of the seeded workload recipes: the tuning sample is
held out from the timed queries."""
import numpy as np
import pytest

from workloads import CONFIGS, make_graph, make_queries

SHIFT = {"rmat20-32m": 6, "bursty22-1b": 10, "rmat22-256m": 8, "serve-rmat20": 6, "rmat24-512m": 10}


@pytest.mark.parametrize("name", sorted(CONFIGS))
def test_held_out_queries_differ_from_timed_ones(name):
    g = make_graph(name, scale_shift=SHIFT.get(name, 0)) if name != "uniform-10k" else make_graph(name)
    k = min(CONFIGS[name]["queries"], 64)
    s, a, w = make_queries(name, g, count=k)
    hs, ha, hw = make_queries(name, g, count=k, held_out=True)
    # same recipe: same window rule, sources with out-edges
    deg = g.out_degree()
    assert (deg[hs] > 0).all() and (deg[s] > 0).all()
    assert (hw >= ha).all()
    # another seed: the sequences differ, and (source, t_alpha) pairs barely meet
    assert not np.array_equal(s, hs)
    shared = set(zip(s.tolist(), a.tolist())) & set(zip(hs.tolist(), ha.tolist()))
    assert len(shared) <= max(1, k // 16)
    # deterministic
    hs2, ha2, hw2 = make_queries(name, g, count=k, held_out=True)
    assert np.array_equal(hs, hs2) and np.array_equal(ha, ha2) and np.array_equal(hw, hw2)
