"""Continuous-batching server: results equal the same query run alone and the
CPU oracle (bit for bit), admission waits for device memory, the waiting
queue is bounded, slots are reused without stale state."""
import threading
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle as O  # noqa: E402
import paper_2401_02563_amd as K  # noqa: E402
from workloads import make_graph, query_kinds  # noqa: E402
from workloads.gen import log_uniform_windows, sample_sources  # noqa: E402

_G = {}


def graph(name, shift):
    key = (name, shift)
    if key not in _G:
        g = make_graph(name, scale_shift=shift)
        G = K.kairos_graph_build(*[K.to_u32_tensor(x) for x in (g.src, g.dst, g.t, g.lam)], g.n)
        se = O.sort_by_departure(g.n, g.src, g.dst, g.t, g.lam)
        _G[key] = (g, G, se)
    return _G[key]


def mixed_queries(g, count, seed, t_lo, t_hi):
    src = sample_sources(g, count, seed)
    ta, tw = log_uniform_windows(count, t_lo, t_hi, seed + 1, f_lo_exp=-1.5)
    kinds = query_kinds(count, seed + 2)
    return src, ta, tw, kinds


def drain(srv, want, timeout=120.0):
    got = {}
    t0 = time.time()
    while len(got) < want:
        for c in K.kairos_server_poll(srv, 512):
            got[c["ticket"]] = c
        if time.time() - t0 > timeout:
            raise TimeoutError(f"only {len(got)} of {want} completions")
        time.sleep(0.0005)
    return got


def expected(se, kind, s, a, w):
    ea, ld, fa = O.profile(se, s, a, w)
    return (ea, ld, fa)[kind]


@pytest.mark.parametrize("name,shift,t_lo,t_hi,codes,rpc,group", [
    ("uniform-10k", 0, 0, 99_999, None, 0, None),
    ("uniform-10k", 0, 0, 99_999, None, 1, 1),
    ("uniform-10k", 0, 0, 99_999, None, 5, 3),
    ("rmat20-32m", 6, 0, (1 << 30) - 1, None, 0, None),
    ("rmat20-32m", 6, 0, (1 << 30) - 1, 2, 3, 1)])
def test_mixed_stream_equals_alone_and_oracle(name, shift, t_lo, t_hi, codes, rpc, group):
    g, G, se = graph(name, shift)
    print("case: mixed stream", name, shift, codes, rpc, group, flush=True)
    old = K.kairos_get_tuning(G)
    if codes is not None:
        K.kairos_set_tuning(G, arrival_filter=codes)
    if group is not None:
        K.kairos_set_tuning(G, sweep_group=group)
    try:
        _mixed_stream(g, G, se, t_lo, t_hi, rpc)
    finally:
        K.kairos_set_tuning(G, **old)


def _mixed_stream(g, G, se, t_lo, t_hi, rpc):
    count = 120
    src, ta, tw, kinds = mixed_queries(g, count, 7, t_lo, t_hi)
    outs = torch.full((count, g.n), 7, dtype=torch.int32, device="cuda")
    srv = K.kairos_server_create(G, max_slots=8, queue_capacity=4096, rounds_per_check=rpc)
    tickets = {}

    def producer():
        # arrivals in bursts while earlier queries are on the device
        for i in range(count):
            tickets[K.kairos_server_submit(srv, int(kinds[i]), int(src[i]), int(ta[i]), int(tw[i]), outs[i])] = i
            if i % 10 == 9:
                time.sleep(0.002)

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    done = drain(srv, count)
    st = K.kairos_server_stats_read(srv)
    K.kairos_server_free(srv)
    assert st["completed"] == count and st["max_slots_seen"] >= 2, st
    alone = torch.empty(g.n, dtype=torch.int32, device="cuda")
    fns = (K.kairos_earliest_arrival, K.kairos_latest_departure, K.kairos_fastest)
    for tk, c in done.items():
        i = tickets[tk]
        assert c["status"] == 0 and c["kind"] == kinds[i]
        assert c["t_done_ns"] >= c["t_submit_ns"]
        mixed = K.as_u32(outs[i])
        fns[kinds[i]](G, int(src[i]), int(ta[i]), int(tw[i]), alone)
        assert np.array_equal(mixed, K.as_u32(alone)), (i, kinds[i])
        assert np.array_equal(mixed, expected(se, int(kinds[i]), src[i], ta[i], tw[i])), (i, kinds[i])


def test_admission_waits_for_memory_and_queue_is_bounded():
    g, G, se = graph("uniform-10k", 0)
    srv = K.kairos_server_create(G, max_slots=4, queue_capacity=3)
    K.kairos_server_set_free_bytes_override(srv, 0)
    outs = torch.empty((4, g.n), dtype=torch.int32, device="cuda")
    src = sample_sources(g, 4, 3)
    for i in range(3):
        K.kairos_server_submit(srv, 0, int(src[i]), 0, 99_999, outs[i])
    with pytest.raises(K.KairosError) as ei:
        K.kairos_server_submit(srv, 0, int(src[3]), 0, 99_999, outs[3])
    assert ei.value.status == 5  # queue full
    time.sleep(0.05)
    assert K.kairos_server_poll(srv) == []
    st = K.kairos_server_stats_read(srv)
    assert st["admitted_waits_mem"] > 0 and st["completed"] == 0
    K.kairos_server_set_free_bytes_override(srv, (1 << 64) - 1)  # real device memory again
    done = drain(srv, 3)
    assert all(c["status"] == 0 for c in done.values())
    for i in range(3):
        assert np.array_equal(K.as_u32(outs[i]), O.earliest_arrival(se, src[i], 0, 99_999))
    with pytest.raises(K.KairosError) as ei:
        K.kairos_server_submit(srv, 0, g.n, 0, 5, outs[0])
    assert ei.value.status == 2
    K.kairos_server_free(srv)


def test_pool_growth_charges_the_transient_peak():
    """Growing the slot pool from k to k' slots allocates the new pool while
    the old one is live, so it needs k' slots' worth of free memory, not
    k' - k.  With room for six slots the pool grows to four but not to
    eight; the queries still all finish, four at a time."""
    g, G, se = graph("uniform-10k", 0)
    srv = K.kairos_server_create(G, max_slots=8, queue_capacity=64)
    K.kairos_server_set_free_bytes_override(srv, 0)
    k = 12
    src = sample_sources(g, k, 5)
    outs = torch.empty((k, g.n), dtype=torch.int32, device="cuda")
    for i in range(k):
        K.kairos_server_submit(srv, 0, int(src[i]), 0, 99_999, outs[i])
    time.sleep(0.05)
    st = K.kairos_server_stats_read(srv)
    assert st["completed"] == 0 and st["pool_slots"] == 0 and st["slot_bytes"] > 0, st
    K.kairos_server_set_free_bytes_override(srv, 6 * st["slot_bytes"])
    drain(srv, k)
    st = K.kairos_server_stats_read(srv)
    K.kairos_server_free(srv)
    assert st["pool_slots"] == 4 and st["admitted_waits_mem"] > 0, st
    for i in range(k):
        assert np.array_equal(K.as_u32(outs[i]), O.earliest_arrival(se, src[i], 0, 99_999)), i


def test_slot_reuse_has_no_stale_state():
    """One slot, queries alternating between wide and narrow windows: each
    result must match its own oracle, so nothing leaks from the previous
    occupant of the slot."""
    g, G, se = graph("uniform-10k", 0)
    srv = K.kairos_server_create(G, max_slots=1, queue_capacity=64)
    k = 12
    src = sample_sources(g, k, 11)
    ta = np.array([0 if i % 2 == 0 else 60_000 for i in range(k)], np.uint32)
    tw = np.array([99_999 if i % 2 == 0 else 61_000 for i in range(k)], np.uint32)
    kinds = np.array([i % 3 for i in range(k)])
    outs = torch.empty((k, g.n), dtype=torch.int32, device="cuda")
    tickets = {K.kairos_server_submit(srv, int(kinds[i]), int(src[i]), int(ta[i]), int(tw[i]), outs[i]): i
               for i in range(k)}
    drain(srv, k)
    K.kairos_server_free(srv)
    for i in tickets.values():
        assert np.array_equal(K.as_u32(outs[i]), expected(se, int(kinds[i]), src[i], ta[i], tw[i])), i


@pytest.mark.parametrize("rpc,group,slots", [(1, 0, 3), (4, 0, 3), (2, 1, 3), (3, 2, 8), (4, 8, 16)])
def test_sweeps_with_no_and_many_departures(rpc, group, slots):
    """Latest departure and fastest through the server for sources whose
    departure list is empty (no out-edges, or a window no edge fits) and for
    the source with the most out-edges (the longest step list), mixed with
    earliest-arrival queries; each equals the oracle.  Sweeps step on one
    slot (group 1) or run groups of departure times on consecutive slots,
    also with fewer free slots than the group width."""
    g, G, se = graph("uniform-10k", 0)
    print("case: sweep departures", rpc, group, slots, flush=True)
    old = K.kairos_get_tuning(G)
    if group:
        K.kairos_set_tuning(G, sweep_group=group)
    try:
        _sweep_departures(g, G, se, rpc, slots)
    finally:
        K.kairos_set_tuning(G, **old)


def _sweep_departures(g, G, se, rpc, slots):
    outdeg = np.bincount(g.src, minlength=g.n)
    hub = int(np.argmax(outdeg))
    cases = [(1, hub, 0, 99_999), (2, hub, 0, 99_999), (1, hub, 40_000, 99_999), (2, hub, 99_990, 99_999),
             (1, hub, 50_000, 50_001), (0, hub, 0, 99_999)]
    lonely = np.flatnonzero(outdeg == 0)
    if lonely.size:
        cases += [(1, int(lonely[0]), 0, 99_999), (2, int(lonely[0]), 0, 99_999)]
    srv = K.kairos_server_create(G, max_slots=slots, queue_capacity=64, rounds_per_check=rpc)
    outs = torch.full((len(cases), g.n), 7, dtype=torch.int32, device="cuda")
    tickets = {K.kairos_server_submit(srv, k, s_, a, w, outs[i]): i for i, (k, s_, a, w) in enumerate(cases)}
    done = drain(srv, len(cases))
    K.kairos_server_free(srv)
    for tk, c in done.items():
        i = tickets[tk]
        k, s_, a, w = cases[i]
        assert c["status"] == 0
        assert np.array_equal(K.as_u32(outs[i]), expected(se, k, s_, a, w)), cases[i]


def test_served_mix_on_the_full_scale20_graph():
    """The serving workload at full size: 240 queries of the 60/20/20
    earliest-arrival / latest-departure / fastest mix with log-uniform
    windows on the whole rmat20-32m graph, arriving as a Poisson stream at
    5,000 q/s while earlier ones are on the device.  Every served result
    equals the same query run alone; every earliest-arrival result and
    twelve latest-departure / fastest results also equal the oracle."""
    from workloads import make_queries, poisson_arrivals
    from workloads.configs import make_kinds
    g, G, se = graph("rmat20-32m", 0)
    count = 240
    src, ta, tw = make_queries("serve-rmat20", g, count)
    kinds = make_kinds("serve-rmat20", count)
    assert (kinds == 0).sum() > 100 and (kinds == 1).sum() > 20 and (kinds == 2).sum() > 20
    arrive = poisson_arrivals(5_000, count, 105)
    outs = torch.full((count, g.n), 7, dtype=torch.int32, device="cuda")
    srv = K.kairos_server_create(G, max_slots=64, queue_capacity=4096)
    tickets = {}
    print("case: served mix on rmat20-32m", flush=True)
    t0 = time.monotonic()
    for i in range(count):
        while time.monotonic() - t0 < arrive[i]:
            time.sleep(0.0001)
        tickets[K.kairos_server_submit(srv, int(kinds[i]), int(src[i]), int(ta[i]), int(tw[i]), outs[i])] = i
    done = drain(srv, count, timeout=300.0)
    st = K.kairos_server_stats_read(srv)
    K.kairos_server_free(srv)
    assert st["completed"] == count and st["max_slots_seen"] >= 2, st
    alone = torch.empty(g.n, dtype=torch.int32, device="cuda")
    fns = (K.kairos_earliest_arrival, K.kairos_latest_departure, K.kairos_fastest)
    profiled = 0
    for tk, c in sorted(done.items()):
        i = tickets[tk]
        assert c["status"] == 0 and c["kind"] == kinds[i]
        mixed = K.as_u32(outs[i])
        fns[kinds[i]](G, int(src[i]), int(ta[i]), int(tw[i]), alone)
        assert np.array_equal(mixed, K.as_u32(alone)), (i, kinds[i])
        if kinds[i] == 0:
            assert np.array_equal(mixed, O.earliest_arrival(se, src[i], ta[i], tw[i])), i
        elif profiled < 12:
            profiled += 1
            assert np.array_equal(mixed, expected(se, int(kinds[i]), src[i], ta[i], tw[i])), (i, kinds[i])
    assert profiled == 12
