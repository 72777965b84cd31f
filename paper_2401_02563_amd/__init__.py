"""Python binding of libkairos (temporal minimal-path queries on MI355X).

Thin ctypes marshalling over the C interface declared in include/kairos.h:
the functions keep the C names and pass torch device buffers as raw
pointers.  Every step of a query runs in the library's HIP kernels; there is
no fallback, and importing raises if libkairos.so has not been built.

uint32 data lives in torch.int32 tensors (same bits); helpers below convert.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "KairosError", "Graph", "INF", "TMAX", "lib_path",
    "kairos_graph_build", "kairos_graph_free", "kairos_graph_stats", "kairos_graph_index",
    "kairos_earliest_arrival", "kairos_latest_departure", "kairos_fastest", "kairos_shortest_duration", "kairos_earliest_arrival_noalloc",
    "kairos_earliest_arrival_batch", "kairos_traversed_edges",
    "kairos_get_tuning", "kairos_set_tuning", "kairos_autotune", "kairos_autotune_form",
    "kairos_profile_enable", "kairos_profile_read",
    "kairos_server_create", "kairos_server_submit", "kairos_server_poll", "kairos_server_free",
    "kairos_server_stats_read", "kairos_server_set_free_bytes_override", "kairos_status_string",
    "as_u32", "to_u32_tensor",
]

INF = 0xFFFFFFFF
TMAX = 0xFFFFFFFE
_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libkairos.so")

if not os.path.exists(lib_path):
    raise ImportError(f"{lib_path} is missing: build it with `python -m paper_2401_02563_amd.build`")

_L = ctypes.CDLL(lib_path)
_u32, _u64, _i32, _p = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p


class kairos_tuning(ctypes.Structure):
    _fields_ = [(k, _u32) for k in ("block", "chunk", "split", "pull_alpha", "pull_beta",
                                    "rounds_per_sync", "batch_persistent", "sweep_group", "batch_layout",
                                    "tail_limit", "dense_frontier", "arrival_filter", "single_persistent",
                                    "run_dedupe", "binned")]


class kairos_profile(ctypes.Structure):
    _fields_ = [("launches", _u64 * 7), ("ms", ctypes.c_double * 7), ("edges_scanned", _u64),
                ("chunk_edges", _u64), ("items", _u64), ("relaxations", _u64), ("relax_attempts", _u64), ("tail_edges", _u64),
                ("tail_items", _u64), ("pull_edges", _u64),
                ("pull_vertices", _u64), ("rounds", _u64), ("binned_edges", _u64), ("binned_items", _u64),
                ("sweep_slabs", _u64), ("sweep_passes", _u64), ("sweep_fix_edges", _u64), ("sweep_fallbacks", _u64)]


class kairos_index_view(ctypes.Structure):
    _fields_ = [(k, _p) for k in ("off_out", "t_out", "dst_a_out", "off_in", "a_in", "src_t_in", "perm")] + [
        ("n_live", _u32)]


class kairos_server_opts(ctypes.Structure):
    _fields_ = [("max_slots", _u32), ("queue_capacity", _u32), ("mem_reserve_bytes", _u64),
                ("hip_stream", _p), ("rounds_per_check", _u32)]


class kairos_completion(ctypes.Structure):
    _fields_ = [("ticket", _u64), ("status", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("t_submit_ns", _u64), ("t_done_ns", _u64)]


class kairos_server_stats(ctypes.Structure):
    _fields_ = [("submitted", _u64), ("completed", _u64), ("iterations", _u64),
                ("admitted_waits_mem", _u64), ("active_slots", _u32), ("waiting", _u32),
                ("max_slots_seen", _u32), ("pool_slots", _u32), ("slot_bytes", _u64)]


def _sig(name, res, *args):
    f = getattr(_L, name)  # a missing export is an error at import
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("kairos_graph_build", _i32, _p, _p, _p, _p, _u64, _u32, _p, ctypes.POINTER(_p))
_sig("kairos_graph_free", None, _p)
_sig("kairos_graph_stats", _i32, _p, ctypes.POINTER(_u32), ctypes.POINTER(_u64), ctypes.POINTER(_u64))
_sig("kairos_graph_index", _i32, _p, ctypes.POINTER(kairos_index_view))
for _n in ("kairos_earliest_arrival", "kairos_latest_departure", "kairos_fastest", "kairos_temporal_bfs",
           "kairos_latest_departure_to", "kairos_shortest_duration", "kairos_earliest_arrival_noalloc"):
    _sig(_n, _i32, _p, _u32, _u32, _u32, _p)
_sig("kairos_earliest_arrival_path", _i32, _p, _u32, _u32, _u32, _p, _p, _p)
_sig("kairos_query", _i32, _p, _i32, _u32, _u32, _u32, _u32, _p)
KAIROS_EARLIEST_ARRIVAL, KAIROS_LATEST_DEPARTURE, KAIROS_FASTEST, KAIROS_TEMPORAL_BFS = 0, 1, 2, 3
KAIROS_LATEST_DEPARTURE_TO = 4
KAIROS_SHORTEST_DURATION = 5
KAIROS_STRICT = 1
_sig("kairos_earliest_arrival_batch", _i32, _p, _u32, _p, _p, _p, _p)
_sig("kairos_traversed_edges", _i32, _p, _u32, _u32, _p, ctypes.POINTER(_u64))
_sig("kairos_get_tuning", _i32, _p, ctypes.POINTER(kairos_tuning))
_sig("kairos_set_tuning", _i32, _p, ctypes.POINTER(kairos_tuning))
_sig("kairos_autotune", _i32, _p, _u32, _p, _p, _p, ctypes.POINTER(kairos_tuning))
_sig("kairos_autotune_form", _i32, _p, _i32, _u32, _p, _p, _p, ctypes.POINTER(kairos_tuning))
_sig("kairos_profile_enable", _i32, _p, _i32)
_sig("kairos_profile_read", _i32, _p, ctypes.POINTER(kairos_profile))
_sig("kairos_server_create", _i32, _p, ctypes.POINTER(kairos_server_opts), ctypes.POINTER(_p))
_sig("kairos_server_submit", _i32, _p, _i32, _u32, _u32, _u32, _p, ctypes.POINTER(_u64))
_sig("kairos_server_poll", _i32, _p, ctypes.POINTER(kairos_completion), _u32, ctypes.POINTER(_u32))
_sig("kairos_server_free", None, _p)
_sig("kairos_server_stats_read", _i32, _p, ctypes.POINTER(kairos_server_stats))
_sig("kairos_server_set_free_bytes_override", _i32, _p, _u64)
_sig("kairos_status_string", ctypes.c_char_p, _i32)


class KairosError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {kairos_status_string(status)} ({status})")


def kairos_status_string(status: int) -> str:
    return _L.kairos_status_string(int(status)).decode()


def _check(rc: int, what: str):
    if rc != 0:
        raise KairosError(rc, what)


def as_u32(t: torch.Tensor):
    """numpy uint32 view of an int32 tensor (copied to host)."""
    return t.detach().cpu().numpy().view("uint32")


def to_u32_tensor(a, device="cuda") -> torch.Tensor:
    """Device int32 tensor holding the bits of a uint32 array."""
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).to(device)


def _dev_ptr(t: torch.Tensor, n: int | None = None, what="tensor") -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if t.dtype not in (torch.int32, torch.uint32) or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous 32-bit tensor")
    if n is not None and t.numel() < n:
        raise ValueError(f"{what} needs {n} entries, has {t.numel()}")
    return t.data_ptr()


def _sync():
    torch.cuda.current_stream().synchronize()


class Graph:
    """Owning wrapper of a kairos_graph handle."""

    def __init__(self, handle: int, n: int, m: int):
        self.handle = handle
        self.n = n
        self.m = m

    def free(self):
        if self.handle:
            _L.kairos_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def kairos_graph_build(src: torch.Tensor, dst: torch.Tensor, t: torch.Tensor, lam: torch.Tensor,
                       n: int, stream=None) -> Graph:
    m = src.numel()
    ptrs = [(_dev_ptr(x, m, nm) if m else None) for x, nm in ((src, "src"), (dst, "dst"), (t, "t"), (lam, "lambda"))]
    _sync()
    h = _p()
    _check(_L.kairos_graph_build(*ptrs, m, n, stream, ctypes.byref(h)), "kairos_graph_build")
    return Graph(h.value, n, m)


def kairos_graph_free(g: Graph):
    g.free()


def kairos_graph_stats(g: Graph):
    n, m, b = _u32(), _u64(), _u64()
    _check(_L.kairos_graph_stats(g.handle, ctypes.byref(n), ctypes.byref(m), ctypes.byref(b)),
           "kairos_graph_stats")
    return n.value, m.value, b.value


def _copy_from_device(ptr: int, count: int) -> torch.Tensor:
    """Copy `count` uint32 words at device address `ptr` into a new device tensor."""
    out = torch.empty(max(count, 1), dtype=torch.int32, device="cuda")
    if count:
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [_p, _p, ctypes.c_size_t, ctypes.c_int]
        hip.hipMemcpy.restype = ctypes.c_int
        rc = hip.hipMemcpy(out.data_ptr(), ptr, count * 4, 3)  # device to device
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out[:count]


def kairos_graph_index(g: Graph) -> dict:
    """Copies of the index arrays as device int32 tensors."""
    v = kairos_index_view()
    _check(_L.kairos_graph_index(g.handle, ctypes.byref(v)), "kairos_graph_index")
    n, m = g.n, g.m
    return dict(off_out=_copy_from_device(v.off_out, n + 1), t_out=_copy_from_device(v.t_out, m),
                dst_a_out=_copy_from_device(v.dst_a_out, 2 * m), off_in=_copy_from_device(v.off_in, n + 1),
                a_in=_copy_from_device(v.a_in, m), src_t_in=_copy_from_device(v.src_t_in, 2 * m),
                perm=_copy_from_device(v.perm, n), n_live=int(v.n_live))


def _single(name, g, src, ta, tw, out):
    p = _dev_ptr(out, g.n, "out")
    _sync()
    _check(getattr(_L, name)(g.handle, int(src), int(ta), int(tw), p), name)
    return out


def kairos_earliest_arrival(g: Graph, src: int, t_alpha: int, t_omega: int, out: torch.Tensor):
    return _single("kairos_earliest_arrival", g, src, t_alpha, t_omega, out)


def kairos_latest_departure(g: Graph, src: int, t_alpha: int, t_omega: int, out: torch.Tensor):
    return _single("kairos_latest_departure", g, src, t_alpha, t_omega, out)


def kairos_fastest(g: Graph, src: int, t_alpha: int, t_omega: int, out: torch.Tensor):
    return _single("kairos_fastest", g, src, t_alpha, t_omega, out)


def kairos_latest_departure_to(g: Graph, target: int, t_alpha: int, t_omega: int, out: torch.Tensor):
    return _single("kairos_latest_departure_to", g, target, t_alpha, t_omega, out)


def kairos_temporal_bfs(g: Graph, src: int, t_alpha: int, t_omega: int, out: torch.Tensor):
    return _single("kairos_temporal_bfs", g, src, t_alpha, t_omega, out)


def kairos_shortest_duration(g: Graph, src: int, t_alpha: int, t_omega: int, out: torch.Tensor):
    return _single("kairos_shortest_duration", g, src, t_alpha, t_omega, out)


def kairos_earliest_arrival_noalloc(g: Graph, src: int, t_alpha: int, t_omega: int, out: torch.Tensor):
    return _single("kairos_earliest_arrival_noalloc", g, src, t_alpha, t_omega, out)


def kairos_query(g: Graph, kind: int, src: int, t_alpha: int, t_omega: int, out: torch.Tensor,
                 strict: bool = False):
    p = _dev_ptr(out, g.n, "out")
    _sync()
    _check(_L.kairos_query(g.handle, int(kind), KAIROS_STRICT if strict else 0, int(src), int(t_alpha),
                           int(t_omega), p), "kairos_query")
    return out


def kairos_earliest_arrival_path(g: Graph, src: int, t_alpha: int, t_omega: int, out: torch.Tensor,
                                 pred_tail: torch.Tensor, pred_departure: torch.Tensor):
    p = [_dev_ptr(x, g.n, w) for x, w in ((out, "out"), (pred_tail, "pred_tail"),
                                          (pred_departure, "pred_departure"))]
    _sync()
    _check(_L.kairos_earliest_arrival_path(g.handle, int(src), int(t_alpha), int(t_omega), *p),
           "kairos_earliest_arrival_path")
    return out, pred_tail, pred_departure


def _host_u32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(_p)


def kairos_earliest_arrival_batch(g: Graph, src, t_alpha, t_omega, out: torch.Tensor):
    s, ps = _host_u32(src)
    a, pa = _host_u32(t_alpha)
    w, pw = _host_u32(t_omega)
    q = len(s)
    if not (len(a) == len(w) == q):
        raise ValueError("src, t_alpha, t_omega differ in length")
    p = _dev_ptr(out, q * g.n, "out") if q else None
    _sync()
    _check(_L.kairos_earliest_arrival_batch(g.handle, q, ps, pa, pw, p), "kairos_earliest_arrival_batch")
    return out


def kairos_traversed_edges(g: Graph, t_alpha: int, t_omega: int, ea: torch.Tensor) -> int:
    c = _u64()
    _sync()
    _check(_L.kairos_traversed_edges(g.handle, int(t_alpha), int(t_omega), _dev_ptr(ea, g.n, "ea"),
                                     ctypes.byref(c)), "kairos_traversed_edges")
    return c.value


def kairos_get_tuning(g: Graph) -> dict:
    t = kairos_tuning()
    _check(_L.kairos_get_tuning(g.handle, ctypes.byref(t)), "kairos_get_tuning")
    return {k: getattr(t, k) for k, _ in t._fields_}


def kairos_set_tuning(g: Graph, **kw):
    cur = kairos_get_tuning(g)
    cur.update(kw)
    t = kairos_tuning(**cur)
    _check(_L.kairos_set_tuning(g.handle, ctypes.byref(t)), "kairos_set_tuning")
    return cur


def kairos_autotune(g: Graph, src, t_alpha, t_omega) -> dict:
    s, ps = _host_u32(src)
    a, pa = _host_u32(t_alpha)
    w, pw = _host_u32(t_omega)
    t = kairos_tuning()
    _sync()
    _check(_L.kairos_autotune(g.handle, len(s), ps, pa, pw, ctypes.byref(t)), "kairos_autotune")
    return {k: getattr(t, k) for k, _ in t._fields_}


KAIROS_TUNE_SINGLE, KAIROS_TUNE_BATCH = 0, 1


def kairos_autotune_form(g: Graph, form: int, src, t_alpha, t_omega) -> dict:
    s, ps = _host_u32(src)
    a, pa = _host_u32(t_alpha)
    w, pw = _host_u32(t_omega)
    t = kairos_tuning()
    _sync()
    _check(_L.kairos_autotune_form(g.handle, int(form), len(s), ps, pa, pw, ctypes.byref(t)),
           "kairos_autotune_form")
    return {k: getattr(t, k) for k, _ in t._fields_}


def kairos_profile_enable(g: Graph, on: bool = True):
    _check(_L.kairos_profile_enable(g.handle, 1 if on else 0), "kairos_profile_enable")


def kairos_profile_read(g: Graph) -> dict:
    p = kairos_profile()
    _check(_L.kairos_profile_read(g.handle, ctypes.byref(p)), "kairos_profile_read")
    names = ["push", "pull", "init", "sort", "chunk", "tail", "binned"]
    d = {f"launches_{k}": p.launches[i] for i, k in enumerate(names)}
    d.update({f"ms_{k}": p.ms[i] for i, k in enumerate(names)})
    for k in ("edges_scanned", "chunk_edges", "tail_edges", "tail_items", "items", "relaxations", "relax_attempts", "pull_edges", "pull_vertices", "rounds", "binned_edges", "binned_items",
              "sweep_slabs", "sweep_passes", "sweep_fix_edges", "sweep_fallbacks"):
        d[k] = getattr(p, k)
    return d


class Server:
    def __init__(self, handle: int, graph: Graph):
        self.handle = handle
        self.graph = graph

    def free(self):
        if self.handle:
            _L.kairos_server_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def kairos_server_create(g: Graph, max_slots=32, queue_capacity=1 << 16, mem_reserve_bytes=0,
                         stream=None, rounds_per_check=0) -> Server:
    o = kairos_server_opts(max_slots, queue_capacity, mem_reserve_bytes, stream, rounds_per_check)
    h = _p()
    _check(_L.kairos_server_create(g.handle, ctypes.byref(o), ctypes.byref(h)), "kairos_server_create")
    return Server(h.value, g)


def kairos_server_submit(s: Server, kind: int, src: int, t_alpha: int, t_omega: int,
                         out: torch.Tensor) -> int:
    """Returns the ticket; raises KairosError (status BUSY when the queue is full)."""
    tk = _u64()
    _check(_L.kairos_server_submit(s.handle, int(kind), int(src), int(t_alpha), int(t_omega),
                                   _dev_ptr(out, s.graph.n, "out"), ctypes.byref(tk)), "kairos_server_submit")
    return tk.value


def kairos_server_poll(s: Server, cap: int = 1024):
    arr = (kairos_completion * cap)()
    nd = _u32()
    _check(_L.kairos_server_poll(s.handle, arr, cap, ctypes.byref(nd)), "kairos_server_poll")
    return [dict(ticket=c.ticket, status=c.status, kind=c.kind, t_submit_ns=c.t_submit_ns,
                 t_done_ns=c.t_done_ns) for c in arr[:nd.value]]


def kairos_server_free(s: Server):
    s.free()


def kairos_server_stats_read(s: Server) -> dict:
    st = kairos_server_stats()
    _check(_L.kairos_server_stats_read(s.handle, ctypes.byref(st)), "kairos_server_stats_read")
    return {k: getattr(st, k) for k, _ in st._fields_}


def kairos_server_set_free_bytes_override(s: Server, nbytes: int):
    _check(_L.kairos_server_set_free_bytes_override(s.handle, int(nbytes)),
           "kairos_server_set_free_bytes_override")
