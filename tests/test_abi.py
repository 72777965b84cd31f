"""The C library loads, exports every function include/kairos.h declares,
and rejects bad arguments on the host before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kairos.h")
LIB = os.path.join(ROOT, "paper_2401_02563_amd", "libkairos.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kairos_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libkairos.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_interface():
    names = declared()
    for need in ("kairos_graph_build", "kairos_earliest_arrival", "kairos_latest_departure",
                 "kairos_fastest", "kairos_earliest_arrival_batch", "kairos_server_create",
                 "kairos_server_submit", "kairos_server_poll", "kairos_server_free"):
        assert need in names
    assert len(names) >= 20


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_argument_errors(lib):
    p = ctypes.c_void_p
    lib.kairos_graph_build.argtypes = [p, p, p, p, ctypes.c_uint64, ctypes.c_uint32, p, ctypes.POINTER(p)]
    lib.kairos_graph_build.restype = ctypes.c_int
    out = p()
    # null out, n == 0, null arrays with m > 0 -> invalid; m >= 2^32 -> range
    assert lib.kairos_graph_build(None, None, None, None, 0, 5, None, None) == 1
    assert lib.kairos_graph_build(None, None, None, None, 0, 0, None, ctypes.byref(out)) == 1
    assert lib.kairos_graph_build(None, None, None, None, 10, 5, None, ctypes.byref(out)) == 1
    dummy = ctypes.c_void_p(16)
    assert lib.kairos_graph_build(dummy, dummy, dummy, dummy, 1 << 32, 5, None, ctypes.byref(out)) == 2
    assert out.value is None
    for fn in ("kairos_earliest_arrival", "kairos_latest_departure", "kairos_fastest"):
        f = getattr(lib, fn)
        f.argtypes = [p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, p]
        f.restype = ctypes.c_int
        assert f(None, 0, 0, 1, dummy) == 1
    lib.kairos_server_create.argtypes = [p, p, ctypes.POINTER(p)]
    assert lib.kairos_server_create(None, None, ctypes.byref(out)) == 1
    lib.kairos_status_string.restype = ctypes.c_char_p
    assert lib.kairos_status_string(0) == b"ok"
    assert lib.kairos_status_string(5) == b"queue full"
    assert lib.kairos_status_string(99) == b"unknown status"
    lib.kairos_graph_free(None)
    lib.kairos_server_free(None)


def test_binding_names_match_header():
    import paper_2401_02563_amd as K
    for n in declared():
        assert hasattr(K, n), n
