"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the header declares, the binding declares the same set, and
host-side argument validation rejects bad calls before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def _header_functions():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(nnqs_[a-z0-9_]+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_2306_16705_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2306_16705_amd import build
        build.build()
    return _lib.load()


def test_header_declares_entry_points():
    names = _header_functions()
    for required in ("nnqs_system_create", "nnqs_table_build", "nnqs_connections", "nnqs_eloc_table"):
        assert required in names


def test_library_exports_every_header_symbol(lib):
    missing = [n for n in sorted(_header_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2306_16705_amd import _lib
    assert set(_lib.SIGNATURES) == _header_functions()


def test_version_and_error_without_gpu(lib):
    assert b"gfx950" in lib.nnqs_version()
    assert lib.nnqs_last_error() is not None


def _create(lib, N, nu, nd, h=None, g=None):
    K = N // 2
    h = np.zeros((max(K, 1), max(K, 1))) if h is None else h
    g = np.zeros((max(K, 1),) * 4) if g is None else g
    out = ctypes.c_void_p()
    code = lib.nnqs_system_create(ctypes.byref(out), N, nu, nd, h.ctypes.data_as(ctypes.c_void_p),
                                  g.ctypes.data_as(ctypes.c_void_p), 0.0)
    return code, out


@pytest.mark.parametrize("N,nu,nd", [(7, 1, 1), (130, 1, 1), (2, 1, 0), (8, 5, 1), (8, -1, 1)])
def test_system_create_rejects_bad_sizes_on_host(lib, N, nu, nd):
    code, out = _create(lib, N, nu, nd)
    assert code == -1  # NNQS_EINVAL, before any device call
    assert out.value is None
    assert lib.nnqs_last_error()


def test_null_pointers_rejected_on_host(lib):
    assert lib.nnqs_system_create(None, 8, 2, 2, None, None, 0.0) == -1
    out = ctypes.c_void_p()
    assert lib.nnqs_system_create(ctypes.byref(out), 8, 2, 2, None, None, 0.0) == -1
    assert lib.nnqs_table_create(None, None, 10) == -1
    assert lib.nnqs_table_build(None, None, None, None, 1, 0, None) == -1
    assert lib.nnqs_eloc_table(None, None, None, None, None, None, 1, None, None, 0, None) == -1
    assert lib.nnqs_connections(None, None, 1, None, None, None, None, 0, None) == -1
    assert lib.nnqs_connection_count(None) == -1
    assert lib.nnqs_system_destroy(None) == 0
    assert lib.nnqs_table_destroy(None) == 0


def test_tune_cache_on_host(lib, tmp_path):
    """The autotuner cache is plain host file work: store, replace, look up."""
    import paper_2306_16705_amd as nn
    path = str(tmp_path / "tune.txt")
    assert nn.tune_cache_lookup(path, "gfx950:cu256:K24:u6:d6:n65536") is None  # no file yet
    t1 = dict(waves_per_block=16, blocks_per_cu=1, filter_log2_bits=20, splitter_levels=10, search=1,
              tile_samples=256)
    nn.tune_cache_store(path, "gfx950:cu256:K24:u6:d6:n65536", t1, 1.99)
    nn.tune_cache_store(path, "gfx950:cu256:K60:u20:d20:n128", dict(t1, search=2), 7.5)
    t2 = dict(t1, waves_per_block=12)
    nn.tune_cache_store(path, "gfx950:cu256:K24:u6:d6:n65536", t2, 1.80)
    got = nn.tune_cache_lookup(path, "gfx950:cu256:K24:u6:d6:n65536")
    assert got[0] == t2 and abs(got[1] - 1.80) < 1e-9
    assert nn.tune_cache_lookup(path, "gfx950:cu256:K60:u20:d20:n128")[0]["search"] == 2
    with open(path) as f:
        assert len(f.read().splitlines()) == 2
    with pytest.raises(nn.NNQSError):
        nn.tune_cache_store(path, "bad key", t1, 1.0)
    with pytest.raises(nn.NNQSError):
        nn.tune_cache_store(path, "k", dict(t1, search=3), 1.0)
