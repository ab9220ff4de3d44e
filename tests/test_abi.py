"""Host-side checks of the native boundary: the library loads and exports every
entry point that include/miann.h declares. No compute calls (no GPU here)."""
import ctypes
import os
import re

import pytest

import paper_2507_17094_amd as miann

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "miann.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(miann_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("miann_build_graph", "miann_build_ghost", "miann_search", "miann_exact_knn", "miann_index_import"):
        assert s in syms


@pytest.mark.skipif(not os.path.exists(miann.LIB_PATH), reason="libmiann.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(miann.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(miann.EXPORTS) <= set(declared_symbols())


@pytest.mark.skipif(not os.path.exists(miann.LIB_PATH), reason="libmiann.so not built")
def test_version_and_host_side_validation():
    L = miann.load()
    assert b"gfx950" in L.miann_version()
    # argument validation happens before any device work: a null index is rejected
    p = miann.SearchParams()
    L.miann_search_params_default(ctypes.byref(p))
    assert p.search_width == 1 and p.ghost_itopk == 32 and p.discard_permille == 500 and p.stage_waves == 0
    # the binding's layout follows the header: 19 int32 fields, then the 8-byte seed at the next 8-byte boundary
    assert miann.SearchParams.stage_waves.offset == 72 and miann.SearchParams.seed.offset == 80
    rc = L.miann_search(None, None, 0, 10, 64, 10, ctypes.byref(p), None, None, None, None)
    assert rc == 1 and b"null index" in L.miann_last_error()
    rc = L.miann_index_info(None, None, None, None, None, None)
    assert rc == 1


@pytest.mark.skipif(not os.path.exists(miann.LIB_PATH), reason="libmiann.so not built")
def test_index_file_errors_are_host_side(tmp_path):
    """Saving a null index and loading a missing, foreign, truncated or oversized file fail
    with EINVAL before any device call."""
    L = miann.load()
    h = ctypes.c_void_p()
    assert L.miann_index_save(None, str(tmp_path / "x").encode()) == 1
    assert L.miann_index_load(str(tmp_path / "missing").encode(), None, ctypes.byref(h)) == 1
    assert b"cannot open" in L.miann_last_error()
    foreign = tmp_path / "foreign"
    foreign.write_bytes(b"NOTANIDX" + bytes(64))
    assert L.miann_index_load(str(foreign).encode(), None, ctypes.byref(h)) == 1
    assert b"not an index file" in L.miann_last_error()
    import struct
    hdr = b"MIANNIX1" + struct.pack("<I7i", 1, 1, 8, 0, 0, 4, 4, 0)
    # a shard that claims more rows than the file holds
    big = tmp_path / "big"
    big.write_bytes(hdr + struct.pack("<qqi", 1 << 40, 0, 0))
    assert L.miann_index_load(str(big).encode(), None, ctypes.byref(h)) == 1
    assert b"bad shard 0 header" in L.miann_last_error()
    # a shard whose arrays stop early
    short = tmp_path / "short"
    short.write_bytes(hdr + struct.pack("<qqi", 4, 0, 0) + bytes(4 * 8 * 4 + 8))
    assert L.miann_index_load(str(short).encode(), None, ctypes.byref(h)) == 1
    assert b"truncated" in L.miann_last_error()
    assert not h.value
