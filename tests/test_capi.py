"""CPU checks of the C ABI: the library loads and exports every declared call,
and the binding's structs match the header's layout."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmz.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbmz_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("lbmz_create", "lbmz_step", "lbmz_decompress_field", "lbmz_stats", "lbmz_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2302_09883_amd import library
    lib = library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_sizes_match_header():
    from paper_2302_09883_amd.lbmz import Grid, Patch, Scheme, Stats
    # sizes of the C structs under the x86-64 SysV ABI
    assert ct.sizeof(Grid) == 4 + 4 + 24 + 4 + 4 + 8
    assert ct.sizeof(Scheme) == 4 + 4 + 24 + 8 + 8 + 8
    assert ct.sizeof(Patch) == 12 + 4 + 4 + 4
    assert ct.sizeof(Stats) == 8 * 5 + 8 + 4 + 4 + 16 * 8 + 8 * 3 + 8


def test_library_fails_loudly_when_missing(tmp_path, monkeypatch):
    import paper_2302_09883_amd.lbmz as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        L.library()
