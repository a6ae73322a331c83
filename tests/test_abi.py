"""The C-ABI library loads and exports every entry point include/g3.h
declares (no compute call: these tests run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "g3.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(g3_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("g3_build_tree", "g3_walk", "g3_density", "g3_hydro_force", "g3_gravity"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2003_10850_amd import g3
    if not os.path.exists(g3.LIB_PATH):
        pytest.fail("libg3.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(g3.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    assert sorted(g3.EXPORTS) == declared()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2003_10850_amd import g3
    monkeypatch.setattr(g3, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(g3, "_lib", None)
    with pytest.raises(ImportError):
        g3.lib()


def test_params_struct_layout():
    from paper_2003_10850_amd import g3
    # 7 doubles + 2 int32, no padding: the C struct is 64 bytes
    assert ctypes.sizeof(g3.g3_params) == 64
