"""The C-ABI library loads on the CPU and exports every symbol its header declares."""
import ctypes
import os
import re

from paper_1812_04719_amd import stiv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(stiv_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported():
    names = declared("stiv.h")
    assert "stiv_detect" in names and "stiv_create" in names
    lib = ctypes.CDLL(stiv.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) <= set(stiv.EXPORTS)


def test_binding_loads_library():
    L = stiv.lib()
    assert L.stiv_last_error(None) == b"null context"


def test_mlp_nparam_matches_layout():
    """The bracket model's parameter count (host-only call, no GPU work)."""
    from paper_1812_04719_amd import toi_model
    assert stiv.mlp_nparam() == toi_model.layout()[1] == 18 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2
