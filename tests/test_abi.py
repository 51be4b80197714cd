"""The C-ABI library loads and exports every symbol include/gdm.h declares;
null contexts and null arguments are rejected on the host (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gdm.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gdm_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_hot_path():
    names = declared()
    for need in ("gdm_build_graph", "gdm_extract_subgraphs", "gdm_subgraph_density", "gdm_find_mu",
                 "gdm_mulliken_charges", "gdm_grid_cores", "gdm_build_hs", "gdm_plan", "gdm_create"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2606_03140_amd._lib import LIB_PATH, load_library
    assert os.path.exists(LIB_PATH), "build libgdm first (python -m paper_2606_03140_amd.build)"
    lib = C.CDLL(LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    load_library()   # signatures bind


def test_null_context_rejected_on_host():
    from paper_2606_03140_amd._lib import load_library
    lib = load_library()
    assert lib.gdm_destroy(None) == -1
    assert lib.gdm_check(None) == -1
    assert lib.gdm_last_error(None) == b"null context"
    assert lib.gdm_plan(None, None, 0) == -1
    assert lib.gdm_set_stream(None, None) == -1
    out = C.c_void_p()
    assert lib.gdm_create(None, 0, None) == -1
