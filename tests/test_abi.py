"""C-ABI contract checks that need no GPU: the library loads and exports every
function that ``include/rt.h`` declares, and the binding covers all of them."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt.h")
LIB = os.path.join(ROOT, "paper_2001_11606_amd", "librt.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(rt_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for n in ("rt_build_neighbors", "rt_assemble", "rt_solve", "rt_newton_step"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librt.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2001_11606_amd import rt
    assert sorted(rt.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="librt.so not built")
def test_version_string_without_gpu():
    from paper_2001_11606_amd import rt
    assert "gfx950" in rt.rt_version()
