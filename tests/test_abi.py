"""The C ABI library loads and exports every function include/gdist.h declares
(CPU only: no compute call is made without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gdist.h")
LIB = os.path.join(ROOT, "paper_2411_11244_amd", "libgdist.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gdist_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("gdist_create", "gdist_destroy", "gdist_build", "gdist_release", "gdist_query",
                 "gdist_query_batch", "gdist_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdist.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdist.so not built")
def test_binding_names_match_header():
    from paper_2411_11244_amd import gdist
    assert sorted(gdist.exported_symbols()) == declared()
    for n in declared():
        assert hasattr(gdist, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdist.so not built")
def test_no_device_fails_loudly():
    """Without a GPU the library reports an error instead of computing
    anything elsewhere."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2411_11244_amd import gdist
    with pytest.raises(gdist.GdistError):
        gdist.gdist_create(0)
