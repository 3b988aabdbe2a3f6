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


STRUCTS = ("gdist_pose_t", "gdist_result_t", "gdist_query_desc_t", "gdist_mesh_info_t", "gdist_stats_t",
           "gdist_server_config_t", "gdist_completion_t", "gdist_server_stats_t")


def test_struct_layouts_match_binding(tmp_path):
    """Every struct of the header has the size and field offsets the binding
    assumes (the header compiled as C by gcc)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    from paper_2411_11244_amd import gdist
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gdist.h"', "int main(void) {"]
    for name in STRUCTS:
        ct = getattr(gdist, name)
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in ct._fields_:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                         text=True).stdout.splitlines())
    for name in STRUCTS:
        ct = getattr(gdist, name)
        assert int(got[name]) == ctypes.sizeof(ct), name
        for f, _ in ct._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(ct, f).offset, (name, f)
