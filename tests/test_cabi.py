"""The C-ABI library loads on the CPU host and exports every entry point that
include/mpg.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mpg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for n in ["sample_seeds", "manifold_walk_batch", "estimate_inv_prob", "fit_guide", "manifold_walk_adjoint",
              "mpg_scene_create", "mpg_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2311_12818_amd as M
    if not os.path.exists(M.LIB_PATH):
        from paper_2311_12818_amd import build
        build.build()
    lib = ctypes.CDLL(M.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_errors_without_gpu():
    """Argument checks run on the host before any device work."""
    import paper_2311_12818_amd as M
    L = M.lib()
    p = M.mpg_walk_params()
    assert L.mpg_walk_params_default(0.0, ctypes.byref(p)) == -1
    assert b"bad argument" in L.mpg_last_error()
    assert L.mpg_walk_params_default(2.0, ctypes.byref(p)) == 0
    assert p.max_iter == 20 and abs(p.tol_vertex - 1e-4) < 1e-9 and p.max_len == 8
    assert L.manifold_walk_batch(None, ctypes.byref(p), None, None, None, None, None, None, None) == -1
    assert L.sample_seeds(None, None, None, None, 0, 0, 0.5, None, None, None, None) == -1


def test_ctypes_structs_match_the_header_layout(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (compiled with the host C compiler)."""
    import shutil
    import subprocess
    import paper_2311_12818_amd as M
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = [M.mpg_heightfield, M.mpg_scene_desc, M.mpg_endpoints, M.mpg_chains, M.mpg_walk_out,
               M.mpg_walk_params, M.mpg_guide_desc, M.mpg_stree_desc]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "mpg.h"', "int main(void) {"]
    expect = []
    for S in structs:
        name = S.__name__
        lines.append('printf("%%zu\\n", sizeof(%s));' % name)
        expect.append(ctypes.sizeof(S))
        for field in S._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (name, field[0]))
            expect.append(getattr(S, field[0]).offset)
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == expect


def test_length_order_default_and_packing():
    import paper_2311_12818_amd as M
    p = M.walk_params(2.0)
    assert p.length_order == 0
    assert M.pack_length_order([8, 7, 6, 5, 4, 3, 2, 1]) == 0x12345678
    assert M.walk_params(2.0, length_order=[3, 8, 7, 6, 5, 4, 2, 1]).length_order == 0x12456783
    with pytest.raises(ValueError):
        M.pack_length_order([1, 1, 2, 3, 4, 5, 6, 7])
