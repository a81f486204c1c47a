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
