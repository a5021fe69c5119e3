"""The C-ABI library loads and exports every function include/*.h declares (CPU only;
no compute call is made without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*\b((?:props|train|serve)_[A-Za-z0-9_]*)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("props_mech_create", "props_mech_destroy", "props_pr", "props_diffusion", "props_dnn",
                 "props_dnn_features", "props_dnn_set_log_outputs", "props_features_hpz", "train_dnn",
                 "serve_create", "props_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2312_04830_amd as P
    L = ctypes.CDLL(P.library_path)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_error_path_without_gpu():
    """Argument validation happens on the host before any HIP call."""
    import paper_2312_04830_amd as P
    L = P.lib()
    h = ctypes.c_void_p()
    assert L.props_mech_create(None, 2, None, ctypes.byref(h)) == -1
    assert b"NULL" in L.props_last_error()
    assert L.props_pr(None, 0, 0, None, None, 10, None, None) == -1
    assert L.props_version().startswith(b"props-mi355x")
    assert L.props_diffusion(None, 0, None, None, None, None, 10, None, None) == -1
    assert b"null mechanism" in L.props_last_error()
    assert L.props_dnn_set_log_outputs(None, 0x3F) == -1
