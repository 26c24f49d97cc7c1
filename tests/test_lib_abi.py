"""The C-ABI library loads and exports every function include/eipc.h
declares; host-side checks that need no GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eipc.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eipc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["eipc_create", "eipc_destroy", "eipc_build_candidates", "eipc_barrier_reduce",
              "eipc_ccd_max_step", "eipc_barrier_hvp"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2409_16385_amd import binding
    lib = C.CDLL(binding.lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_argument_errors_without_gpu():
    from paper_2409_16385_amd import binding as B
    L = B._load()
    assert L.eipc_status_string(0) == b"ok"
    assert L.eipc_status_string(-3).startswith(b"intersecting")
    assert L.eipc_create(None, 0, 0) == B.ERR_ARG
    h = C.c_void_p()
    assert L.eipc_create(C.byref(h), -1, 0) == B.ERR_ARG
    r, hw = C.c_size_t(), C.c_size_t()
    assert L.eipc_scratch_bytes(None, C.byref(r), C.byref(hw)) == B.ERR_ARG
    # NULL context is rejected before any device work
    assert L.eipc_build_candidates(None, None, None, 1e-3, None, 0, None, 0, None, None, None) == B.ERR_ARG
    assert L.eipc_barrier_reduce(None, None, None, None, 0, None, 0, 1e-3, 1.0, 0, None, None, None, None,
                                 None, None) == B.ERR_ARG


def test_product_path_fails_loudly_without_gpu():
    import torch
    import paper_2409_16385_amd as E
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        E.Context(0)
