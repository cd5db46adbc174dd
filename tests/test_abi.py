"""The C-ABI library loads and exports every function include/topk.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "topk.h")
LIB = os.path.join(ROOT, "paper_1502_03942_amd", "libtopk.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(topk_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for want in ("topk_create", "topk_destroy", "topk_select_u32", "topk_select_f32",
                 "topk_workspace_bytes", "topk_set_param", "topk_strerror",
                 "topk_rows_fwd_f32", "topk_scatter_bwd_f32", "topk_select_batched_f32",
                 "topk_tune_batched_f32", "topk_save_tuning", "topk_load_tuning", "topk_tune_f32",
                 "topk_stream_read"):
        assert want in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libtopk.so not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_without_device():
    lib = ctypes.CDLL(LIB)
    lib.topk_strerror.restype = ctypes.c_char_p
    assert lib.topk_strerror(0) == b"ok"
    assert lib.topk_strerror(-2) == b"workspace too small"


def test_binding_flags_match_header():
    # every TOPK_* flag the binding passes has the value the header defines
    import paper_1502_03942_amd as tk
    text = open(HEADER).read()
    defines = {m.group(1): int(m.group(2)) for m in
               re.finditer(r"^#define\s+(TOPK_[A-Z_]+)\s+(\d+)u?\b", text, flags=re.M)}
    names = [n for n in dir(tk) if n.startswith("TOPK_") and isinstance(getattr(tk, n), int)]
    assert {"TOPK_LARGEST", "TOPK_SORTED", "TOPK_WRITE_KEYS", "TOPK_TRACE", "TOPK_GRAPH"} <= set(names)
    for n in names:
        assert n in defines and getattr(tk, n) == defines[n], n
