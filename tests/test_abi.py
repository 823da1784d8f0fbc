"""The C-ABI library loads and exports every symbol include/tcrnet.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os

import pytest

import paper_2112_06613_amd as tn


def test_library_present():
    assert os.path.exists(tn.LIB_PATH), "libtcrnet.so not built"


def test_exports_every_declared_symbol():
    names = tn.declared_symbols()
    assert len(names) >= 14
    lib = ctypes.CDLL(tn.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_flag_constants_match_header():
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "include", "tcrnet.h")) as f:
        hdr = f.read()
    flags = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define (TCRNET_F_\w+) (\d+)u", hdr)}
    assert set(flags) >= {"TCRNET_F_NO_AUTOTUNE", "TCRNET_F_PEQ_LDS", "TCRNET_F_NO_PACK", "TCRNET_F_PEQ_VGPR"}
    for name, value in flags.items():
        assert getattr(tn, name) == value, name


def test_host_only_calls():
    lib = tn.load_library()
    assert lib.tcrnet_version().decode().startswith("tcrnet")
    assert lib.tcrnet_status_string(tn.TCRNET_EINVAL) == b"TCRNET_EINVAL"
    assert lib.tcrnet_status_string(99) == b"TCRNET_UNKNOWN"
    # NULL arguments are rejected before any device call
    assert lib.tcrnet_ctx_create(0, None, None) == tn.TCRNET_EINVAL
    assert b"NULL" in lib.tcrnet_last_error()
    assert lib.tcrnet_build(None, None, 1, None) == tn.TCRNET_EINVAL
    # bulk graph views: nothing to describe is fine, missing arrays or graphs are not
    assert lib.tcrnet_graphs_views(None, 0, None, None, None, None, None) == tn.TCRNET_OK
    assert lib.tcrnet_graphs_views(None, 1, None, None, None, None, None) == tn.TCRNET_EINVAL
    slots = [ctypes.create_string_buffer(16) for _ in range(5)]
    nulls = (ctypes.c_void_p * 1)()
    assert lib.tcrnet_graphs_views(nulls, 1, *slots) == tn.TCRNET_EINVAL
    assert b"graph 0 is NULL" in lib.tcrnet_last_error()


def test_no_device_reports_edevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = tn.load_library().tcrnet_ctx_create(0, None, ctypes.byref(h))
    assert rc == tn.TCRNET_EDEVICE and not h.value
