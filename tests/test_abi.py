"""The C-ABI library loads and exports every entry point include/lsort.h
declares.  Host-only calls are exercised; nothing here launches a kernel."""
import ctypes
import os
import re

import pytest

import paper_2107_03290_amd as ls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsort.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_api():
    names = declared()
    for must in ("ls_sort_f64", "ls_sort_u64", "ls_sort_segments", "ls_create", "ls_destroy",
                 "ls_model_train", "ls_stage_hist", "ls_server_submit"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ls.lib()
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(ls.EXPORTS) == declared()


def test_status_strings_host_only():
    lib = ls.lib()
    for code, text in ls.STATUS.items():
        assert lib.ls_status_string(code).decode() == text
    assert lib.ls_status_string(99).decode() == "unknown status"


def test_default_params_host_only():
    p = ls.params()
    assert p.struct_size == ctypes.sizeof(ls.Params) == 48
    assert (p.fanout, p.leaves, p.tile, p.base_threshold) == (1024, 1024, 0, 4096)   # tile 0: automatic
    assert p.sample_rate == 0.01
    assert p.sample_cap == 1 << 18          # the 1% rate holds up to 26.2M keys


def test_null_arguments_rejected_before_any_launch():
    lib = ls.lib()
    assert lib.ls_sort_f64(None, None, 10, None, None) == 1
    assert lib.ls_sort_u64(None, None, 10, None, None) == 1
    assert lib.ls_create(None, 0) == 1
    assert lib.ls_server_create(None, 0, 1 << 30, 1, None) == 1
    assert lib.ls_last_error(None).decode() == "null context"


def test_built_for_gfx950():
    data = open(ls.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_profile_only_flag_encoding_host_only():
    # LS_FLAG_PROFILE_ONLY(k) of include/lsort.h: class k + 1 in bits 8..11
    assert [ls.FLAG_PROFILE_ONLY(k) for k in range(8)] == [(k + 1) << 8 for k in range(8)]
    assert ls.KERNEL_CLASSES.index("scatter") == 4
    hdr = open(os.path.join(os.path.dirname(ls.LIB_PATH), "..", "include", "lsort.h")).read()
    assert "#define LS_FLAG_PROFILE_ONLY(k) (((uint32_t)(k) + 1u) << 8)" in hdr
