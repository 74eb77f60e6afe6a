"""CPU checks of the C-ABI boundary: the library loads and exports every entry point mr.h declares,
and the Python structures match the header's layout."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mr.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:mr_status|const char\*)\s+(mr_\w+)\s*\(", txt, re.M)))


def _lib():
    from paper_1309_0215_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1309_0215_amd import build
        build.build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["mr_run", "mr_batch_run", "mr_job_create", "mr_job_destroy", "mr_status_str", "mr_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    from paper_1309_0215_amd import _lib as L
    names = _declared()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(L.EXPORTS) == names


def test_status_strings_without_a_gpu():
    lib = _lib()
    assert lib.mr_status_str(0) == b"MR_OK"
    assert lib.mr_status_str(-2) == b"MR_ERR_CAPACITY"
    assert lib.mr_status_str(12345) == b"MR_ERR_UNKNOWN"


def test_null_arguments_are_rejected_without_a_gpu():
    lib = _lib()
    from paper_1309_0215_amd import _lib as L
    assert lib.mr_job_create(None, None) == L.MR_ERR_INVALID_ARG
    assert lib.mr_run(None, 0, 0, None, 0, None, 0, 0, None) == L.MR_ERR_INVALID_ARG
    assert b"NULL" in lib.mr_last_error()
    assert lib.mr_job_destroy(None) == L.MR_OK
    assert lib.mr_workspace_bytes(None, 0, 0, 0, None) == L.MR_ERR_INVALID_ARG
    assert lib.mr_selector_load(None, None) == L.MR_ERR_INVALID_ARG


def test_struct_sizes_match_the_header():
    # sizes computed from the C declarations with the usual x86-64 alignment rules
    from paper_1309_0215_amd import _lib as L
    assert C.sizeof(L.JobConfig) == 4 + 4 + 8 + 4 * 5 + 4 + 8 + 4 + 4 + 4 + 4 + 8 + 4 + 4 + 4 + 4 + 8 + 8
    assert C.sizeof(L.Stats) == 4 + 4 + 8 + 8 + 4 + 4 + 4 + 4 + 4 + 4 + 8
    assert C.sizeof(L.Output) == 8 * 8 + 8 * 4 + 8 + C.sizeof(L.Stats) + 8 * 4
    assert C.sizeof(L.BatchItem) == 4 + 4 + 8 + 8 + 8 + 8 + 8
    assert C.sizeof(L.TuneEntry) == 4 + 4 + 8 + 8 + 4 * 4
    assert C.sizeof(L.TrainConfig) == 4 * 6 + 8


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1309_0215_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "oracle.cpp" not in txt and "liboracle" not in txt, f
