"""The C-ABI library loads and exports every entry point include/smash.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smash.h")
LIB = os.path.join(ROOT, "paper_2105_14156_amd", "libsmash.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(smash_[a-z_0-9]+)\s*\(", text))
    return sorted(n for n in names if not n.endswith("_fn"))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libsmash.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_boundary():
    fns = declared_functions()
    for required in ("smash_spgemm_symbolic", "smash_spgemm_numeric", "smash_spgemm", "smash_create",
                     "smash_destroy", "smash_last_error", "smash_workspace_size", "smash_sync"):
        assert required in fns


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_kernel_table(lib):
    lib.smash_status_string.restype = ctypes.c_char_p
    assert lib.smash_status_string(0) == b"SMASH_OK"
    assert lib.smash_status_string(2) == b"SMASH_ERR_INVALID_CSR"
    assert lib.smash_status_string(99) == b"SMASH_ERR_UNKNOWN"
    assert lib.smash_kernel_count() > 5


def test_null_arguments_rejected(lib):
    # argument checks that return before any HIP call
    assert lib.smash_create(None, 0) == 1
    lib.smash_last_error.restype = ctypes.c_char_p
    assert lib.smash_last_error(None) == b"null context"
    assert lib.smash_spgemm_symbolic(None, None, None, None, None, None, 0, None) == 1
    assert lib.smash_workspace_size(None, 0, None, None, None, None) == 1
    assert lib.smash_sync(None, None) == 1


def test_binding_matches_header():
    from paper_2105_14156_amd import smash
    for n in declared_functions():
        assert hasattr(smash._lib, n)


def _struct_fields(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + ";", text).group(1)
    return [f for decl in body.split(";") if decl.strip()
            for f in re.sub(r"^\s*[a-z0-9_]+\s+", "", decl.strip()).replace(" ", "").split(",")]


def test_binding_layouts_match_header():
    """Field order of smash_stats and the option numbers in the binding
    follow the header (the binding mirrors them by hand)."""
    from paper_2105_14156_amd import smash
    assert [n for n, _ in smash.Stats._fields_] == _struct_fields("smash_stats")
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    opts = dict((k, int(v)) for k, v in re.findall(r"SMASH_OPT_([A-Z_]+)\s*=\s*(\d+)", text))
    for k, v in opts.items():
        if k != "COUNT":
            assert getattr(smash, "OPT_" + k) == v, k
    assert opts["COUNT"] == len(opts) - 1


def test_batch_config_layout_matches_header():
    from paper_2105_14156_amd import smash
    assert [n for n, _ in smash.BatchConfig._fields_] == _struct_fields("smash_batch_config")
