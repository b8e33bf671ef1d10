"""CPU checks of the C-ABI library: it loads and exports every entry point
that include/sccg.h declares.  No compute call is made (no GPU here)."""

import ctypes
import os
import re

import pytest

import paper_1208_0277_amd as sccg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sccg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sccg_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sccg.LIB_PATH):
        pytest.skip("device library not built")
    return sccg.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("sccg_create", "sccg_area_pairs", "sccg_jaccard_sets", "sccg_sync", "sccg_destroy"):
        assert need in names
    assert set(names) == set(sccg.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_null_context_is_an_argument_error(lib):
    assert lib.sccg_sync(None) == sccg.SCCG_E_ARG
    assert lib.sccg_destroy(None) == sccg.SCCG_E_ARG
    assert lib.sccg_area_pairs(None, None, None, 0, None, None, None, None, 0) == sccg.SCCG_E_ARG
    assert lib.sccg_jaccard_sets(None, 0, None, None, None, 0, None, None, None, None, None) == sccg.SCCG_E_ARG
    assert lib.sccg_create(None, 0, None, None) == sccg.SCCG_E_ARG
    assert lib.sccg_version().decode().startswith("sccg")


def test_params_struct_matches_header():
    text = open(os.path.join(ROOT, "include", "sccg.h")).read()
    body = re.search(r"typedef struct \{(.*?)\} sccg_params;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(?:u?int32_t)\s+([a-z_0-9]+)\s*;", body)
    assert fields == [f for f, _ in sccg.sccg_params._fields_]
    assert ctypes.sizeof(sccg.sccg_params) == 4 * len(fields)
