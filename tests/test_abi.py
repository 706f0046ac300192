"""The C-ABI library loads and exports every entry point declared in include/*.h.

No compute call is made here (no GPU needed).
"""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2607_17571_amd", "libwg.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"\b(wg_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ["wg_engine_create", "wg_engine_destroy", "wg_tc", "wg_sg", "wg_result_size",
                     "wg_result_copy", "wg_result_free", "wg_status_string", "wg_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail(f"library not built: {LIB}")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_covers_every_declared_symbol():
    from paper_2607_17571_amd import wg
    bound = {name for name, _, _ in wg.SIGNATURES}
    assert set(declared_functions()) <= bound
    for name in declared_functions():
        assert callable(getattr(wg, name)), name


def test_status_strings_without_gpu():
    from paper_2607_17571_amd import wg
    assert wg.wg_status_string(wg.WG_OK) == "ok"
    assert "invalid" in wg.wg_status_string(wg.WG_ERR_INVALID_ARG)


def test_options_struct_matches_header_layout():
    from paper_2607_17571_amd import wg
    assert ctypes.sizeof(wg.WgOptions) == 48
    assert wg.WgStats.delta_sizes.offset == 8 * 6 + 8 + 8 + 3 * 8 * wg.WG_NUM_STAGES
