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
                     "wg_result_copy", "wg_result_free", "wg_status_string", "wg_last_error",
                     "wg_tc_batch", "wg_sg_batch", "wg_result_offsets", "wg_result_instances",
                     "wg_autotune", "wg_get_sort_config", "wg_set_sort_config", "wg_triangles",
                     "wg_sort_keys", "wg_merge_keys",
                     "wg_server_create", "wg_server_destroy", "wg_submit", "wg_poll", "wg_wait",
                     "wg_cancel", "wg_job_get_info", "wg_job_free", "wg_server_get_stats"]:
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


LAYOUT_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "wg.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
#define S(T) printf(#T " %zu\n", sizeof(T))
int main(void) {
  S(wg_options); F(wg_options, max_iterations); F(wg_options, radix_digit_bits);
  F(wg_options, tile_items);
  S(wg_stats); F(wg_stats, solve_ms); F(wg_stats, stage_bytes); F(wg_stats, delta_sizes);
  F(wg_stats, digit_bits); F(wg_stats, sort_passes);
  S(wg_sort_config); S(wg_tune_report); F(wg_tune_report, best); F(wg_tune_report, best_ms);
  F(wg_tune_report, tried); F(wg_tune_report, tried_ms);
  S(wg_server_config); F(wg_server_config, mem_budget_bytes);
  S(wg_server_stats); F(wg_server_stats, slots); F(wg_server_stats, budget_bytes);
  F(wg_server_stats, busy_ms);
  S(wg_job_info); F(wg_job_info, reservation_bytes); F(wg_job_info, submit_ms); F(wg_job_info, end_ms);
  return 0;
}
"""


def test_struct_layouts_match_the_header(tmp_path):
    """Sizes and offsets of every ABI struct, from gcc on the header, equal the binding's."""
    import shutil
    import subprocess

    from paper_2607_17571_amd import wg
    gcc = shutil.which("gcc") or shutil.which("cc")
    if gcc is None:
        pytest.skip("no C compiler")
    c = tmp_path / "probe.c"
    c.write_text(LAYOUT_PROBE)
    exe = tmp_path / "probe"
    subprocess.run([gcc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.splitlines())
    types = {"wg_options": wg.WgOptions, "wg_stats": wg.WgStats, "wg_sort_config": wg.WgSortConfig,
             "wg_tune_report": wg.WgTuneReport, "wg_server_config": wg.WgServerConfig,
             "wg_server_stats": wg.WgServerStats, "wg_job_info": wg.WgJobInfo}
    for key, val in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(types[t], f).offset == int(val), key
        else:
            assert ctypes.sizeof(types[key]) == int(val), key
