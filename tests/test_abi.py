"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/tc.h, and the ctypes structures match the C layouts."""
import os
import re
import subprocess

import ctypes
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("tc_build_oriented", "tc_count_total", "tc_count_per_node", "tc_count_batch"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1406_5687_amd import tc

    lib = tc.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(tc.EXPORTED) == set(declared_functions())


def test_struct_layouts_match_header(tmp_path):
    from paper_1406_5687_amd import tc

    src = tmp_path / "sz.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "tc.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(tc_options),'
        ' sizeof(tc_graph_info_t), sizeof(tc_edges), offsetof(tc_options, hbm_budget_bytes),'
        ' offsetof(tc_options, min_chunk), offsetof(tc_options, lds_list_max), offsetof(tc_graph_info_t, device_bytes),'
        ' offsetof(tc_options, hash), offsetof(tc_graph_info_t, hash), offsetof(tc_options, bitmap_ratio),'
        ' offsetof(tc_graph_info_t, core_rows), offsetof(tc_graph_info_t, core_bytes)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [ctypes.sizeof(tc.Options), ctypes.sizeof(tc.GraphInfo), ctypes.sizeof(tc.Edges),
                    tc.Options.hbm_budget_bytes.offset, tc.Options.min_chunk.offset, tc.Options.lds_list_max.offset,
                    tc.GraphInfo.device_bytes.offset, tc.Options.hash.offset, tc.GraphInfo.hash.offset,
                    tc.Options.bitmap_ratio.offset, tc.GraphInfo.core_rows.offset, tc.GraphInfo.core_bytes.offset]


def test_status_strings_and_defaults():
    from paper_1406_5687_amd import tc

    lib = tc.load()
    assert lib.tc_status_str(0) == b"ok"
    assert lib.tc_status_str(2) == b"node id out of range"
    o = tc.Options()
    lib.tc_options_default(ctypes.byref(o))
    assert o.cost_fn == tc.COST_PRIOR and o.workers == 0 and o.hbm_budget_bytes == 0
    assert o.hash == tc.HASH_AUTO and o.bitmap_ratio == 0


def test_argument_errors_without_device():
    # NULL arguments are rejected before any device work.
    from paper_1406_5687_amd import tc

    lib = tc.load()
    h = ctypes.c_void_p(0)
    assert lib.tc_build_oriented(None, 1, None, ctypes.byref(h)) == tc.TC_ERR_INVALID_ARG
    assert lib.tc_count_total(None, None, None) == tc.TC_ERR_INVALID_ARG
    assert lib.tc_count_batch(None, 0, None, None, None) == tc.TC_ERR_INVALID_ARG
    lib.tc_graph_free(None)
    assert b"non-NULL" in lib.tc_last_error() or lib.tc_last_error()


def test_no_cpu_fallback_when_library_missing(tmp_path, monkeypatch):
    from paper_1406_5687_amd import tc

    monkeypatch.setattr(tc, "_lib", None)
    with pytest.raises(ImportError):
        tc.load(str(tmp_path / "missing.so"))
