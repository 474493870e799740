"""Host-side checks of the C ABI that need no GPU: every declared symbol is
exported, the ctypes structures match the C layout, and argument validation
rejects bad calls before any device work."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1907_11803_amd import lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qwlsh.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qw_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(lib.LIB_PATH):
        from paper_1907_11803_amd import build
        build.build()
    return lib.load()


def test_every_declared_symbol_is_exported(so):
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(so, n), n
    assert set(names) == set(lib.SIGNATURES), "binding and header disagree"


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "qwlsh.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\","
        " sizeof(qw_opts), sizeof(qw_stats),"
        " sizeof(qw_index_info), offsetof(qw_stats, ms_stage), offsetof(qw_index_info, buckets),"
        " offsetof(qw_index_info, has_count_model), offsetof(qw_index_info, probing),"
        " sizeof(qw_tune_result), offsetof(qw_tune_result, ms_default),"
        " offsetof(qw_stats, ooc_index_files), offsetof(qw_stats, ooc_splits),"
        " offsetof(qw_index_info, host_bytes), sizeof(qw_ooc_opts), offsetof(qw_ooc_opts, keep),"
        " sizeof(qw_ooc_tune_result), offsetof(qw_ooc_tune_result, splits));"
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(lib.qw_opts), ctypes.sizeof(lib.qw_stats), ctypes.sizeof(lib.qw_index_info),
            lib.qw_stats.ms_stage.offset, lib.qw_index_info.buckets.offset,
            lib.qw_index_info.has_count_model.offset, lib.qw_index_info.probing.offset,
            ctypes.sizeof(lib.qw_tune_result), lib.qw_tune_result.ms_default.offset,
            lib.qw_stats.ooc_index_files.offset, lib.qw_stats.ooc_splits.offset,
            lib.qw_index_info.host_bytes.offset, ctypes.sizeof(lib.qw_ooc_opts),
            lib.qw_ooc_opts.keep.offset, ctypes.sizeof(lib.qw_ooc_tune_result),
            lib.qw_ooc_tune_result.splits.offset]
    assert got == want


def test_host_only_entry_points(so):
    assert so.qw_status_string(0) == b"ok"
    assert so.qw_status_string(1) == b"invalid argument"
    assert so.qw_mlp_param_count(16) == 64 * 16 + 2 * 64 + 1 == 1153
    o = lib.qw_opts()
    so.qw_default_opts(ctypes.byref(o))
    assert (o.form, o.sched, o.group, o.graph, o.timing) == (lib.QW_FORM_FAST, lib.QW_SCHED_LEARNED, -1, 1, 0)


def test_validation_rejects_before_device_work(so):
    out = ctypes.c_void_p()
    # null data / params
    assert so.qw_build_index(None, 10, 4, 0, None, None, 1.0, 1, 1, None, None, ctypes.byref(out)) == lib.QW_EINVAL
    # null index
    assert so.qw_query_workload(None, None, 0, 10, None, None, None, None, None) == lib.QW_EINVAL
    assert so.qw_hash(None, None, 0, 0, None, None, None) == lib.QW_EINVAL
    assert so.qw_autotune(None, None, 1, 1, None, b"/nonexistent/t.json", None, None) == lib.QW_EINVAL
    assert so.qw_get_index_info(None, None) == lib.QW_EINVAL
    assert so.qw_set_count_model(None, None, 0) == lib.QW_EINVAL
    assert so.qw_set_count_margin(None, 0.5) == lib.QW_EINVAL
    assert so.qw_set_probing(None, 1, 0) == lib.QW_EINVAL
    assert so.qw_set_counting(None, 1, 0) == lib.QW_EINVAL
    assert so.qw_set_out_of_core(None, None, None) == lib.QW_EINVAL
    assert so.qw_autotune_ooc(None, None, 1, 1, None, None, None) == lib.QW_EINVAL
    assert so.qw_mlp_loss_grad(None, 4, None, None, 1, None, None, None) == lib.QW_EINVAL
    so.qw_free_index(None)  # no-op


def test_oracle_and_library_share_no_code():
    """The oracle directory and the library sources never include one another."""
    csrc = os.path.join(ROOT, "paper_1907_11803_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "oracle" not in text.lower(), f
    for f in ("qw_oracle.c", "__init__.py", "mlp.py", "collision.py"):
        text = open(os.path.join(ROOT, "oracle", f)).read()
        assert "paper_1907_11803_amd" not in text and "qwlsh" not in text, f
