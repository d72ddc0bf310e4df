"""The C-ABI libraries load and export every function their headers declare
(include/hpop.h: libhpop.so; include/hpop_collect.h: libhpop_collect.so), and
the Python bindings cover them (CPU only)."""
import ctypes
import os
import re

import paper_2603_26576_amd as hp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="hpop.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hpop_[a-z_0-9]+)\s*\(", src)))


def test_every_header_has_a_library():
    assert sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")) == \
        ["hpop.h", "hpop_collect.h"]


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("hpop_session_create", "hpop_add_events", "hpop_region_define", "hpop_metrics_compute",
                 "hpop_batch_compute", "hpop_server_submit", "hpop_autotune"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(hp.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    missing = [n for n in declared_functions() if not hasattr(hp, n) and n != "hpop_last_error"
               and n != "hpop_server_last_error"]
    assert not missing, missing


def test_status_strings_without_gpu():
    assert hp.hpop_status_string(0) == "ok"
    assert "interval" in hp.hpop_status_string(hp.HPOP_E_BAD_INTERVAL)
    assert hp.hpop_status_string(12345) == "unknown status"


def test_tree_layout_matches_header():
    assert ctypes.sizeof(hp.hpop_metric_tree) == 8 + 8 + 10 * 8 + 9 * 8 + 8


def test_collector_exports_every_declared_symbol():
    from paper_2603_26576_amd import collect
    names = declared_functions("hpop_collect.h")
    assert "hpop_collect_poll" in names and "hpop_collect_copy" in names
    lib = ctypes.CDLL(collect.COLLECT_LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert hasattr(lib, "rocprofiler_configure")
    missing = [n for n in names if not hasattr(collect, n)]
    assert not missing, missing
