"""The C-ABI library loads and exports every function include/hpop.h declares (CPU only)."""
import ctypes
import os
import re

import paper_2603_26576_amd as hp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(hpop_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


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
