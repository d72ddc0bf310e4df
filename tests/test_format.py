"""Text and JSON renderings of metric trees (host code; CPU only).

The trees come from the oracle on the PILS use cases (Sec. 5.1 tables): the
text rendering must show exactly the printed two-decimal strings in the
paper's tree order, and the JSON rendering must give back every ratio and integer exactly.
"""
import json

import numpy as np
import pytest

import oracle
import paper_2603_26576_amd as hp
import pils


def oracle_tree(trace, g=0):
    want = oracle.compute(trace)
    t = hp.hpop_metric_tree()
    a, b = trace.regions[g]
    t.E, t.n, t.m = b - a, trace.n_hosts, trace.n_devices
    for f, v in zip(hp.SUM_FIELDS, want["sums"][g]):
        setattr(t, f, int(v))
    for f, v in zip(hp.RATIO_FIELDS, want["ratios"][g]):
        setattr(t, f, float(v))
    t.undefined_mask = int(want["mask"][g])
    return t


@pytest.mark.parametrize("case", pils.load(), ids=lambda c: c[0])
def test_text_tree_shows_the_printed_values(case):
    name, printed, t = case
    tree = oracle_tree(pils.build_trace(t))
    lines = hp.hpop_tree_format(tree, hp.HPOP_FORMAT_TEXT).splitlines()
    labels = ["Host Parallel Efficiency", "MPI Parallel Efficiency", "MPI Load Balance",
              "MPI Communication Efficiency", "Device Offload Efficiency", "Device Parallel Efficiency",
              "Load Balance", "Communication Efficiency", "Orchestration Efficiency"]
    rows = [l for l in lines if any(l.strip().startswith(x) for x in labels)]
    assert [r.strip().rsplit(None, 1)[0].strip() for r in rows] == labels
    # indentation: children two spaces deeper than their parent
    assert [len(r) - len(r.lstrip()) for r in rows] == [0, 2, 4, 4, 2, 0, 2, 2, 2]
    # the fixtures reproduce the tables, so each rendered value is the printed string
    assert [r.split()[-1] for r in rows] == ["%.2f" % v for v in printed]


@pytest.mark.parametrize("case", pils.load()[:3], ids=lambda c: c[0])
def test_json_round_trips_exactly(case):
    name, printed, t = case
    tree = oracle_tree(pils.build_trace(t))
    d = json.loads(hp.hpop_tree_format(tree, hp.HPOP_FORMAT_JSON))
    assert (d["E"], d["n"], d["m"]) == (tree.E, tree.n, tree.m)
    host = [d["host"][k] for k in ("parallel_efficiency", "mpi_parallel_efficiency", "mpi_load_balance",
                                   "mpi_communication_efficiency", "device_offload_efficiency")]
    dev = [d["device"][k] for k in ("parallel_efficiency", "load_balance", "communication_efficiency",
                                    "orchestration_efficiency")]
    np.testing.assert_array_equal(np.array(host + dev).view(np.int64), hp.tree_ratios(tree).view(np.int64))
    assert d["times"]["useful"] == tree.sumU and d["times"]["max_kernel_plus_memory"] == tree.maxKM


def test_undefined_ratios_are_marked():
    t = hp.hpop_metric_tree()
    t.E, t.n, t.m = 100, 1, 1
    t.sumU, t.sumUW, t.maxUW = 100, 100, 100
    for f in hp.RATIO_FIELDS:
        setattr(t, f, 1.0)
    t.undefined_mask = (1 << 5) | (1 << 6) | (1 << 7)  # no device time at all
    text = hp.hpop_tree_format(t, hp.HPOP_FORMAT_TEXT)
    assert sum(l.endswith(" *") for l in text.splitlines()) == 3
    d = json.loads(hp.hpop_tree_format(t, hp.HPOP_FORMAT_JSON))
    assert d["undefined"] == ["device.parallel_efficiency", "device.load_balance", "device.communication_efficiency"]


def test_bad_arguments_and_truncation():
    t = hp.hpop_metric_tree()
    L = hp.lib()
    import ctypes
    assert L.hpop_tree_format(None, 0, None, 0, None) == hp.HPOP_E_ARG
    assert L.hpop_tree_format(ctypes.byref(t), 7, None, 0, None) == hp.HPOP_E_ARG
    assert L.hpop_tree_format(ctypes.byref(t), 0, None, 10, None) == hp.HPOP_E_ARG
    need = ctypes.c_int64()
    buf = ctypes.create_string_buffer(16)
    assert L.hpop_tree_format(ctypes.byref(t), 1, buf, 16, ctypes.byref(need)) == 0
    assert len(buf.value) == 15 and need.value > 16


def test_json_and_text_keep_long_values_whole():
    """Every integer at its widest (20 characters) and ratios with 17 significant
    digits: the JSON still parses and gives back every value exactly, and the
    text shows every integer in full."""
    t = hp.hpop_metric_tree()
    t.E, t.n, t.m = -(2 ** 63) + 1, 2 ** 31 - 1, -(2 ** 31)
    big = [-(2 ** 63) + 1 + i for i in range(10)]
    for f, v in zip(hp.SUM_FIELDS, big):
        setattr(t, f, v)
    vals = [1.2345678901234567e-300 * (i + 1) for i in range(9)]
    for f, v in zip(hp.RATIO_FIELDS, vals):
        setattr(t, f, v)
    t.undefined_mask = 0x1ff
    d = json.loads(hp.hpop_tree_format(t, hp.HPOP_FORMAT_JSON))
    assert (d["E"], d["n"], d["m"]) == (t.E, t.n, t.m)
    times = d["times"]
    assert [times[k] for k in ("useful", "offload", "mpi", "other", "useful_plus_offload", "max_useful_plus_offload",
                               "kernel", "memory_operations", "max_kernel", "max_kernel_plus_memory")] == big
    assert len(d["undefined"]) == 9
    text = hp.hpop_tree_format(t, hp.HPOP_FORMAT_TEXT)
    for v in big[:4] + big[6:8]:
        assert str(v) in text
