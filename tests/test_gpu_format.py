"""Reports rendered from the engine's own trees (hpop_region_format) against
the same renderings of the oracle's trees and state times.

* PILS use cases (Sec. 5.1 tables): the text report's tree part is byte for
  byte the rendering of the oracle's tree, and every ratio shows the printed
  two-decimal string exactly; every resource line holds the oracle's times.
* A generated trace with several regions: text and JSON reports of every
  region against the oracle, the JSON's doubles bit for bit.
"""
import json

import numpy as np
import pytest

import oracle
import paper_2603_26576_amd as hp
import pils
import tracegen as tg
from engine_util import gpu_available, new_session

pytestmark = pytest.mark.gpu

LABELS = ["Host Parallel Efficiency", "MPI Parallel Efficiency", "MPI Load Balance",
          "MPI Communication Efficiency", "Device Offload Efficiency", "Device Parallel Efficiency",
          "Load Balance", "Communication Efficiency", "Orchestration Efficiency"]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")
    hp.lib()


def oracle_tree(trace, want, g):
    t = hp.hpop_metric_tree()
    a, b = trace.regions[g]
    t.E, t.n, t.m = b - a, trace.n_hosts, trace.n_devices
    for f, v in zip(hp.SUM_FIELDS, want["sums"][g]):
        setattr(t, f, int(v))
    for f, v in zip(hp.RATIO_FIELDS, want["ratios"][g]):
        setattr(t, f, float(v))
    t.undefined_mask = int(want["mask"][g])
    return t


def expected_text(trace, want, g):
    """The oracle's tree rendered by hpop_tree_format, then one line per resource."""
    out = hp.hpop_tree_format(oracle_tree(trace, want, g), hp.HPOP_FORMAT_TEXT)
    out += "Resource times in the region (ns):\n"
    n = trace.n_hosts
    for r, x in enumerate(want["times"][g]):
        if r < n:
            out += "  host %d: useful %d, offload %d, MPI %d, other %d\n" % (r, x[0], x[1], x[2], x[3])
        else:
            out += "  device %d: kernels %d, memory operations %d, idle %d\n" % (r - n, x[0], x[1], x[2])
    return out


def check_json(report, trace, want, g):
    d = json.loads(report)
    a, b = trace.regions[g]
    assert (d["E"], d["n"], d["m"]) == (b - a, trace.n_hosts, trace.n_devices)
    host = [d["host"][k] for k in ("parallel_efficiency", "mpi_parallel_efficiency", "mpi_load_balance",
                                   "mpi_communication_efficiency", "device_offload_efficiency")]
    dev = [d["device"][k] for k in ("parallel_efficiency", "load_balance", "communication_efficiency",
                                    "orchestration_efficiency")]
    np.testing.assert_array_equal(np.array(host + dev, np.float64).view(np.int64), want["ratios"][g].view(np.int64))
    t = d["times"]
    got_sums = [t["useful"], t["offload"], t["mpi"], t["other"], t["useful_plus_offload"],
                t["max_useful_plus_offload"], t["kernel"], t["memory_operations"], t["max_kernel"],
                t["max_kernel_plus_memory"]]
    assert got_sums == [int(v) for v in want["sums"][g]]
    n = trace.n_hosts
    assert len(d["resources"]) == trace.n_hosts + trace.n_devices
    for r, (obj, x) in enumerate(zip(d["resources"], want["times"][g])):
        if r < n:
            assert obj == {"host": r, "useful": x[0], "offload": x[1], "mpi": x[2], "other": x[3]}
        else:
            assert obj == {"device": r - n, "kernel": x[0], "memory_operations": x[1], "idle": x[2]}


@pytest.mark.parametrize("case", pils.load(), ids=lambda c: c[0])
@pytest.mark.parametrize("device", [False, True])
def test_pils_reports_from_engine_trees(case, device):
    name, printed, t = case
    trace = pils.build_trace(t, kernel_streams=3)
    want = oracle.compute(trace)
    s, keep = new_session(trace, device=device)
    try:
        text = hp.hpop_region_format(s, 0, hp.HPOP_FORMAT_TEXT)
        js = hp.hpop_region_format(s, 0, hp.HPOP_FORMAT_JSON)
        engine_tree = hp.hpop_metrics_compute(s, 0)
    finally:
        hp.hpop_session_destroy(s)
    assert text == expected_text(trace, want, 0)
    assert text.startswith(hp.hpop_tree_format(engine_tree, hp.HPOP_FORMAT_TEXT))
    rows = [l for l in text.splitlines() if any(l.strip().startswith(x) for x in LABELS)]
    assert [r.split()[-1] for r in rows] == ["%.2f" % v for v in printed]
    check_json(js, trace, want, 0)


def test_generated_trace_every_region():
    trace = tg.make_trace(11, 6, 5, 3, 3000, 900, regions="tiles", n_regions=7)
    want = oracle.compute(trace)
    s, keep = new_session(trace, device=True)
    try:
        for g in range(len(trace.regions)):
            assert hp.hpop_region_format(s, g, hp.HPOP_FORMAT_TEXT) == expected_text(trace, want, g)
            check_json(hp.hpop_region_format(s, g, hp.HPOP_FORMAT_JSON), trace, want, g)
    finally:
        hp.hpop_session_destroy(s)


def test_region_format_errors_and_truncation():
    import ctypes
    trace = tg.make_trace(3, 2, 2, 2, 200, 60, regions="tiles", n_regions=2)
    s, keep = new_session(trace)
    try:
        L = hp.lib()
        assert L.hpop_region_format(s, 5, 0, None, 0, None) == hp.HPOP_E_REGION
        assert L.hpop_region_format(s, 0, 9, None, 0, None) == hp.HPOP_E_ARG
        assert L.hpop_region_format(s, 0, 0, None, 4, None) == hp.HPOP_E_ARG
        assert L.hpop_region_format(None, 0, 0, None, 0, None) == hp.HPOP_E_ARG
        need = ctypes.c_int64()
        buf = ctypes.create_string_buffer(40)
        assert L.hpop_region_format(s, 1, 1, buf, 40, ctypes.byref(need)) == 0
        full = hp.hpop_region_format(s, 1, hp.HPOP_FORMAT_JSON)
        assert need.value == len(full) + 1 and buf.value.decode() == full[:39]
    finally:
        hp.hpop_session_destroy(s)
