"""Error behaviour of the C ABI (needs the HIP runtime and a GPU)."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2603_26576_amd as hp
import tracegen as tg
from engine_util import assert_same, engine_results, gpu_available, new_session

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")
    hp.lib()


def status_of(fn, *a):
    with pytest.raises(hp.HpopError) as ei:
        fn(*a)
    return ei.value.status, ei.value.message


def test_null_and_bad_arguments():
    L = hp.lib()
    assert L.hpop_session_create(None, None) == hp.HPOP_E_ARG
    assert L.hpop_session_destroy(None) == hp.HPOP_E_ARG
    assert L.hpop_metrics_compute_all(None, 0, None) == hp.HPOP_E_ARG
    assert L.hpop_batch_compute(None, 0, 0, None) == hp.HPOP_E_ARG
    assert L.hpop_server_create(None, None) == hp.HPOP_E_ARG
    assert status_of(hp.hpop_session_create, -1, 2)[0] == hp.HPOP_E_ARG


def test_add_events_errors_leave_session_unchanged():
    tr = tg.make_trace(3, 2, 2, 2, 300, 100, regions="tiles", n_regions=3)
    s, keep = new_session(tr)
    try:
        a = np.array([1, 2, 3], np.int64)
        b = np.array([2, 3, 4], np.int64)
        assert status_of(hp.hpop_add_events, s, 9, hp.HPOP_DEV_KERNEL, a, b)[0] == hp.HPOP_E_RESOURCE
        assert status_of(hp.hpop_add_events, s, 0, hp.HPOP_DEV_KERNEL, a, b)[0] == hp.HPOP_E_KIND
        assert status_of(hp.hpop_add_events, s, 3, hp.HPOP_HOST_MPI, a, b)[0] == hp.HPOP_E_KIND
        assert status_of(hp.hpop_add_events, s, 3, 7, a, b)[0] == hp.HPOP_E_KIND
        st, msg = status_of(hp.hpop_add_events, s, 3, hp.HPOP_DEV_KERNEL, a, np.array([2, 1, 4], np.int64))
        assert st == hp.HPOP_E_BAD_INTERVAL and "record 1" in msg
        st, _ = status_of(hp.hpop_add_events, s, 0, hp.HPOP_HOST_USEFUL, np.array([-5], np.int64),
                          np.array([3], np.int64))
        assert st == hp.HPOP_E_BAD_INTERVAL
        st, _ = status_of(hp.hpop_add_events, s, 0, hp.HPOP_HOST_USEFUL, np.array([0], np.int64),
                          np.array([1 << 62], np.int64))
        assert st == hp.HPOP_E_BAD_INTERVAL
        # a multi-add with one bad chunk adds nothing
        bad = [(0, hp.HPOP_HOST_USEFUL, a, b), (2, hp.HPOP_HOST_USEFUL, a, b)]
        assert status_of(hp.hpop_add_events_multi, s, bad, hp.HPOP_MEM_HOST)[0] == hp.HPOP_E_KIND
        assert_same(engine_results(s, tr), oracle.compute(tr), "after rejected calls")
    finally:
        hp.hpop_session_destroy(s)


def test_region_errors():
    s = hp.hpop_session_create(4, 4)
    try:
        assert status_of(hp.hpop_region_define, s, 10, 10)[0] == hp.HPOP_E_REGION
        assert status_of(hp.hpop_region_define, s, 10, 5)[0] == hp.HPOP_E_REGION
        assert status_of(hp.hpop_region_define, s, 0, 1 << 51)[0] == hp.HPOP_E_OVERFLOW
        assert hp.hpop_region_define(s, 0, 1 << 50) == 0
        assert status_of(hp.hpop_metrics_compute, s, 5)[0] == hp.HPOP_E_REGION
        assert status_of(hp.hpop_resource_times, s, 0, 0)[0] == hp.HPOP_E_STATE
        hp.hpop_metrics_compute_all(s)
        assert hp.hpop_resource_times(s, 0, 0) == [0, 0, 0, 1 << 50]
        assert status_of(hp.hpop_resource_times, s, 0, 8)[0] == hp.HPOP_E_RESOURCE
        t = hp.hpop_metrics_compute(s, 0)
        assert t.undefined_mask & (1 << 4) and t.host_oe == 1.0 and t.host_pe == 0.0
    finally:
        hp.hpop_session_destroy(s)


def test_flags_and_tuning_validation():
    s = hp.hpop_session_create(1, 1)
    try:
        L = hp.lib()
        out = (hp.hpop_metric_tree * 1)()
        assert L.hpop_metrics_compute_all(s, 0x80, out) == hp.HPOP_E_ARG
        t = hp.hpop_tuning(-1, 0, 0, 0)
        assert L.hpop_session_set_tuning(s, ctypes.byref(t)) == hp.HPOP_E_ARG
        hp.hpop_session_set_tuning(s, bucket_target=100, bucket_cap=4096, tile_elems=8192)
        got = hp.hpop_session_get_tuning(s)
        assert (got.bucket_target, got.bucket_cap, got.tile_elems) == (100, 4096, 8192)
    finally:
        hp.hpop_session_destroy(s)


def test_clear_events():
    tr = tg.make_trace(4, 2, 2, 2, 300, 100)
    s, keep = new_session(tr)
    try:
        engine_results(s, tr)
        hp.hpop_clear_events(s)
        empty = tg.Trace(2, 2, [], tr.regions)
        assert_same(engine_results(s, empty), oracle.compute(empty), "cleared")
    finally:
        hp.hpop_session_destroy(s)


def test_server_argument_errors():
    assert status_of(hp.hpop_server_create, 0, 1)[0] == hp.HPOP_E_ARG
    srv = hp.hpop_server_create(max_sessions=1)
    try:
        sid = hp.hpop_server_open_session(srv, 1, 1, 0)
        with pytest.raises(hp.HpopError) as ei:
            hp.hpop_server_open_session(srv, 1, 1, 0)
        assert ei.value.status == hp.HPOP_E_STATE
        a = np.array([1], np.int64)
        b = np.array([2], np.int64)
        with pytest.raises(hp.HpopError) as ei:
            hp.hpop_server_submit(srv, sid, [(0, hp.HPOP_DEV_KERNEL, a, b)], hp.HPOP_MEM_HOST, 0, 10)
        assert ei.value.status == hp.HPOP_E_KIND
        with pytest.raises(hp.HpopError) as ei:
            hp.hpop_server_submit(srv, sid, [(1, hp.HPOP_DEV_KERNEL, a, b)], hp.HPOP_MEM_HOST, 10, 10)
        assert ei.value.status == hp.HPOP_E_REGION
        with pytest.raises(hp.HpopError) as ei:
            hp.hpop_server_wait(srv, 12345)
        assert ei.value.status == hp.HPOP_E_ARG
        t = hp.hpop_server_submit(srv, sid, [(1, hp.HPOP_DEV_KERNEL, a, b)], hp.HPOP_MEM_HOST, 0, 10)
        reg, glob = hp.hpop_server_wait(srv, t, timeout_ns=10 ** 10)
        assert reg.sumK == 1 and reg.E == 10 and glob.E == 2
    finally:
        hp.hpop_server_destroy(srv)


def test_time_one_stage():
    """Timing every stage, then one named stage only (two events around its
    launches), then every stage again; the results never change."""
    tr = tg.make_trace(5, 2, 2, 2, 3000, 800, regions="tiles", n_regions=3)
    want = oracle.compute(tr)
    s, keep = new_session(tr)
    try:
        hp.hpop_session_enable_timing(s, True)
        assert_same(engine_results(s, tr, hp.HPOP_FORCE_REBUILD), want, "every stage timed")
        names_all = [n for n, _ in hp.hpop_session_stage_times(s)]
        assert names_all[:2] == ["reset", "stats"] and "merge_wave" in names_all and names_all[-1] == "region"
        hp.hpop_session_time_stage(s, "scatter")
        assert_same(engine_results(s, tr, hp.HPOP_FORCE_REBUILD), want, "scatter timed")
        st = hp.hpop_session_stage_times(s)
        assert [n for n, _ in st] == ["scatter"] and st[0][1] > 0
        hp.hpop_session_time_stage(s, "hist")  # the count pass: not run with fixed slots
        assert_same(engine_results(s, tr, hp.HPOP_FORCE_REBUILD), want, "hist timed")
        assert hp.hpop_session_stage_times(s) == []
        with pytest.raises(hp.HpopError) as ei:
            hp.hpop_session_time_stage(s, "no_such_stage")
        assert ei.value.status == hp.HPOP_E_ARG
        hp.hpop_session_time_stage(s, None)
        assert_same(engine_results(s, tr, hp.HPOP_FORCE_REBUILD), want, "every stage again")
        assert [n for n, _ in hp.hpop_session_stage_times(s)] == names_all
    finally:
        hp.hpop_session_destroy(s)
