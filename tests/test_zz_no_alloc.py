"""hpop_metrics_compute_static (the entry point that allocates nothing) against
the session path (hpop_session_create, hpop_add_events_multi on device
memory, hpop_region_define, hpop_metrics_compute_all, hpop_resource_times)
on the same device records: every tree bit for bit and every state time,
over calls in a row where a later call is smaller than the one before (the
shared scratch array keeps the earlier call's contents), and after calls
that failed.
"""
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


def device_chunks(trace):
    import torch
    out = [(c.resource, c.kind, torch.from_numpy(c.start).cuda(), torch.from_numpy(c.end).cuda())
           for c in trace.chunks]
    torch.cuda.synchronize()
    return out


def static_results(trace, chunks):
    trees, times = hp.hpop_metrics_compute_static(trace.n_hosts, trace.n_devices, chunks, trace.regions, times=True)
    n = len(trace.regions)
    return {"times": times,
            "sums": np.array([hp.tree_sums(trees[g]) for g in range(n)], np.int64).reshape(n, 10),
            "ratios": np.array([hp.tree_ratios(trees[g]) for g in range(n)], np.float64).reshape(n, 9),
            "mask": np.array([trees[g].undefined_mask for g in range(n)], np.uint32),
            "trees": trees}


def session_results(trace):
    s, keep = new_session(trace, device=True)
    try:
        return engine_results(s, trace)
    finally:
        hp.hpop_session_destroy(s)


def check_same_trees(got, want):
    for g in range(len(want["trees"])):
        a, b = got["trees"][g], want["trees"][g]
        assert (a.E, a.n, a.m) == (b.E, b.n, b.m)
        assert bytes(a) == bytes(b), g


def test_two_calls_in_a_row_second_smaller():
    big = tg.make_trace(31, 16, 16, 4, 40000, 10000, w_range=(0.5, 1.5), idle_range=(0.1, 0.4),
                        regions="tiles", n_regions=9)
    small = tg.make_trace(32, 3, 2, 2, 3000, 700, regions="tiles", n_regions=4)
    for trace in (big, small):
        got = static_results(trace, device_chunks(trace))
        want = session_results(trace)
        assert_same(got, want, "static vs session")
        check_same_trees(got, want)
        assert_same(got, oracle.compute(trace), "static vs oracle")


def test_after_failures_and_with_edge_cases():
    import torch
    trace = tg.make_trace(33, 4, 4, 2, 5000, 1200, regions="tiles", n_regions=5)
    chunks = device_chunks(trace)
    want = session_results(trace)
    # an invalid device record: reported with its chunk and index, no trees
    s0 = chunks[0][2].clone()
    e0 = chunks[0][3].clone()
    s0[7] = e0[7] + 1
    bad = [(chunks[0][0], chunks[0][1], s0, e0)] + chunks[1:]
    with pytest.raises(hp.HpopError) as ei:
        hp.hpop_metrics_compute_static(trace.n_hosts, trace.n_devices, bad, trace.regions)
    assert ei.value.status == hp.HPOP_E_BAD_INTERVAL and "chunk 0, index 7" in ei.value.message
    # more records than the scratch array can hold: refused before any work
    n = 1 << 23
    z = torch.zeros(n, dtype=torch.int64, device="cuda")
    with pytest.raises(hp.HpopError) as ei:
        hp.hpop_metrics_compute_static(1, 1, [(1, tg.DEV_KERNEL, z, z)], [(0, 10)])
    assert ei.value.status == hp.HPOP_E_ARG and "bytes of scratch" in ei.value.message
    # host memory is refused (records must be device memory)
    c = trace.chunks[0]
    with pytest.raises(hp.HpopError) as ei:
        hp.hpop_metrics_compute_static(trace.n_hosts, trace.n_devices, [(c.resource, c.kind, c.start, c.end)],
                                       trace.regions)
    assert ei.value.status == hp.HPOP_E_ARG
    # wrong kind for the resource, bad region
    with pytest.raises(hp.HpopError) as ei:
        hp.hpop_metrics_compute_static(trace.n_hosts, trace.n_devices, [(0, tg.DEV_KERNEL) + chunks[0][2:]],
                                       trace.regions)
    assert ei.value.status == hp.HPOP_E_KIND
    with pytest.raises(hp.HpopError) as ei:
        hp.hpop_metrics_compute_static(trace.n_hosts, trace.n_devices, chunks, [(5, 5)])
    assert ei.value.status == hp.HPOP_E_REGION
    # the same records after the failures: identical to the session path
    got = static_results(trace, chunks)
    assert_same(got, want, "after failures")
    check_same_trees(got, want)
    # no records at all: every resource idle, device ratios 0/0
    empty = tg.Trace(trace.n_hosts, trace.n_devices, [], list(trace.regions))
    assert_same(static_results(empty, []), oracle.compute(empty), "no records")
    # no regions: nothing to write, still OK
    out = hp.hpop_metrics_compute_static(trace.n_hosts, trace.n_devices, chunks, [])
    assert len(out) == 1


def test_crowded_bucket_takes_exact_offsets():
    # every kernel of one device starts within a few ns: one bucket outgrows
    # its fixed slots, so the call redoes the build with exact offsets
    rng = np.random.default_rng(5)
    s = np.sort(rng.integers(1_000_000, 1_000_008, 60000)).astype(np.int64)
    e = s + rng.integers(1, 5000, s.size)
    spread = np.arange(0, 60000 * 1000, 1000, dtype=np.int64) + 2_000_000
    trace = tg.Trace(1, 2, [tg.Chunk(1, tg.DEV_KERNEL, s, e),
                            tg.Chunk(2, tg.DEV_KERNEL, spread, spread + 700),
                            tg.Chunk(0, tg.HOST_USEFUL, np.array([0], np.int64), np.array([10**8], np.int64))],
                     [(0, 10**8), (1_000_000, 3_000_000)])
    got = static_results(trace, device_chunks(trace))
    want = session_results(trace)
    assert_same(got, want, "crowded")
    assert_same(got, oracle.compute(trace), "crowded vs oracle")
