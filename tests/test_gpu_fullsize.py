"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (device-resident records, default tuning, graph-replayed rebuilds).

Mid trace (1.25e7 records): every output against the oracle.
Large trace (1.25e8 records): sampled resources against the oracle's union
measure computed one resource at a time, and properties that hold at any size
(exact additivity of the 63 tiles over the whole span, the trees' product
identities, every time non-negative and summing to E).
Regions entered repeatedly on the large trace (16 regions, every resource 32
times each) and stream concurrency of 256 devices x 4 streams (2.56e7
records), both as bench.py times them: sampled resources against the oracle
run on those resources alone, and the same kind of properties.
"""
import numpy as np
import pytest

import bench
import oracle
import paper_2603_26576_amd as hp
import tracegen as tg
from engine_util import assert_same, gpu_available

pytestmark = pytest.mark.gpu

DEV_LEVELS = [(tg.DEV_KERNEL,), (tg.DEV_KERNEL, tg.DEV_MEMOP)]
HOST_LEVELS = [(tg.HOST_USEFUL,), (tg.HOST_USEFUL, tg.HOST_OFFLOAD), (tg.HOST_USEFUL, tg.HOST_OFFLOAD, tg.HOST_MPI)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")
    hp.lib()


def device_session(trace):
    import torch
    s = hp.hpop_session_create(trace.n_hosts, trace.n_devices)
    dev = [(c.resource, c.kind, torch.from_numpy(c.start).cuda(), torch.from_numpy(c.end).cuda())
           for c in trace.chunks]
    torch.cuda.synchronize()
    hp.hpop_add_events_multi(s, dev, hp.HPOP_MEM_DEVICE)
    hp.hpop_session_synchronize(s)
    del dev
    for a, b in trace.regions:
        hp.hpop_region_define(s, a, b)
    return s


def all_times(s, trace):
    R = trace.n_hosts + trace.n_devices
    out = np.zeros((len(trace.regions), R, 4), np.int64)
    for g in range(len(trace.regions)):
        for r in range(R):
            out[g, r] = hp.hpop_resource_times(s, g, r)
    return out


def test_mid_full_size_every_output():
    tr = tg.mid()
    print("mid: %d records" % tr.n_events, flush=True)
    want = oracle.compute(tr, threads=16)
    s = device_session(tr)
    try:
        for _ in range(3):  # first build, then graph replays
            trees = hp.hpop_metrics_compute_all(s, hp.HPOP_FORCE_REBUILD)
        got = {"times": all_times(s, tr),
               "sums": np.array([hp.tree_sums(t) for t in trees]),
               "ratios": np.array([hp.tree_ratios(t) for t in trees]),
               "mask": np.array([t.undefined_mask for t in trees], np.uint32)}
    finally:
        hp.hpop_session_destroy(s)
    assert_same(got, want, "mid full size")


@pytest.fixture(scope="module")
def large_trace():
    tr = tg.large()
    print("large: %d records" % tr.n_events, flush=True)
    return tr


def sub_trace(tr, keep, regions=()):
    """The records of the resources in keep (sorted, hosts first), renumbered."""
    idx = {r: j for j, r in enumerate(keep)}
    chunks = [tg.Chunk(idx[c.resource], c.kind, c.start, c.end) for c in tr.chunks if c.resource in idx]
    return tg.Trace(sum(r < tr.n_hosts for r in keep), sum(r >= tr.n_hosts for r in keep), chunks, list(regions))


def test_large_full_size_sampled_and_properties(large_trace):
    tr = large_trace
    s = device_session(tr)
    try:
        for _ in range(2):
            trees = hp.hpop_metrics_compute_all(s, hp.HPOP_FORCE_REBUILD)
        times = all_times(s, tr)
    finally:
        hp.hpop_session_destroy(s)
    n, m = tr.n_hosts, tr.n_devices
    E = np.array([b - a for a, b in tr.regions], np.int64)
    # sampled resources, one at a time, through the oracle's union measure
    for r in (0, 101, n - 1, n, n + 77, n + m - 1):
        host = r < n
        levels = HOST_LEVELS if host else DEV_LEVELS
        D = []
        for kinds in levels:
            sel = [c for c in tr.chunks if c.resource == r and c.kind in kinds]
            st = np.concatenate([c.start for c in sel])
            en = np.concatenate([c.end for c in sel])
            D.append(oracle.union_measure(st, en, tr.regions))
        if host:
            want = np.stack([D[0], D[1] - D[0], D[2] - D[1], E - D[2]], 1)
        else:
            want = np.stack([D[0], D[1] - D[0], E - D[1], np.zeros_like(E)], 1)
        np.testing.assert_array_equal(times[:, r, :], want, err_msg="resource %d" % r)
    # the 63 tiles add up exactly to the whole span, for every resource
    np.testing.assert_array_equal(times[1:].sum(0), times[0])
    assert (times >= 0).all()
    np.testing.assert_array_equal(times[:, :n, :].sum(2), np.broadcast_to(E[:, None], (len(E), n)))
    np.testing.assert_array_equal(times[:, n:, :3].sum(2), np.broadcast_to(E[:, None], (len(E), m)))
    # trees from the per-resource times (exact integers) and their identities
    for g, t in enumerate(trees):
        h, d = times[g, :n], times[g, n:]
        assert t.sumU == h[:, 0].sum() and t.sumW == h[:, 1].sum() and t.sumMPI == h[:, 2].sum()
        assert t.maxUW == (h[:, 0] + h[:, 1]).max() and t.sumK == d[:, 0].sum() and t.maxKM == (d[:, 0] + d[:, 1]).max()
        assert t.host_pe == t.sumU / (n * t.E) and t.dev_oe == t.maxKM / t.E
        assert abs(t.host_pe - t.host_mpi_pe * t.host_oe) <= 4e-15 * t.host_pe
        assert abs(t.host_mpi_pe - t.host_mpi_lb * t.host_mpi_ce) <= 4e-15 * t.host_mpi_pe
        assert abs(t.dev_pe - t.dev_lb * t.dev_ce * t.dev_oe) <= 6e-15 * t.dev_pe


def test_entered_regions_full_size_sampled_and_properties(large_trace):
    tr = large_trace
    regions = bench.entered_regions(tr)
    n, m = tr.n_hosts, tr.n_devices
    R = n + m
    print("entered: %d regions, %d intervals" % (len(regions), sum(len(q) for q in regions)), flush=True)
    import torch
    s = hp.hpop_session_create(n, m)
    try:
        dev = [(c.resource, c.kind, torch.from_numpy(c.start).cuda(), torch.from_numpy(c.end).cuda())
               for c in tr.chunks]
        torch.cuda.synchronize()
        hp.hpop_add_events_multi(s, dev, hp.HPOP_MEM_DEVICE)
        hp.hpop_session_synchronize(s)
        del dev
        for ivls in regions:
            hp.hpop_region_define_multi(s, ivls)
        hp.hpop_session_set_tuning(s, 256, 2048, 2048)
        hp.hpop_metrics_compute_all(s)
        trees = hp.hpop_metrics_compute_all(s)  # the pass bench.py times: region kernels only
        times = np.zeros((len(regions), R, 4), np.int64)
        for g in range(len(regions)):
            for r in range(R):
                times[g, r] = hp.hpop_resource_times(s, g, r)
    finally:
        hp.hpop_session_destroy(s)
    Er = np.zeros((len(regions), R), np.int64)
    for g, ivls in enumerate(regions):
        for r, a, b in ivls:
            Er[g, r] += b - a
    # sampled resources through the oracle's definition, on their records alone
    keep = [0, 101, n - 1, n, n + 77, n + m - 1]
    sub = sub_trace(tr, keep)
    idx = {r: j for j, r in enumerate(keep)}
    sub_regions = [[(idx[r], a, b) for r, a, b in ivls if r in idx] for ivls in regions]
    want = oracle.compute_multi(sub, sub_regions)["times"]
    for j, r in enumerate(keep):
        np.testing.assert_array_equal(times[:, r, :], want[:, j, :], err_msg="resource %d" % r)
    # at any size: states add up to each resource's own time, trees from the times
    assert (times >= 0).all()
    np.testing.assert_array_equal(times[:, :n, :].sum(2), Er[:, :n])
    np.testing.assert_array_equal(times[:, n:, :3].sum(2), Er[:, n:])
    assert (times[:, n:, 3] == 0).all()
    for g, t in enumerate(trees):
        h, d = times[g, :n], times[g, n:]
        assert t.E == Er[g, :n].max()
        assert t.sumU == h[:, 0].sum() and t.sumW == h[:, 1].sum() and t.sumMPI == h[:, 2].sum()
        assert t.maxUW == (h[:, 0] + h[:, 1]).max() and t.sumK == d[:, 0].sum() and t.maxKM == (d[:, 0] + d[:, 1]).max()
        assert t.host_pe == t.sumU / (n * t.E) and t.dev_oe == t.maxKM / t.E


def test_streams_full_size_sampled_and_properties():
    n_streams, chunks, regions = bench.streams_workload()
    m = len(n_streams)
    print("streams: %d devices, %d records" % (m, sum(c[2].size for c in chunks)), flush=True)
    import torch
    s = hp.hpop_session_create(0, m)
    try:
        hp.hpop_session_set_tuning(s, 256, 2048, 2048)
        hp.hpop_session_set_streams(s, n_streams)
        dev = [(g, k, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for g, k, a, b in chunks]
        torch.cuda.synchronize()
        for g, k, a, b in dev:
            hp.hpop_add_stream_events(s, g, k, a, b)
        hp.hpop_session_synchronize(s)
        del dev
        for t0, t1 in regions:
            hp.hpop_region_define(s, t0, t1)
        for _ in range(2):  # rebuilds, as bench.py times them
            trees, per = hp.hpop_stream_metrics(s, hp.HPOP_FORCE_REBUILD, n_devices=m)
    finally:
        hp.hpop_session_destroy(s)
    # sampled devices through the oracle's definition, on their records alone
    keep = [0, 77, 200, m - 1]
    sub = [(keep.index(g), k, a, b) for g, k, a, b in chunks if g in keep]
    want = oracle.compute_streams([n_streams[g] for g in keep], sub, regions)["per_device"]
    np.testing.assert_array_equal(per[:, keep, :], want)
    # at any size: tiles add up to the whole span, the bounds of the stream count,
    # the trees' sums from the per-device values, each ratio one division
    np.testing.assert_array_equal(per[1:, :, :2].sum(0), per[0, :, :2])
    S = np.array(n_streams, np.int64)
    assert (per[:, :, 2] == S).all()
    B, ST = per[:, :, 0], per[:, :, 1]
    assert (B >= 0).all() and (B <= ST).all() and (ST <= S * B).all()
    for r, t in enumerate(trees):
        assert t.busy == B[r].sum() and t.stream_time == ST[r].sum() and t.capacity == (S * B[r]).sum()
        assert t.m == m and t.n_streams == S.sum() and t.undefined_mask == 0
        assert t.stream_eff == t.stream_time / t.capacity and t.mean_active == t.stream_time / t.busy
