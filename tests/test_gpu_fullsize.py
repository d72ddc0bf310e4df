"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (device-resident records, graph-replayed rebuilds), against the oracle
on the whole input:

* mid trace (1.25e7 records) and large trace (1.25e8 records, 512 resources,
  64 regions): every state time of every resource and every tree;
* stream concurrency of 256 devices x 4 streams (2.56e7 records): every
  device's values and every tree;
* the 1000-trace batch (1.38e8 records) at the tuning hpop_autotune picks,
  with its cache file written, read back and planted: every tree;
* the serving workload (32 sessions, 1e6 warm records each, 96 Poisson
  queries of 10^4-10^6 records, device and host payloads): every answer.

Regions entered repeatedly on the large trace (16 regions, every resource 32
times each) are checked on sampled resources (the oracle for them runs one
resource at a time in Python) plus properties that hold at any size.
"""
import json
import os

import numpy as np
import pytest

import bench
import oracle
import paper_2603_26576_amd as hp
import tracegen as tg
from engine_util import assert_same, gpu_available

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))  # the oracle's threads (the GPU host's share)

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


def test_large_full_size_every_output(large_trace):
    """Every state time of all 512 resources in all 64 regions, every tree,
    against the oracle on the whole trace."""
    tr = large_trace
    want = oracle.compute(tr, threads=THREADS)
    s = device_session(tr)
    try:
        for _ in range(3):  # first build, then graph replays, as bench.py times them
            trees = hp.hpop_metrics_compute_all(s, hp.HPOP_FORCE_REBUILD)
        got = {"times": all_times(s, tr),
               "sums": np.array([hp.tree_sums(t) for t in trees]),
               "ratios": np.array([hp.tree_ratios(t) for t in trees]),
               "mask": np.array([t.undefined_mask for t in trees], np.uint32)}
    finally:
        hp.hpop_session_destroy(s)
    assert_same(got, want, "large full size")
    # and what holds at any size: the 63 tiles add up exactly to the whole span
    np.testing.assert_array_equal(got["times"][1:].sum(0), got["times"][0])


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


def test_streams_full_size_every_device():
    """All 256 devices x 4 streams (2.56e7 records) as bench.py times them:
    every device's busy time, stream time and stream count in every region,
    and every tree, against the oracle."""
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
    want = oracle.compute_streams(n_streams, chunks, regions)
    np.testing.assert_array_equal(per, want["per_device"])
    for r, t in enumerate(trees):
        assert [t.busy, t.stream_time, t.capacity] == list(want["sums"][r]), r
        assert t.m == m and t.n_streams == sum(n_streams)
        np.testing.assert_array_equal(np.array([t.stream_eff, t.mean_active]).view(np.int64),
                                      want["ratios"][r].view(np.int64))
        assert t.undefined_mask == want["mask"][r]
    # at any size: tiles add up to the whole span
    np.testing.assert_array_equal(per[1:, :, :2].sum(0), per[0, :, :2])


def size_class_key(traces):
    """The autotuner's cache key of a batch (log2 of records, resources and traces, rounded)."""
    ev = sum(t.n_events for t in traces)
    res = sum(t.n_hosts + t.n_devices for t in traces)
    r = lambda x: int(np.floor(np.log2(max(1, x)) + 0.5))
    return "ev2^%d_res2^%d_k2^%d" % (r(ev), r(res), r(len(traces)))


def check_batch(trees, traces, wants, what):
    i = 0
    for j, (tr, want) in enumerate(zip(traces, wants)):
        for g in range(len(tr.regions)):
            t = trees[i]
            i += 1
            np.testing.assert_array_equal(hp.tree_sums(t), want["sums"][g], err_msg="%s trace %d region %d" % (what, j, g))
            np.testing.assert_array_equal(hp.tree_ratios(t).view(np.int64), want["ratios"][g].view(np.int64),
                                          err_msg="%s trace %d region %d" % (what, j, g))
            assert t.undefined_mask == want["mask"][g], (what, j, g)
    assert i == len(trees)


def test_batched_1000_traces_autotuned_and_cached(tmp_path):
    """The 1000-trace batch bench.py times (1.38e8 records): tuned by
    hpop_autotune with a cache file, every tree of every trace against the
    oracle; a second hpop_autotune reads its choice back from the cache
    (file untouched, same tuning, same trees); a tuning planted in the cache
    for this size class is the one applied, with the same trees again."""
    traces = tg.batched(n_traces=1000)
    print("batched: %d traces, %d records" % (len(traces), sum(t.n_events for t in traces)), flush=True)
    wants = [oracle.compute(tr, threads=THREADS) for tr in traces]
    cache = str(tmp_path / "tune.json")
    sessions = [device_session(tr) for tr in traces]
    try:
        tun = hp.hpop_autotune(sessions, cache)
        print("autotuned: target %d cap %d tile %d" % (tun.bucket_target, tun.bucket_cap, tun.tile_elems), flush=True)
        body = open(cache).read()
        key = size_class_key(traces)
        assert json.loads(body) == {key: [tun.bucket_target, tun.bucket_cap, tun.tile_elems]}
        for _ in range(2):  # first build at the chosen tuning, then a graph replay
            first = hp.hpop_batch_compute(sessions, hp.HPOP_FORCE_REBUILD)
        check_batch(first, traces, wants, "autotuned")
        # second call: served from the cache
        for s in sessions:
            hp.hpop_session_set_tuning(s, 128, 2048, 8192)
        again = hp.hpop_autotune(sessions, cache)
        assert (again.bucket_target, again.bucket_cap, again.tile_elems) == (tun.bucket_target, tun.bucket_cap,
                                                                             tun.tile_elems)
        assert open(cache).read() == body
        for s in (sessions[0], sessions[-1]):
            t = hp.hpop_session_get_tuning(s)
            assert (t.bucket_target, t.bucket_cap, t.tile_elems) == (tun.bucket_target, tun.bucket_cap, tun.tile_elems)
        second = hp.hpop_batch_compute(sessions, hp.HPOP_FORCE_REBUILD)
        for a, b in zip(first, second):
            assert bytes(a) == bytes(b)
        # a different choice planted for this size class is read and applied
        planted = [1024, 4096, 4096] if tun.bucket_target != 1024 else [128, 2048, 2048]
        with open(cache, "w") as f:
            json.dump({"ev2^1_res2^1_k2^0": [256, 2048, 512], key: planted}, f)
        got = hp.hpop_autotune(sessions, cache)
        assert [got.bucket_target, got.bucket_cap, got.tile_elems] == planted
        third = hp.hpop_batch_compute(sessions, hp.HPOP_FORCE_REBUILD)
        check_batch(third, traces, wants, "planted tuning %s" % planted)
    finally:
        for s in sessions:
            hp.hpop_session_destroy(s)


def test_serving_full_shape_against_oracle():
    """The serving workload bench.py times: 32 sessions x (16 hosts + 16
    devices x 4 streams), each warmed with 1e6 records, then 96 Poisson
    queries of 10^4-10^6 records, replayed natively with device-resident
    payloads at 20000 queries/s and with host payloads at 5000 queries/s.
    Every warm-up and query answer (its region and its session's global
    region) against the oracle over the records its session had received up
    to and including it."""
    W = bench.serving_workload(96)
    wants = {}
    for lam, host in ((20000, False), (5000, True)):
        res, kept = bench.serving_run(hp, W, lam, host, keep=True)
        print("serving %s: %s" % ("host" if host else "device", res), flush=True)
        entries = [("warm", e, t) for e, t in zip(kept["warm"], kept["warm_trees"])] + \
                  [("query", e, t) for e, t in zip(kept["queries"], kept["query_trees"])]
        for q, (what, entry, (reg, glob)) in enumerate(entries):
            k = (what, entry[0], entry[1], entry[2], tuple(entry[3]))
            if k not in wants:
                wants[k] = oracle.compute(bench.serving_expected_trace(W, entry), threads=THREADS)
            want = wants[k]
            for g, t in ((0, reg), (1, glob)):
                msg = "%s payload, %s %d of session %d, %s" % ("host" if host else "device", what, q, entry[0],
                                                               "region" if g == 0 else "global")
                np.testing.assert_array_equal(hp.tree_sums(t), want["sums"][g], err_msg=msg)
                np.testing.assert_array_equal(hp.tree_ratios(t).view(np.int64), want["ratios"][g].view(np.int64),
                                              err_msg=msg)
                assert t.undefined_mask == want["mask"][g], msg
    assert len(wants) == 32 + 96  # both runs served the same queries
