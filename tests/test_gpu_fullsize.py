"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (device-resident records, default tuning, graph-replayed rebuilds).

Mid trace (1.25e7 records): every output against the oracle.
Large trace (1.25e8 records): sampled resources against the oracle's union
measure computed one resource at a time, and properties that hold at any size
(exact additivity of the 63 tiles over the whole span, the trees' product
identities, every time non-negative and summing to E).
"""
import numpy as np
import pytest

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


def test_large_full_size_sampled_and_properties():
    tr = tg.large()
    print("large: %d records" % tr.n_events, flush=True)
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
