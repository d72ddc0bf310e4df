"""Shared streaming tiles: record batches of fewer than half a tile of records
are packed several to a tile (at most 32 batches and one tile of records), and
the start-range, count and scatter passes find each record's batch, resource,
kind and bucket geometry per record.

Every case is compared with the oracle bit for bit (integers exactly, the FP64
ratios as bit patterns), and with the same records built at the default tuning
(4096-record tiles, which keep one batch per tile).
"""
import numpy as np
import pytest

import oracle
import paper_2603_26576_amd as hp
import tracegen as tg
from engine_util import assert_same, engine_results, gpu_available, new_session, run_engine

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")
    hp.lib()


def in_batches(trace, rng, max_batch, shuffle):
    """The trace's records cut into batches of 1..max_batch consecutive records
    of one resource and kind; with shuffle the batches arrive in random order."""
    out = []
    for c in trace.chunks:
        n, i = len(c.start), 0
        while i < n:
            k = int(rng.integers(1, max_batch + 1))
            out.append(tg.Chunk(c.resource, c.kind, c.start[i:i + k].copy(), c.end[i:i + k].copy()))
            i += k
    if shuffle:
        out = [out[j] for j in rng.permutation(len(out))]
    return tg.Trace(trace.n_hosts, trace.n_devices, out, list(trace.regions))


def check(trace, tuning):
    print("case: n=%d m=%d events=%d batches=%d %s" % (trace.n_hosts, trace.n_devices, trace.n_events,
                                                       len(trace.chunks), tuning), flush=True)
    want = oracle.compute(trace)
    got = run_engine(trace, tuning=tuning)
    assert_same(got, want, str(tuning))
    plain = run_engine(trace)
    for a, b in zip(got["trees"], plain["trees"]):
        assert bytes(a) == bytes(b)


TUNINGS = [
    {"bucket_target": 64, "tile_elems": 512},
    {"bucket_target": 256, "bucket_cap": 2048, "tile_elems": 2048},
    {"bucket_target": 64, "tile_elems": 512, "scatter_slots": -1},    # exact offsets: the count pass too
    {"bucket_target": 128, "tile_elems": 2048, "scatter_slots": -1},
]


@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: "-".join("%s%d" % (k[0], v) for k, v in t.items()))
@pytest.mark.parametrize("max_batch,shuffle", [(8, False), (8, True), (300, False), (300, True)])
def test_small_batches(tuning, max_batch, shuffle):
    rng = np.random.default_rng(1000 + max_batch + (7 if shuffle else 0))
    base = tg.make_trace(41, 4, 4, 4, 3000, 900, w_range=(0.5, 1.5), regions="nested", n_regions=5)
    check(in_batches(base, rng, max_batch, shuffle), tuning)


def test_batch_limit_per_tile():
    """Single-record batches: 32 of them fill a shared tile long before its
    records do."""
    rng = np.random.default_rng(5)
    base = tg.make_trace(42, 2, 3, 2, 700, 300, regions="tiles", n_regions=4)
    check(in_batches(base, rng, 1, True), {"bucket_target": 32, "tile_elems": 512})


def test_window_wider_than_the_tile():
    """Small batches of two resources with thousands of buckets of large
    resources between them in the bucket order: their shared tile spans more
    buckets than its LDS window and counts with global atomics instead."""
    rng = np.random.default_rng(6)
    chunks = []
    for dev in range(6):
        n = 200 if dev in (0, 5) else 20000
        s = np.sort(rng.integers(0, 1 << 28, size=n)).astype(np.int64)
        e = s + rng.integers(0, 50000, size=n)
        kind = rng.random(n) < 0.3
        for k, sel in ((tg.DEV_KERNEL, ~kind), (tg.DEV_MEMOP, kind)):
            if dev in (0, 5):
                idx = np.flatnonzero(sel)
                for a in range(0, idx.size, 37):
                    chunks.append(tg.Chunk(dev, k, s[idx[a:a + 37]], e[idx[a:a + 37]]))
            else:
                chunks.append(tg.Chunk(dev, k, s[sel], e[sel]))
    tr = tg.Trace(0, 6, chunks, [(0, 1 << 28), (1 << 26, 1 << 27), (12345, 1 << 29)])
    for tuning in ({"bucket_target": 16, "tile_elems": 512}, {"bucket_target": 16, "tile_elems": 512,
                                                             "scatter_slots": -1}):
        check(tr, tuning)


def test_both_record_forms_and_clamped_ends():
    """Small batches of a resource whose buckets are wider than 2^30 ns (the
    16 B record form), of one with far-ending records (8 B form, clamped
    ends), and of a host with long MPI states."""
    rng = np.random.default_rng(7)
    s = np.sort(rng.integers(0, 1 << 34, size=4000)).astype(np.int64)
    e = s + rng.integers(0, 2000, size=s.size)
    far = rng.random(s.size) < 0.01
    e[far] = s[far] + rng.integers(1 << 32, 1 << 35, size=int(far.sum()))
    s2 = np.sort(rng.integers(0, 1 << 45, size=600)).astype(np.int64)
    e2 = s2 + rng.integers(0, 1 << 40, size=s2.size)
    s3 = np.sort(rng.integers(0, 1 << 36, size=3000)).astype(np.int64)
    kinds = rng.integers(0, 3, size=s3.size)
    e3 = s3 + np.where(kinds == 2, rng.integers(1 << 31, 1 << 33, size=s3.size), rng.integers(0, 5000, size=s3.size))
    chunks = [tg.Chunk(1, tg.DEV_KERNEL, s, e), tg.Chunk(2, tg.DEV_KERNEL, s2, e2)]
    chunks += [tg.Chunk(0, kd, s3[kinds == kd], e3[kinds == kd]) for kd in (tg.HOST_USEFUL, tg.HOST_OFFLOAD, tg.HOST_MPI)]
    tr = in_batches(tg.Trace(1, 2, chunks, [(0, 1 << 46), (1 << 20, 1 << 33), (5 << 30, 7 << 30)]), rng, 90, True)
    for tuning in ({"bucket_target": 64, "tile_elems": 512}, {"bucket_target": 256, "tile_elems": 2048}):
        check(tr, tuning)


def test_invalid_record_in_a_shared_tile():
    import torch
    rng = np.random.default_rng(8)
    good = in_batches(tg.make_trace(43, 2, 2, 2, 500, 200), rng, 40, True)
    s, keep = new_session(good, tuning={"bucket_target": 64, "tile_elems": 512})
    try:
        bad_s = torch.tensor([10, 20, 30], dtype=torch.int64, device="cuda")
        bad_e = torch.tensor([11, 19, 31], dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        hp.hpop_add_events(s, 2, hp.HPOP_DEV_KERNEL, bad_s, bad_e)
        with pytest.raises(hp.HpopError) as ei:
            hp.hpop_metrics_compute_all(s)
        assert ei.value.status == hp.HPOP_E_BAD_INTERVAL
        assert "index 1" in ei.value.message
        assert_same(engine_results(s, good), oracle.compute(good), "after drop")
    finally:
        hp.hpop_session_destroy(s)


@pytest.mark.parametrize("tile", [512, 2048])
def test_batched_sessions_share_tiles(tile):
    """A batched build of many small traces: shared tiles hold batches of
    several sessions; a repeated build (graph replay) gives the same bytes."""
    rng = np.random.default_rng(9 + tile)
    traces = [in_batches(tg.make_trace(int(rng.integers(0, 1 << 30)), int(rng.integers(1, 5)), int(rng.integers(1, 5)),
                                       int(rng.integers(1, 4)), int(rng.integers(20, 600)), int(rng.integers(10, 200)),
                                       regions="nested", n_regions=3), rng, 60, False) for _ in range(30)]
    sessions = [new_session(tr, tuning={"bucket_target": 64, "tile_elems": tile})[0] for tr in traces]
    try:
        first = hp.hpop_batch_compute(sessions, hp.HPOP_FORCE_REBUILD)
        again = hp.hpop_batch_compute(sessions, hp.HPOP_FORCE_REBUILD)
        k = 0
        for tr in traces:
            want = oracle.compute(tr)
            for g in range(len(tr.regions)):
                np.testing.assert_array_equal(hp.tree_sums(first[k]), want["sums"][g])
                np.testing.assert_array_equal(hp.tree_ratios(first[k]).view(np.int64), want["ratios"][g].view(np.int64))
                assert bytes(first[k]) == bytes(again[k])
                k += 1
    finally:
        for s in sessions:
            hp.hpop_session_destroy(s)


def many_resources_trace(seed, n_hosts, n_devices, big_every):
    """Mostly resources of 0-40 records (one bucket each), every big_every-th
    one with thousands (many buckets)."""
    rng = np.random.default_rng(seed)
    chunks = []
    for r in range(n_hosts + n_devices):
        n = int(rng.integers(3000, 6000)) if r % big_every == 0 else int(rng.integers(0, 41))
        if n == 0:
            continue
        s = np.sort(rng.integers(0, 1 << 30, size=n)).astype(np.int64)
        e = s + rng.integers(0, 1 << 22, size=n)
        kinds = (tg.HOST_USEFUL, tg.HOST_OFFLOAD, tg.HOST_MPI) if r < n_hosts else (tg.DEV_KERNEL, tg.DEV_MEMOP)
        k = rng.integers(0, len(kinds), size=n)
        for i, kd in enumerate(kinds):
            if (k == i).any():
                chunks.append(tg.Chunk(r, kd, s[k == i], e[k == i]))
    return tg.Trace(n_hosts, n_devices, chunks, [(0, 1 << 30), (1 << 28, 1 << 29), (12345, (1 << 30) + (1 << 22))])


@pytest.mark.parametrize("tuning", [{"bucket_target": 64, "tile_elems": 512},
                                    {"bucket_target": 16, "tile_elems": 2048, "scatter_slots": -1}])
def test_thousands_of_small_resources(tuning):
    """5000 resources, most of a bucket or two: the per-resource passes take
    them eight to a wave; the large ones among them take a whole wave."""
    check(many_resources_trace(12, 3000, 2000, 97), tuning)


@pytest.mark.parametrize("device", [False, True])
def test_batch_sees_records_added_between_batched_calls(device):
    """Each session copies its records on its own stream; a batched call waits
    only for sessions that copied records since the last wait. Records added
    after one batched call (to a session that is not the first) are in the
    next one, and a call with nothing new repeats the same trees."""
    rng = np.random.default_rng(31)
    traces = [tg.make_trace(int(rng.integers(0, 1 << 30)), 2, 2, 2, 3000, 800, regions="nested", n_regions=2)
              for _ in range(6)]
    halves = []
    for tr in traces:
        first, second = [], []
        for c in tr.chunks:
            h = len(c.start) // 2
            first.append(tg.Chunk(c.resource, c.kind, c.start[:h].copy(), c.end[:h].copy()))
            second.append(tg.Chunk(c.resource, c.kind, c.start[h:].copy(), c.end[h:].copy()))
        halves.append((tg.Trace(tr.n_hosts, tr.n_devices, first, list(tr.regions)), second))
    sessions, keep = [], []
    try:
        for tr, _ in halves:
            s, kp = new_session(tr, device=device, tuning={"bucket_target": 64, "tile_elems": 512})
            sessions.append(s)
            keep.append(kp)

        def check_all(trees, trs):
            k = 0
            for tr in trs:
                want = oracle.compute(tr)
                for g in range(len(tr.regions)):
                    np.testing.assert_array_equal(hp.tree_sums(trees[k]), want["sums"][g])
                    np.testing.assert_array_equal(hp.tree_ratios(trees[k]).view(np.int64),
                                                  want["ratios"][g].view(np.int64))
                    k += 1

        check_all(hp.hpop_batch_compute(sessions), [tr for tr, _ in halves])
        # the second half of sessions 2 and 5 only, then at once a batched call
        for i in (2, 5):
            keep.append(hp.add_chunks(sessions[i], [(c.resource, c.kind, c.start, c.end) for c in halves[i][1]],
                                      device=device))
        now = [traces[i] if i in (2, 5) else halves[i][0] for i in range(len(traces))]
        got = hp.hpop_batch_compute(sessions)
        check_all(got, now)
        again = hp.hpop_batch_compute(sessions, hp.HPOP_FORCE_REBUILD)
        for a, b in zip(got, again):
            assert bytes(a) == bytes(b)
    finally:
        for s in sessions:
            hp.hpop_session_destroy(s)


def test_slot_overflow_in_shared_tiles_falls_back_to_exact_offsets():
    """Small batches (shared tiles) whose buckets outgrow 64 fixed scatter
    slots: the build is redone with exact offsets (count pass included) and
    gives the oracle's results; with enough slots the single pass is back."""
    rng = np.random.default_rng(17)
    base = tg.make_trace(44, 3, 3, 4, 6000, 1500, w_range=(0.5, 1.5), regions="nested", n_regions=3)
    tr = in_batches(base, rng, 120, True)
    want = oracle.compute(tr)
    s, keep = new_session(tr)
    try:
        hp.hpop_session_enable_timing(s, 1)
        for tuning, exact in (({"bucket_target": 256, "tile_elems": 512, "scatter_slots": 64}, True),
                              ({"bucket_target": 256, "tile_elems": 512}, False)):
            print("case: tuning=%s" % tuning, flush=True)
            hp.hpop_session_set_tuning(s, **tuning)
            assert_same(engine_results(s, tr, hp.HPOP_FORCE_REBUILD), want, str(tuning))
            names = [n for n, _ in hp.hpop_session_stage_times(s)]
            assert ("hist" in names) == exact, (tuning, names)
    finally:
        hp.hpop_session_destroy(s)
