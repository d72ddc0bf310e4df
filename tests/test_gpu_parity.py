"""GPU parity: the HIP engine, called through its C ABI, against the CPU oracle.

Integers (state times, sums, maxima) must be bit-exact; the FP64 ratios come
from the same exact integers through one IEEE division each, so they must be
bit-identical (the stated bound is 1e-15 relative; the test demands 0).
"""
import numpy as np
import pytest

import oracle
import paper_2603_26576_amd as hp
import tracegen as tg
import pils
from engine_util import assert_same, engine_results, gpu_available, new_session, run_engine

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")
    hp.lib()


def check(trace, **kw):
    print("case: n=%d m=%d events=%d regions=%d %s" % (trace.n_hosts, trace.n_devices, trace.n_events,
                                                        len(trace.regions), kw), flush=True)
    want = oracle.compute(trace)
    got = run_engine(trace, **kw)
    assert_same(got, want, str(kw))
    return got


@pytest.mark.parametrize("case", pils.load(), ids=lambda c: c[0])
def test_pils_tables(case):
    name, printed, t = case
    for variant in ({}, {"kernel_streams": 4, "hidden_memops": 3}, {"t0": tg.T0}):
        got = check(pils.build_trace(t, **variant))
        assert np.all(np.abs(got["ratios"][0] - np.array(printed)) <= 0.005 + 1e-12)


@pytest.mark.parametrize("seed", range(40))
def test_random_tiny(seed):
    rng = np.random.default_rng(1000 + seed)
    tr = tg.random_tiny(rng, max_span=int(rng.integers(2, 5000)), max_events=int(rng.integers(1, 300)),
                        t0=int(rng.integers(0, 1 << 61)), n_regions=4)
    check(tr)


def test_small_config_full_size():
    check(tg.small())


def test_mid_config_scaled():
    check(tg.mid(scale=0.02))


def test_large_config_scaled():
    check(tg.large(scale=0.004, ranks=32))


def test_device_pointer_input_matches_host_input():
    tr = tg.make_trace(21, 5, 5, 4, 3000, 1000, regions="tiles", n_regions=7)
    a = run_engine(tr)
    b = run_engine(tr, device=True)
    assert_same(b, a, "device input")


@pytest.mark.parametrize("tuning", [
    {"bucket_target": 16, "bucket_cap": 2048, "tile_elems": 2048},
    {"bucket_target": 256, "bucket_cap": 4096, "tile_elems": 8192},
    {"bucket_target": 4096, "bucket_cap": 2048, "tile_elems": 4096},
    {"bucket_target": 4096, "bucket_cap": 4096, "tile_elems": 2048},
    {"bucket_target": 256, "scatter_slots": -1},
    {"bucket_target": 64, "scatter_slots": 64},
    {"bucket_target": 256, "bucket_cap": 2048, "tile_elems": 512},
    {"bucket_target": 64, "tile_elems": 512, "scatter_slots": -1},
])
def test_tunings_agree(tuning):
    tr = tg.make_trace(22, 4, 4, 8, 20000, 5000, w_range=(0.5, 1.5), regions="nested", n_regions=6)
    check(tr, tuning=tuning)


def test_block_path_queue_longer_than_its_grid():
    """Buckets of about 1024 records all leave the wave path (at most 512
    records); more of them than the block path has workgroups (1024), so the
    workgroups take them from the shared counter instead of by index."""
    tr = tg.make_trace(24, 4, 4, 4, 250000, 60000, w_range=(0.5, 1.5), regions="nested", n_regions=4)
    sizes = {}
    for c in tr.chunks:
        sizes[c.resource] = sizes.get(c.resource, 0) + c.start.size
    buckets = sum(-(-n // 1024) for n in sizes.values())
    assert buckets > 1024, buckets
    check(tr, tuning={"bucket_target": 1024, "bucket_cap": 2048, "tile_elems": 2048})


def test_slot_overflow_does_not_outlive_its_tuning():
    """A tuning whose scatter slots overflow falls back to exact offsets
    (k_hist); a later tuning with large enough slots takes the single-pass
    scatter again, single session and batched, with the same results."""
    tr = tg.make_trace(23, 3, 3, 4, 20000, 5000, w_range=(0.5, 1.5), regions="nested", n_regions=4)
    want = oracle.compute(tr)
    s, keep = new_session(tr)
    s2, keep2 = new_session(tr)
    try:
        for ss in ([s], [s, s2]):
            for x in ss:
                hp.hpop_session_enable_timing(x, 1)
            for tuning, exact in (({"bucket_target": 256, "scatter_slots": 64}, True),
                                  ({"bucket_target": 256}, False)):
                print("case: sessions=%d tuning=%s" % (len(ss), tuning), flush=True)
                for x in ss:
                    hp.hpop_session_set_tuning(x, **tuning)
                if len(ss) == 1:
                    got = engine_results(s, tr, hp.HPOP_FORCE_REBUILD)
                    assert_same(got, want, str(tuning))
                else:
                    trees = hp.hpop_batch_compute(ss, hp.HPOP_FORCE_REBUILD)
                    for g, t in enumerate(trees):
                        np.testing.assert_array_equal(hp.tree_sums(t), want["sums"][g % len(tr.regions)])
                names = [n for n, _ in hp.hpop_session_stage_times(s)]
                assert ("hist" in names) == exact, (tuning, names)
    finally:
        hp.hpop_session_destroy(s)
        hp.hpop_session_destroy(s2)


def test_oversized_bucket_slow_path():
    """Most starts packed in a few ns with one far outlier: one bucket gets
    every record and must take the global-memory sort path."""
    rng = np.random.default_rng(5)
    n = 30000
    s = rng.integers(0, 3000, size=n).astype(np.int64)
    e = s + rng.integers(1, 50, size=n)
    s[-1], e[-1] = 10 ** 9, 10 ** 9 + 5
    k = rng.random(n) < 0.3
    chunks = [tg.Chunk(0, tg.DEV_KERNEL, s[~k], e[~k]), tg.Chunk(0, tg.DEV_MEMOP, s[k], e[k])]
    hs = np.sort(rng.integers(0, 5000, size=9000)).astype(np.int64)
    chunks.append(tg.Chunk(1, tg.DEV_KERNEL, hs, hs + 3))
    tr = tg.Trace(0, 2, chunks, [(0, 10 ** 9 + 10), (100, 2000), (1500, 10 ** 9 + 1)])
    got = check(tr)
    s_ = hp.hpop_session_create(0, 2)
    try:
        hp.add_chunks(s_, [(c.resource, c.kind, c.start, c.end) for c in tr.chunks])
        for a, b in tr.regions:
            hp.hpop_region_define(s_, a, b)
        hp.hpop_metrics_compute_all(s_)
        assert hp.hpop_session_get_info(s_).n_oversized >= 1
    finally:
        hp.hpop_session_destroy(s_)


def test_crowded_sub_bins_fall_back_to_block_path():
    """A bucket small enough for one wave but with hundreds of starts packed in
    one sub-bin of the wave path's counting sort."""
    rng = np.random.default_rng(9)
    spread = rng.integers(0, 1 << 22, size=150)
    packed = 5000 + rng.integers(0, 60, size=250)
    s = np.concatenate([spread, packed]).astype(np.int64)
    e = s + rng.integers(1, 900, size=s.size)
    k = rng.random(s.size) < 0.4
    chunks = [tg.Chunk(0, tg.DEV_KERNEL, s[~k], e[~k]), tg.Chunk(0, tg.DEV_MEMOP, s[k], e[k]),
              tg.Chunk(1, tg.HOST_USEFUL, s[:200], e[:200]), tg.Chunk(1, tg.HOST_MPI, s[200:], e[200:] + 7)]
    tr = tg.Trace(0, 1, chunks[:2], [(0, 1 << 23), (5000, 5030), (4000, 6000)])
    check(tr)
    tr2 = tg.Trace(1, 0, [tg.Chunk(0, c.kind, c.start, c.end) for c in chunks[2:]], tr.regions)
    check(tr2)


@pytest.mark.parametrize("n", [2, 60, 200, 300, 512])
def test_largest_narrow_key(n):
    """One bucket 2^30 ns wide (the widest the 8 B form holds) whose records
    include starts at its first time and 2^30 - 1 ns after it: the largest
    key the wave path sorts. One bucket per resource (target 512), so every
    wave size of the path is taken, for a device (2 levels) and a host (3)."""
    rng = np.random.default_rng(7000 + n)
    t0 = 1 << 40
    chunks = []
    for res, kinds in ((0, (tg.HOST_USEFUL, tg.HOST_OFFLOAD, tg.HOST_MPI)), (1, (tg.DEV_KERNEL, tg.DEV_MEMOP))):
        s = np.sort(rng.integers(t0, t0 + (1 << 30), size=n)).astype(np.int64)
        s[0], s[-1] = t0, t0 + (1 << 30) - 1
        e = s + rng.integers(0, 1 << 22, size=n)
        e[-1] = s[-1] + int(rng.integers(0, 3))
        k = rng.integers(0, len(kinds), size=n)
        for i, kind in enumerate(kinds):
            if np.any(k == i):
                chunks.append(tg.Chunk(res, kind, s[k == i], e[k == i]))
    tr = tg.Trace(1, 1, chunks, [(t0, t0 + (1 << 31)), (t0 + (1 << 29), t0 + (1 << 30) - 1),
                                 (t0 + (1 << 30) - 2, t0 + (1 << 30) + 5)])
    check(tr, tuning={"bucket_target": 512, "bucket_cap": 2048, "tile_elems": 2048})


def test_long_intervals_and_wide_buckets():
    """Buckets the wave path's 32-bit form cannot hold: records ending 2^32 ns
    or more after their bucket's start, and sparse resources whose buckets are
    wider than 2^30 ns. They take the block path; the rest stays on the wave
    path, and the carry between the two kinds of bucket must line up."""
    rng = np.random.default_rng(13)
    chunks = []
    # dense resource with a few very long records sprinkled in
    s = np.sort(rng.integers(0, 1 << 34, size=60000)).astype(np.int64)
    e = s + rng.integers(0, 2000, size=s.size)
    far = rng.random(s.size) < 0.002
    e[far] = s[far] + rng.integers(1 << 32, 1 << 35, size=int(far.sum()))
    k = rng.random(s.size) < 0.35
    chunks += [tg.Chunk(0, tg.DEV_KERNEL, s[~k], e[~k]), tg.Chunk(0, tg.DEV_MEMOP, s[k], e[k])]
    # sparse resource: 3000 records over 2^45 ns, buckets far wider than 2^30
    s2 = np.sort(rng.integers(0, 1 << 45, size=3000)).astype(np.int64)
    e2 = s2 + rng.integers(0, 1 << 40, size=s2.size)
    chunks.append(tg.Chunk(1, tg.DEV_KERNEL, s2, e2))
    # host with long MPI states next to short useful ones
    s3 = np.sort(rng.integers(0, 1 << 36, size=20000)).astype(np.int64)
    kinds = rng.integers(0, 3, size=s3.size)
    e3 = s3 + np.where(kinds == 2, rng.integers(1 << 31, 1 << 33, size=s3.size), rng.integers(0, 5000, size=s3.size))
    host = [tg.Chunk(0, kd, s3[kinds == kd], e3[kinds == kd]) for kd in (tg.HOST_USEFUL, tg.HOST_OFFLOAD, tg.HOST_MPI)]
    regions = [(0, 1 << 46), (1 << 20, 1 << 33), (5 << 30, 7 << 30)]
    check(tg.Trace(0, 2, chunks, regions))
    check(tg.Trace(1, 0, host, regions))
    # the sparse resource keeps 16 B components and records, the dense one
    # 8 B ones
    s_ = hp.hpop_session_create(0, 2)
    try:
        hp.add_chunks(s_, [(c.resource, c.kind, c.start, c.end) for c in chunks])
        hp.hpop_region_define(s_, 0, 1 << 46)
        hp.hpop_metrics_compute_all(s_)
        info = hp.hpop_session_get_info(s_)
        assert 0 < info.n_wide_components < info.n_components
        # only the sparse resource's records take the 16 B form; the dense
        # resource's far ends are clamped in the 8 B form
        assert info.n_wide_records == len(s2)
    finally:
        hp.hpop_session_destroy(s_)


def long_interval_traces(seed):
    """A dense device resource with far-ending records next to a sparse one
    (buckets wider than 2^30 ns), and a host with long MPI states."""
    rng = np.random.default_rng(seed)
    s = np.sort(rng.integers(0, 1 << 34, size=20000)).astype(np.int64)
    e = s + rng.integers(0, 2000, size=s.size)
    far = rng.random(s.size) < 0.003
    e[far] = s[far] + rng.integers(1 << 32, 1 << 35, size=int(far.sum()))
    k = rng.random(s.size) < 0.35
    s2 = np.sort(rng.integers(0, 1 << 45, size=1500)).astype(np.int64)
    e2 = s2 + rng.integers(0, 1 << 40, size=s2.size)
    dev = [tg.Chunk(0, tg.DEV_KERNEL, s[~k], e[~k]), tg.Chunk(0, tg.DEV_MEMOP, s[k], e[k]),
           tg.Chunk(1, tg.DEV_KERNEL, s2, e2)]
    s3 = np.sort(rng.integers(0, 1 << 36, size=8000)).astype(np.int64)
    kinds = rng.integers(0, 3, size=s3.size)
    e3 = s3 + np.where(kinds == 2, rng.integers(1 << 31, 1 << 33, size=s3.size), rng.integers(0, 5000, size=s3.size))
    host = [tg.Chunk(0, kd, s3[kinds == kd], e3[kinds == kd]) for kd in (tg.HOST_USEFUL, tg.HOST_OFFLOAD, tg.HOST_MPI)]
    regions = [(0, 1 << 46), (1 << 20, 1 << 33), (5 << 30, 7 << 30)]
    return tg.Trace(0, 2, dev, regions), tg.Trace(1, 0, host, regions)


def test_batched_mixed_record_forms():
    """One batched build over traces whose resources take the 8 B form (with
    clamped far ends), the 16 B form, or are tiny."""
    rng = np.random.default_rng(91)
    traces = list(long_interval_traces(92)) + [tg.random_tiny(rng, max_span=3000, max_events=200, t0=int(rng.integers(0, 1 << 60)),
                                                             n_regions=3) for _ in range(4)]
    sessions = []
    try:
        for tr in traces:
            s, _ = new_session(tr)
            sessions.append(s)
        for flags in (0, hp.HPOP_FORCE_REBUILD):
            trees = hp.hpop_batch_compute(sessions, flags)
            k = 0
            for tr in traces:
                want = oracle.compute(tr)
                for g in range(len(tr.regions)):
                    np.testing.assert_array_equal(hp.tree_sums(trees[k]), want["sums"][g])
                    np.testing.assert_array_equal(hp.tree_ratios(trees[k]).view(np.int64),
                                                  want["ratios"][g].view(np.int64))
                    k += 1
    finally:
        for s in sessions:
            hp.hpop_session_destroy(s)


def test_identical_starts_and_degenerate_intervals():
    n = 5000
    s = np.full(n, 7_000_000, np.int64)
    e = s + np.arange(n) % 17  # many empty intervals
    chunks = [tg.Chunk(0, tg.HOST_USEFUL, s, e), tg.Chunk(0, tg.HOST_MPI, s - 3, s + 40),
              tg.Chunk(1, tg.DEV_KERNEL, np.array([5, 5, 5, 9], np.int64), np.array([5, 9, 9, 9], np.int64)),
              tg.Chunk(1, tg.DEV_MEMOP, np.array([0, 9], np.int64), np.array([20, 9], np.int64))]
    tr = tg.Trace(1, 1, chunks, [(0, 8_000_000), (7_000_001, 7_000_016), (6, 7)])
    check(tr)


def test_resources_without_records_and_empty_session():
    tr = tg.Trace(3, 2, [tg.Chunk(1, tg.HOST_USEFUL, np.array([10], np.int64), np.array([20], np.int64))],
                  [(0, 100)])
    check(tr)
    check(tg.Trace(2, 2, [], [(0, 100), (5, 6)]))


def test_extreme_timestamps():
    top = (1 << 62) - 1
    chunks = [tg.Chunk(0, tg.DEV_KERNEL, np.array([0, top - 10, top - 5], np.int64),
                       np.array([3, top - 1, top], np.int64)),
              tg.Chunk(0, tg.DEV_MEMOP, np.array([1, top - 20], np.int64), np.array([top - 30, top - 2], np.int64))]
    tr = tg.Trace(0, 1, chunks, [(top - (1 << 52), top), (0, 1 << 40)])
    check(tr)


def test_repeated_builds_identical_and_graph_replay():
    tr = tg.make_trace(31, 6, 6, 4, 20000, 4000, regions="tiles", n_regions=5)
    want = oracle.compute(tr)
    s, keep = new_session(tr)
    try:
        for _ in range(5):
            got = engine_results(s, tr, flags=hp.HPOP_FORCE_REBUILD)
            assert_same(got, want, "replay")
        replays = hp.hpop_session_get_info(s).graph_replays
        assert replays >= 4
        # kernels launched one by one: same results, no replay
        for _ in range(2):
            got = engine_results(s, tr, flags=hp.HPOP_FORCE_REBUILD | hp.HPOP_NO_GRAPH)
            assert_same(got, want, "direct launches")
        assert hp.hpop_session_get_info(s).graph_replays == replays
        assert_same(engine_results(s, tr, flags=hp.HPOP_FORCE_REBUILD), want, "replay after direct launches")
    finally:
        hp.hpop_session_destroy(s)


def test_incremental_add_and_new_region():
    tr = tg.make_trace(32, 4, 4, 4, 5000, 2000, regions="nested", n_regions=3)
    half = len(tr.chunks) // 2
    first = tg.Trace(tr.n_hosts, tr.n_devices, tr.chunks[:half], tr.regions)
    s, keep = new_session(first)
    try:
        assert_same(engine_results(s, first), oracle.compute(first), "first half")
        keep2 = hp.add_chunks(s, [(c.resource, c.kind, c.start, c.end) for c in tr.chunks[half:]])
        assert_same(engine_results(s, tr), oracle.compute(tr), "all")
        lo, hi = tr.span()
        hp.hpop_region_define(s, lo + 1000, hi - 999)
        tr2 = tg.Trace(tr.n_hosts, tr.n_devices, tr.chunks, tr.regions + [(lo + 1000, hi - 999)])
        assert_same(engine_results(s, tr2), oracle.compute(tr2), "new region")
    finally:
        hp.hpop_session_destroy(s)


def test_invalid_device_record_reported_and_dropped():
    import torch
    good = tg.make_trace(33, 2, 2, 2, 500, 200)
    s, keep = new_session(good)
    try:
        bad_s = torch.tensor([10, 20, 30], dtype=torch.int64, device="cuda")
        bad_e = torch.tensor([11, 19, 31], dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        hp.hpop_add_events(s, 2, hp.HPOP_DEV_KERNEL, bad_s, bad_e)
        with pytest.raises(hp.HpopError) as ei:
            hp.hpop_metrics_compute_all(s)
        assert ei.value.status == hp.HPOP_E_BAD_INTERVAL
        assert "index 1" in ei.value.message
        # the offending call was dropped: the session equals the good trace again
        assert_same(engine_results(s, good), oracle.compute(good), "after drop")
    finally:
        hp.hpop_session_destroy(s)


def test_batched_small_tiles():
    """Many traces of small record batches with 512-record tiles (the tiles of
    the streaming passes, each holding one batch, mostly partly filled)."""
    rng = np.random.default_rng(61)
    traces = [tg.make_trace(int(rng.integers(0, 1 << 30)), int(rng.integers(1, 6)), int(rng.integers(1, 6)),
                            int(rng.integers(1, 5)), int(rng.integers(50, 3000)), int(rng.integers(20, 800)),
                            regions="nested", n_regions=3) for _ in range(40)]
    sessions = [new_session(tr, tuning={"bucket_target": 64, "tile_elems": 512})[0] for tr in traces]
    try:
        trees = hp.hpop_batch_compute(sessions)
        k = 0
        for tr in traces:
            want = oracle.compute(tr)
            for g in range(len(tr.regions)):
                np.testing.assert_array_equal(hp.tree_sums(trees[k]), want["sums"][g])
                np.testing.assert_array_equal(hp.tree_ratios(trees[k]).view(np.int64), want["ratios"][g].view(np.int64))
                k += 1
    finally:
        for s in sessions:
            hp.hpop_session_destroy(s)


def test_batched_equals_single():
    traces = tg.batched(seed=77, n_traces=12, max_events=3e4)
    sessions = []
    try:
        for tr in traces:
            s, _ = new_session(tr)
            sessions.append(s)
        trees = hp.hpop_batch_compute(sessions)
        k = 0
        for tr in traces:
            want = oracle.compute(tr)
            for g in range(len(tr.regions)):
                np.testing.assert_array_equal(hp.tree_sums(trees[k]), want["sums"][g])
                np.testing.assert_array_equal(hp.tree_ratios(trees[k]).view(np.int64),
                                              want["ratios"][g].view(np.int64))
                k += 1
        # replayed graph gives the same trees
        again = hp.hpop_batch_compute(sessions, hp.HPOP_FORCE_REBUILD)
        for a, b in zip(trees, again):
            np.testing.assert_array_equal(hp.tree_sums(a), hp.tree_sums(b))
    finally:
        for s in sessions:
            hp.hpop_session_destroy(s)


def multi_session(trace, multi):
    s, keep = new_session(trace)
    for ivls in multi:
        hp.hpop_region_define_multi(s, ivls)
    return s, keep


@pytest.mark.parametrize("seed", range(12))
def test_regions_entered_repeatedly(seed):
    """Per-resource interval lists against the oracle's definition, next to
    ordinary regions of the same session (those stay as before)."""
    rng = np.random.default_rng(6000 + seed)
    tr = tg.make_trace(seed, int(rng.integers(1, 5)), int(rng.integers(1, 5)), 3, int(rng.integers(50, 3000)),
                       int(rng.integers(20, 800)), regions="tiles", n_regions=3)
    R = tr.n_hosts + tr.n_devices
    lo, hi = tr.info["t0"], tr.info["t_end"]
    multi = []
    for _ in range(3):
        ivls = []
        for r in range(R):
            k = int(rng.integers(0, 5))
            cuts = np.sort(rng.choice(np.arange(lo - 1000, hi + 1000, max(1, (hi - lo) // 5000)), size=2 * k,
                                      replace=False)) if k else []
            ivls += [(r, int(cuts[2 * i]), int(cuts[2 * i + 1])) for i in range(k) if cuts[2 * i] < cuts[2 * i + 1]]
        if not ivls:
            ivls = [(0, lo, hi)]
        multi.append(ivls)
    want = oracle.compute_multi(tr, multi)
    want_plain = oracle.compute(tr)
    s, keep = multi_session(tr, multi)
    try:
        for flags in (0, hp.HPOP_FORCE_REBUILD):
            trees = hp.hpop_metrics_compute_all(s, flags)
            G = len(tr.regions)
            for g in range(G):
                np.testing.assert_array_equal(hp.tree_sums(trees[g]), want_plain["sums"][g])
            for j in range(len(multi)):
                t = trees[G + j]
                assert t.E == want["E"][j]
                np.testing.assert_array_equal(hp.tree_sums(t), want["sums"][j], err_msg="multi %d" % j)
                np.testing.assert_array_equal(hp.tree_ratios(t).view(np.int64), want["ratios"][j].view(np.int64))
                assert t.undefined_mask == want["mask"][j]
                for r in range(R):
                    np.testing.assert_array_equal(hp.hpop_resource_times(s, G + j, r), want["times"][j][r])
    finally:
        hp.hpop_session_destroy(s)


def test_region_define_multi_errors():
    s = hp.hpop_session_create(2, 1)
    try:
        for bad, code in [([(3, 0, 10)], hp.HPOP_E_RESOURCE), ([(0, 5, 5)], hp.HPOP_E_REGION),
                          ([(0, 0, 10), (0, 5, 20)], hp.HPOP_E_REGION), ([(0, 0, 1 << 52)], hp.HPOP_E_OVERFLOW)]:
            with pytest.raises(hp.HpopError) as ei:
                hp.hpop_region_define_multi(s, bad)
            assert ei.value.status == code
        assert hp.hpop_num_regions(s) == 0
        assert hp.hpop_region_define_multi(s, [(0, 0, 10), (0, 10, 20), (2, 3, 4)]) == 0
    finally:
        hp.hpop_session_destroy(s)
