"""Stream concurrency on the GPU (hpop_session_set_streams, hpop_add_stream_events,
hpop_stream_metrics) against oracle.compute_streams: the integers exactly, the
two FP64 ratios bit for bit, the 0/0 flags; the stream records also count as
kernel records in the device tree; error paths leave the session unchanged."""
import numpy as np
import pytest

import oracle
import paper_2603_26576_amd as hp
import tracegen as tg
from engine_util import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")
    hp.lib()


def run(n_hosts, n_streams, chunks, regions, device=False, tuning=None):
    m = len(n_streams)
    s = hp.hpop_session_create(n_hosts, m)
    keep = []
    try:
        if tuning:
            hp.hpop_session_set_tuning(s, **tuning)
        hp.hpop_session_set_streams(s, n_streams)
        for g, st, a, b in chunks:
            a = np.ascontiguousarray(a, np.int64)
            b = np.ascontiguousarray(b, np.int64)
            if device:
                import torch
                a, b = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
                torch.cuda.synchronize()
            keep.append((a, b))
            hp.hpop_add_stream_events(s, n_hosts + g, st, a, b)
        for t0, t1 in regions:
            hp.hpop_region_define(s, t0, t1)
        trees, per = hp.hpop_stream_metrics(s, n_devices=m)
        main = hp.hpop_metrics_compute_all(s)
        K = np.array([[hp.hpop_resource_times(s, r, n_hosts + g)[0] for g in range(m)]
                      for r in range(len(regions))], np.int64).reshape(len(regions), m)
        return trees, per, main, K
    finally:
        hp.hpop_session_destroy(s)


def check(n_hosts, n_streams, chunks, regions, **kw):
    print("case: devices=%d streams=%s records=%d regions=%d %s" % (
        len(n_streams), sorted(set(n_streams)), sum(len(c[2]) for c in chunks), len(regions), kw), flush=True)
    want = oracle.compute_streams(n_streams, chunks, regions)
    trees, per, main, K = run(n_hosts, n_streams, chunks, regions, **kw)
    np.testing.assert_array_equal(per, want["per_device"])
    got_sums = np.array([[t.busy, t.stream_time, t.capacity] for t in trees], np.int64).reshape(-1, 3)
    np.testing.assert_array_equal(got_sums, want["sums"])
    got_r = np.array([[t.stream_eff, t.mean_active] for t in trees], np.float64).reshape(-1, 2)
    np.testing.assert_array_equal(got_r.view(np.int64), want["ratios"].view(np.int64))
    np.testing.assert_array_equal(np.array([t.undefined_mask for t in trees], np.uint32), want["mask"])
    for t in trees:
        assert t.m == len(n_streams) and t.n_streams == sum(n_streams)
    # the stream records are kernel records of the device tree: its K is the busy time
    np.testing.assert_array_equal(K, want["per_device"][:, :, 0])
    return trees


def random_case(rng, m, max_streams, span, max_rec):
    n_streams = [int(rng.integers(0, max_streams + 1)) for _ in range(m)]
    chunks = []
    for g in range(m):
        for st in range(n_streams[g]):
            if rng.random() < 0.2:
                continue
            for _ in range(int(rng.integers(1, 3))):
                k = int(rng.integers(0, max_rec))
                s = rng.integers(0, span, size=k).astype(np.int64)
                e = s + rng.integers(0, span // 8 + 1, size=k)
                chunks.append((g, st, s, e))
    return n_streams, chunks


@pytest.mark.parametrize("seed", range(12))
def test_random_small(seed):
    rng = np.random.default_rng(900 + seed)
    n_streams, chunks = random_case(rng, int(rng.integers(1, 6)), 5, int(rng.integers(50, 5000)), 60)
    hi = max([int(c[3].max()) for c in chunks if len(c[3])] + [10])
    regions = [(0, hi + 1), (hi // 3, hi // 2 + 1), (hi + 5, hi + 9)]
    check(int(rng.integers(0, 3)), n_streams, chunks, regions, device=bool(seed % 2))


@pytest.mark.parametrize("streams", [1, 4, 16])
def test_launch_groups_many_buckets(streams):
    """Generator-shaped streams at sizes spanning many tiles and buckets, with
    a ragged tail per stream."""
    n_streams, chunks = tg.stream_kernels(77 + streams, 6, streams, 30_011)
    lo = min(int(c[2].min()) for c in chunks)
    hi = max(int(c[3].max()) for c in chunks)
    cuts = np.linspace(lo, hi, 9).astype(np.int64)
    regions = [(lo, hi)] + [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:])] + [(lo + 1, lo + 2)]
    trees = check(2, n_streams, chunks, regions, tuning={"bucket_target": 128})
    if streams == 1:
        assert trees[0].stream_eff == 1.0 and trees[0].mean_active == 1.0


def test_identical_and_alternating_streams():
    t = np.arange(0, 40_000, 10, dtype=np.int64)
    S = 4
    same = [(0, k, t, t + 10) for k in range(S)]
    turns = [(1, k, t[k::S], t[k::S] + 10) for k in range(S)]
    trees = check(0, [S, S], same + turns, [(0, 40_000), (100, 105)])
    per = oracle.compute_streams([S, S], same + turns, [(0, 40_000)])["per_device"][0]
    assert tuple(per[0]) == (40_000, 4 * 40_000, S) and tuple(per[1]) == (40_000, 40_000, S)
    assert trees[0].stream_eff == 5 * 40_000 / (2 * S * 40_000)


def test_undefined_and_idle():
    # declared streams with no records, and a device with no streams at all
    trees = check(1, [3, 0], [], [(0, 100)])
    assert trees[0].undefined_mask == 0b11 and trees[0].stream_eff == 1.0


def test_errors_leave_the_session_unchanged():
    s = hp.hpop_session_create(1, 2)
    try:
        a = np.array([5, 10], np.int64)
        b = np.array([8, 30], np.int64)
        with pytest.raises(hp.HpopError) as e:
            hp.hpop_add_stream_events(s, 1, 0, a, b)
        assert e.value.status == hp.HPOP_E_STATE
        with pytest.raises(hp.HpopError) as e:
            hp.hpop_stream_metrics(s)
        assert e.value.status == hp.HPOP_E_STATE
        with pytest.raises(hp.HpopError) as e:
            hp.hpop_session_set_streams(s, [1, -1])
        assert e.value.status == hp.HPOP_E_ARG
        hp.hpop_session_set_streams(s, [2, 1])
        for res, st in ((0, 0), (3, 0), (1, 2), (2, 1), (1, -1)):
            with pytest.raises(hp.HpopError) as e:
                hp.hpop_add_stream_events(s, res, st, a, b)
            assert e.value.status == hp.HPOP_E_RESOURCE, (res, st)
        with pytest.raises(hp.HpopError) as e:
            hp.hpop_add_stream_events(s, 1, 0, np.array([5, 10], np.int64), np.array([8, 9], np.int64))
        assert e.value.status == hp.HPOP_E_BAD_INTERVAL
        hp.hpop_add_stream_events(s, 1, 1, a, b)
        with pytest.raises(hp.HpopError) as e:
            hp.hpop_session_set_streams(s, [3, 3])
        assert e.value.status == hp.HPOP_E_STATE
        hp.hpop_region_define(s, 0, 40)
        trees, per = hp.hpop_stream_metrics(s, n_devices=2)
        want = oracle.compute_streams([2, 1], [(0, 1, a, b)], [(0, 40)])
        np.testing.assert_array_equal(per, want["per_device"])
        assert hp.hpop_session_get_info(s).n_events == 2
        hp.hpop_region_define_multi(s, [(0, 0, 10), (1, 5, 20)])
        with pytest.raises(hp.HpopError) as e:
            hp.hpop_stream_metrics(s)
        assert e.value.status == hp.HPOP_E_REGION
        # clearing the records clears the stream records too
        hp.hpop_clear_events(s)
        s2 = hp.hpop_session_create(1, 2)
        hp.hpop_session_destroy(s2)
    finally:
        hp.hpop_session_destroy(s)
    s = hp.hpop_session_create(0, 1)
    try:
        hp.hpop_session_set_streams(s, [1 << 20])
        hp.hpop_region_define(s, 0, 1 << 40)
        with pytest.raises(hp.HpopError) as e:
            hp.hpop_stream_metrics(s)
        assert e.value.status == hp.HPOP_E_OVERFLOW
    finally:
        hp.hpop_session_destroy(s)


def test_cleared_session_and_records_added_later():
    n_streams, chunks = tg.stream_kernels(5, 3, 3, 3000)
    lo = min(int(c[2].min()) for c in chunks)
    hi = max(int(c[3].max()) for c in chunks)
    s = hp.hpop_session_create(0, 3)
    try:
        hp.hpop_session_set_streams(s, n_streams)
        for g, st, a, b in chunks[:4]:
            hp.hpop_add_stream_events(s, g, st, a, b)
        hp.hpop_region_define(s, lo, hi)
        hp.hpop_stream_metrics(s)
        hp.hpop_clear_events(s)
        hp.hpop_session_set_streams(s, n_streams)  # allowed again: no stream record left
        for g, st, a, b in chunks:
            hp.hpop_add_stream_events(s, g, st, a, b)
        hp.hpop_region_define(s, (lo + hi) // 2, hi)
        trees, per = hp.hpop_stream_metrics(s, n_devices=3)
        want = oracle.compute_streams(n_streams, chunks, [(lo, hi), ((lo + hi) // 2, hi)])
        np.testing.assert_array_equal(per, want["per_device"])
    finally:
        hp.hpop_session_destroy(s)
