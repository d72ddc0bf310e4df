"""Pins of the stream-concurrency oracle (oracle.compute_streams), CPU only.

The oracle reads streams as the stream-level row defines them (the paper
leaves streams to future work, Sec. 4.1): per device, stream time ST is the
integral of the number of active streams, busy time B the time with at least
one. These are checked against a per-nanosecond brute force of that number,
against closed forms, against the main oracle's K, and against invariances
that a dropped term, a wrong index or a swapped operand would break."""
import numpy as np
import pytest

import oracle
import tracegen as tg


def brute(n_streams, chunks, t0, t1):
    """Per device: histogram A[c] = ns of [t0, t1) with exactly c active streams."""
    out = []
    for g, S in enumerate(n_streams):
        active = np.zeros((S, t1 - t0), bool)
        for d, st, s, e in chunks:
            if d != g:
                continue
            for a, b in zip(s, e):
                lo, hi = max(int(a), t0), min(int(b), t1)
                if lo < hi:
                    active[st, lo - t0:hi - t0] = True
        out.append(np.bincount(active.sum(axis=0), minlength=S + 1))
    return out


def random_case(rng, m=3, max_streams=4, span=300, max_rec=12):
    n_streams = [int(rng.integers(1, max_streams + 1)) for _ in range(m)]
    chunks = []
    for g in range(m):
        for st in range(n_streams[g]):
            if rng.random() < 0.2:
                continue  # a declared stream with no records
            for _ in range(int(rng.integers(1, 3))):
                k = int(rng.integers(0, max_rec))
                s = rng.integers(0, span, size=k).astype(np.int64)
                e = s + rng.integers(0, 40, size=k)
                chunks.append((g, st, s, e))
    return n_streams, chunks


@pytest.mark.parametrize("seed", range(25))
def test_against_brute_force_histogram(seed):
    rng = np.random.default_rng(400 + seed)
    n_streams, chunks = random_case(rng)
    regions = [(0, 340), (17, 18), (50, 220), (300, 341)]
    got = oracle.compute_streams(n_streams, chunks, regions)
    for r, (t0, t1) in enumerate(regions):
        hist = brute(n_streams, chunks, t0, t1)
        for g, A in enumerate(hist):
            c = np.arange(A.size)
            B, ST, S = got["per_device"][r, g]
            assert ST == int((c * A).sum())
            assert B == int(A[1:].sum())
            assert S == n_streams[g]
        busy, stream_time, capacity = got["sums"][r]
        assert busy == sum(int(A[1:].sum()) for A in hist)
        assert capacity == sum(int(A[1:].sum()) * S for A, S in zip(hist, n_streams))
        if capacity:
            assert got["ratios"][r, 0] == stream_time / capacity
            assert got["ratios"][r, 1] == stream_time / busy
            assert 1.0 / max(n_streams) <= got["ratios"][r, 0] <= 1.0


def test_closed_forms():
    rng = np.random.default_rng(3)
    s = np.sort(rng.integers(0, 10_000, size=50)).astype(np.int64)
    e = s + rng.integers(1, 50, size=50)
    # one stream: every busy instant has exactly one of one stream active
    r = oracle.compute_streams([1], [(0, 0, s, e)], [(0, 10_100)])
    assert tuple(r["ratios"][0]) == (1.0, 1.0) and r["mask"][0] == 0
    # S identical streams: always all active together
    S = 4
    r = oracle.compute_streams([S], [(0, k, s, e) for k in range(S)], [(0, 10_100)])
    assert r["ratios"][0, 0] == 1.0 and r["ratios"][0, 1] == float(S)
    # S streams taking turns (disjoint kernels): one active at a time
    t = np.arange(0, 4000, 10, dtype=np.int64)
    chunks = [(0, k, t[k::S], t[k::S] + 10) for k in range(S)]
    r = oracle.compute_streams([S], chunks, [(0, 4000)])
    assert r["ratios"][0, 0] == 1.0 / S and r["ratios"][0, 1] == 1.0
    assert tuple(r["per_device"][0, 0]) == (4000, 4000, S)
    # a declared stream with no work halves the efficiency of a one-stream device
    r = oracle.compute_streams([2], [(0, 0, s, e)], [(0, 10_100)])
    assert r["ratios"][0, 0] == 0.5 and r["ratios"][0, 1] == 1.0


def test_undefined_ratios():
    r = oracle.compute_streams([2, 3], [], [(0, 100)])
    assert tuple(r["sums"][0]) == (0, 0, 0)
    assert tuple(r["ratios"][0]) == (1.0, 1.0) and r["mask"][0] == 0b11
    r = oracle.compute_streams([], [], [(0, 100)])
    assert r["mask"][0] == 0b11


def test_busy_time_equals_kernel_time_of_main_oracle():
    rng = np.random.default_rng(9)
    n_streams, chunks = random_case(rng, m=4, span=5000, max_rec=200)
    regions = [(0, 6000), (1000, 2500), (4999, 5001)]
    got = oracle.compute_streams(n_streams, chunks, regions)
    tr = tg.Trace(0, len(n_streams), [tg.Chunk(g, tg.DEV_KERNEL, s, e) for g, _, s, e in chunks], regions)
    want = oracle.compute(tr)
    np.testing.assert_array_equal(got["per_device"][:, :, 0], want["times"][:, :, 0])


def test_additive_over_adjacent_regions_and_invariant_to_record_layout():
    rng = np.random.default_rng(21)
    n_streams, chunks = random_case(rng, m=3, span=2000, max_rec=100)
    a = oracle.compute_streams(n_streams, chunks, [(0, 700), (700, 2100), (0, 2100)])
    np.testing.assert_array_equal(a["per_device"][0][:, :2] + a["per_device"][1][:, :2], a["per_device"][2][:, :2])
    # split every record in two touching halves, shuffle, regroup per stream
    pieces = {}
    for g, st, s, e in chunks:
        mid = (s + e) // 2
        pieces.setdefault((g, st), []).append((np.concatenate([s, mid]), np.concatenate([mid, e])))
    regrouped = []
    for (g, st), lst in pieces.items():
        s = np.concatenate([p[0] for p in lst])
        e = np.concatenate([p[1] for p in lst])
        perm = rng.permutation(s.size)
        regrouped.append((g, st, s[perm], e[perm]))
    b = oracle.compute_streams(n_streams, regrouped[::-1], [(0, 700), (700, 2100), (0, 2100)])
    np.testing.assert_array_equal(a["per_device"], b["per_device"])
    np.testing.assert_array_equal(a["ratios"].view(np.int64), b["ratios"].view(np.int64))
