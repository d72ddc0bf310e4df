"""Pins of the oracle's regions entered repeatedly (per-resource interval lists).

* a per-nanosecond count restricted to each resource's own intervals (brute
  force, independent of the oracle) gives the same state times;
* one interval [t0, t1) on every resource reproduces the single-region oracle
  (integers, ratios and 0/0 flags), so the ratio wiring is the pinned one;
* splitting intervals changes nothing (additivity), E is the largest host
  in-region time (eq. 1), and Other/Idle complete each resource's own time.
"""
import numpy as np
import pytest

import oracle
import tracegen as tg
from brute import HOST_MPI, HOST_OFFLOAD, HOST_USEFUL, DEV_KERNEL, DEV_MEMOP


def random_lists(rng, trace, lo, hi, max_pieces=4):
    """Disjoint random intervals per resource inside [lo, hi)."""
    out = []
    for r in range(trace.n_hosts + trace.n_devices):
        k = int(rng.integers(0, max_pieces + 1))
        cuts = np.sort(rng.choice(np.arange(lo, hi + 1), size=2 * k, replace=False)) if k else []
        for i in range(k):
            a, b = int(cuts[2 * i]), int(cuts[2 * i + 1])
            if a < b:
                out.append((r, a, b))
    return out


def brute_multi(trace, ivls):
    n, m = trace.n_hosts, trace.n_devices
    R = n + m
    pts = [a for _, a, _ in ivls] + [b for _, _, b in ivls]
    for c in trace.chunks:
        if c.start.size:
            pts += [int(c.start.min()), int(c.end.max())]
    lo, hi = min(pts), max(pts)
    occ = np.zeros((R, 5, hi - lo), bool)
    for c in trace.chunks:
        for s, e in zip(c.start.tolist(), c.end.tolist()):
            occ[c.resource, c.kind, s - lo:e - lo] = True
    inside = np.zeros((R, hi - lo), bool)
    for r, a, b in ivls:
        inside[r, a - lo:b - lo] = True
    out = np.zeros((R, 4), np.int64)
    for r in range(R):
        w = inside[r]
        E_r = int(w.sum())
        if r < n:
            u = occ[r, HOST_USEFUL] & w
            wo = occ[r, HOST_OFFLOAD] & w & ~u
            mp = occ[r, HOST_MPI] & w & ~u & ~wo
            out[r] = [u.sum(), wo.sum(), mp.sum(), E_r - u.sum() - wo.sum() - mp.sum()]
        else:
            k = occ[r, DEV_KERNEL] & w
            mm = occ[r, DEV_MEMOP] & w & ~k
            out[r] = [k.sum(), mm.sum(), E_r - k.sum() - mm.sum(), 0]
    return out


@pytest.mark.parametrize("seed", range(60))
def test_brute_force_times(seed):
    rng = np.random.default_rng(4000 + seed)
    tr = tg.random_tiny(rng, max_span=int(rng.integers(8, 300)), max_events=int(rng.integers(1, 40)))
    pts = [int(x) for c in tr.chunks for x in (c.start.min(), c.end.max())] if tr.chunks else [0, 10]
    lo, hi = min(pts) - 5, max(pts) + 5
    ivls = random_lists(rng, tr, lo, hi)
    got = oracle.compute_multi(tr, [ivls])
    np.testing.assert_array_equal(got["times"][0], brute_multi(tr, ivls))
    n = tr.n_hosts
    E_r = np.zeros(tr.n_hosts + tr.n_devices, np.int64)
    for r, a, b in ivls:
        E_r[r] += b - a
    want_E = E_r[:n].max() if n and E_r[:n].max() > 0 else (E_r[n:].max() if tr.n_devices else 0)
    assert got["E"][0] == want_E


@pytest.mark.parametrize("seed", range(20))
def test_one_interval_everywhere_is_the_single_region(seed):
    rng = np.random.default_rng(5000 + seed)
    tr = tg.random_tiny(rng, max_span=int(rng.integers(8, 2000)), max_events=int(rng.integers(1, 100)), n_regions=3)
    R = tr.n_hosts + tr.n_devices
    want = oracle.compute(tr)
    got = oracle.compute_multi(tr, [[(r, a, b) for r in range(R)] for a, b in tr.regions])
    np.testing.assert_array_equal(got["times"], want["times"])
    np.testing.assert_array_equal(got["sums"], want["sums"])
    np.testing.assert_array_equal(got["ratios"].view(np.int64), want["ratios"].view(np.int64))
    np.testing.assert_array_equal(got["mask"], want["mask"])


def test_split_intervals_change_nothing():
    rng = np.random.default_rng(77)
    tr = tg.random_tiny(rng, max_span=500, max_events=80)
    ivls = random_lists(rng, tr, 0, 600, max_pieces=3)
    split = []
    for r, a, b in ivls:
        if b - a >= 2:
            c = int(rng.integers(a + 1, b))
            split += [(r, a, c), (r, c, b)]
        else:
            split.append((r, a, b))
    x, y = oracle.compute_multi(tr, [ivls, split])["times"]
    np.testing.assert_array_equal(x, y)
