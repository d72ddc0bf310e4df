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


# ---------------------------------------------------------------------------
# Hand-worked fixtures: E and every tree value derived by hand from eq. 1
# (E = the largest in-region time of a host process), the state rules of
# Sec. 4.1 and eqs. 4-12, independently of the oracle's code.
# ---------------------------------------------------------------------------

def _trace(n, m, recs):
    chunks = [tg.Chunk(r, k, np.array([s], np.int64), np.array([e], np.int64)) for r, k, s, e in recs]
    return tg.Trace(n, m, chunks, [])


# Two hosts, one device. Host 0 is in the region over [0, 10) and [20, 30)
# (20 ns), host 1 over [5, 17) (12 ns), the device over [0, 40) (40 ns).
# E = max(20, 12) = 20: not the device's 40 (max over all resources), not the
# 40 ns span of all intervals, not the 30 ns span of the hosts' intervals.
# Host 0: Useful [0, 5) and [25, 30), Offloading [5, 10), MPI [20, 25)
#   -> U 10, W 5, MPI 5, Other 20 - 20 = 0.
# Host 1: Useful [5, 9), MPI [9, 12); outside records [0, 5) and [17, 19)
#   -> U 4, W 0, MPI 3, Other 12 - 7 = 5 (E - 7 = 13 would be wrong).
# Device: Kernel [0, 8) and [30, 35), Memory [4, 12), Kernel [38, 45)
#   -> K 8 + 5 + 2 = 15, M 4, Idle 40 - 19 = 21.
FIX1 = dict(
    n=2, m=1,
    recs=[(0, HOST_USEFUL, 0, 5), (0, HOST_OFFLOAD, 5, 10), (0, HOST_MPI, 20, 25), (0, HOST_USEFUL, 25, 30),
          (0, HOST_USEFUL, 10, 20),  # between host 0's intervals: outside the region
          (1, HOST_USEFUL, 5, 9), (1, HOST_MPI, 9, 12), (1, HOST_USEFUL, 0, 5), (1, HOST_OFFLOAD, 17, 19),
          (2, DEV_KERNEL, 0, 8), (2, DEV_KERNEL, 30, 35), (2, DEV_MEMOP, 4, 12), (2, DEV_KERNEL, 38, 45)],
    ivls=[(0, 0, 10), (0, 20, 30), (1, 5, 17), (2, 0, 40)],
    E=20,
    times=[[10, 5, 5, 0], [4, 0, 3, 5], [15, 4, 21, 0]],
    # sumU sumW sumMPI sumOther sumUW maxUW sumK sumM maxK maxKM
    sums=[14, 5, 8, 5, 19, 15, 15, 4, 15, 19],
    ratios=[(14, 40), (19, 40), (19, 30), (15, 20), (14, 19), (15, 20), (15, 15), (15, 19), (19, 20)],
    mask=0)

# Device-only session: device 0 in the region over [0, 10) and [50, 60)
# (20 ns), device 1 over [0, 15) (15 ns); no host process, so E is the
# largest device time, 20.
# Device 0: Kernel [2, 8) and [55, 70) -> K 6 + 5 = 11, M 0, Idle 9.
# Device 1: Memory [0, 30) -> K 0, M 15, Idle 0.
# Host ratios: n = 0 gives 0/0 for host PE, MPI PE, MPI LB and offload
# efficiency (bits 0, 1, 2, 4); MPI CE is max(U+W)/E = 0/20 = 0.
FIX2 = dict(
    n=0, m=2,
    recs=[(0, DEV_KERNEL, 2, 8), (0, DEV_KERNEL, 55, 70), (1, DEV_MEMOP, 0, 30)],
    ivls=[(0, 0, 10), (0, 50, 60), (1, 0, 15)],
    E=20,
    times=[[11, 0, 9, 0], [0, 15, 0, 0]],
    sums=[0, 0, 0, 0, 0, 0, 11, 15, 11, 15],
    ratios=[None, None, None, (0, 20), None, (11, 40), (11, 22), (11, 15), (15, 20)],
    mask=0b10111)

# A host without any interval stays out of E; the other host's time is split
# over three intervals. Host 0: [0, 4), [6, 9), [12, 20) -> 15 ns; host 1: no
# interval; device 2: [0, 3) -> 3 ns. E = 15.
# Host 0: Useful [0, 20) -> U 15, Other 0. Host 1: Useful [0, 20) but outside
# -> all 0. Device: Kernel [1, 2) -> K 1, Idle 2.
FIX3 = dict(
    n=2, m=1,
    recs=[(0, HOST_USEFUL, 0, 20), (1, HOST_USEFUL, 0, 20), (2, DEV_KERNEL, 1, 2)],
    ivls=[(0, 0, 4), (0, 6, 9), (0, 12, 20), (2, 0, 3)],
    E=15,
    times=[[15, 0, 0, 0], [0, 0, 0, 0], [1, 0, 2, 0]],
    sums=[15, 0, 0, 0, 15, 15, 1, 0, 1, 1],
    ratios=[(15, 30), (15, 30), (15, 30), (15, 15), (15, 15), (1, 15), (1, 1), (1, 1), (1, 15)],
    mask=0)

FIXTURES = {"hosts and device differ": FIX1, "device-only session": FIX2, "host without intervals": FIX3}


def _fixture_fails(fx, compute_multi):
    tr = _trace(fx["n"], fx["m"], fx["recs"])
    got = compute_multi(tr, [fx["ivls"]])
    if got["E"][0] != fx["E"]:
        return "E %d != %d" % (got["E"][0], fx["E"])
    if not np.array_equal(got["times"][0], np.array(fx["times"], np.int64)):
        return "times %s" % got["times"][0].tolist()
    if not np.array_equal(got["sums"][0], np.array(fx["sums"], np.int64)):
        return "sums %s" % got["sums"][0].tolist()
    want = [1.0 if q is None else q[0] / q[1] for q in fx["ratios"]]
    if not np.array_equal(got["ratios"][0], np.array(want)):
        return "ratios %s" % got["ratios"][0].tolist()
    if got["mask"][0] != fx["mask"]:
        return "mask %d" % got["mask"][0]
    return None


@pytest.mark.parametrize("name", sorted(FIXTURES))
def test_hand_worked_fixture(name):
    assert _fixture_fails(FIXTURES[name], oracle.compute_multi) is None


# Planted mistakes in compute_multi, each of which some pin above must reject.
MULTI_MUTANTS = [
    ("E over all resources",
     "E = int(Er[:n].max()) if n and Er[:n].max() > 0 else (int(Er[n:].max()) if m else 0)",
     "E = int(Er.max())"),
    ("E as the span of the intervals",
     "E = int(Er[:n].max()) if n and Er[:n].max() > 0 else (int(Er[n:].max()) if m else 0)",
     "E = (max(b for _, _, b in ivls) - min(a for _, a, _ in ivls)) if ivls else 0"),
    ("E over devices first",
     "E = int(Er[:n].max()) if n and Er[:n].max() > 0 else (int(Er[n:].max()) if m else 0)",
     "E = int(Er[n:].max()) if m and Er[n:].max() > 0 else (int(Er[:n].max()) if n else 0)"),
    ("E as the sum over hosts",
     "E = int(Er[:n].max()) if n and Er[:n].max() > 0 else (int(Er[n:].max()) if m else 0)",
     "E = int(Er[:n].sum()) if n and Er[:n].max() > 0 else (int(Er[n:].max()) if m else 0)"),
    ("Other from E instead of E_r", "Er[r] - D[2]]", "E - D[2]]"),
    ("Idle from E instead of E_r", "Er[r] - D[1], 0]", "E - D[1], 0]"),
]


def _multi_pins_fail(compute_multi):
    for fx in FIXTURES.values():
        if _fixture_fails(fx, compute_multi):
            return True
    for seed in range(20):
        rng = np.random.default_rng(4000 + seed)
        tr = tg.random_tiny(rng, max_span=int(rng.integers(8, 300)), max_events=int(rng.integers(1, 40)))
        pts = [int(x) for c in tr.chunks for x in (c.start.min(), c.end.max())] if tr.chunks else [0, 10]
        ivls = random_lists(rng, tr, min(pts) - 5, max(pts) + 5)
        if not np.array_equal(compute_multi(tr, [ivls])["times"][0], brute_multi(tr, ivls)):
            return True
    return False


def test_unmodified_compute_multi_passes_the_pins():
    assert not _multi_pins_fail(oracle.compute_multi)


@pytest.mark.parametrize("mutant", MULTI_MUTANTS, ids=lambda m: m[0])
def test_planted_mistake_in_compute_multi_is_caught(mutant, tmp_path):
    import importlib.util
    import inspect
    name, old, new = mutant
    src = inspect.getsource(oracle)
    assert src.count(old) == 1, "mutation anchor not found: " + name
    path = tmp_path / "oracle_mut.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("oracle_mut", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._lib = oracle._load()  # the C union measure is the pinned one
    assert _multi_pins_fail(mod.compute_multi), "planted mistake not caught: " + name
