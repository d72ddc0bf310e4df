"""Pins for the CPU oracle: brute force, the paper's printed tables, closed
forms and invariants. All CPU-only."""
import itertools

import numpy as np
import pytest

import oracle
import tracegen as tg
from brute import occupancy_times, tree_from_times
import pils


def _check_against_brute(trace):
    got = oracle.compute(trace)
    want_times = occupancy_times(trace)
    np.testing.assert_array_equal(got["times"], want_times)
    sums, ratios, mask = tree_from_times(want_times, trace.n_hosts, trace.n_devices, trace.regions)
    np.testing.assert_array_equal(got["sums"], sums)
    np.testing.assert_array_equal(got["ratios"], ratios)  # same exact operands, one division
    np.testing.assert_array_equal(got["mask"], mask)


@pytest.mark.parametrize("seed", range(200))
def test_random_tiny_vs_brute_force(seed):
    rng = np.random.default_rng(seed)
    tr = tg.random_tiny(rng, max_span=int(rng.integers(2, 80)), max_events=int(rng.integers(1, 15)),
                        t0=int(rng.integers(0, 1 << 40)))
    _check_against_brute(tr)


def test_random_many_streams_vs_brute_force():
    rng = np.random.default_rng(7)
    for _ in range(20):
        tr = tg.random_tiny(rng, max_span=4096, max_events=200, n_hosts=2, n_devices=2, n_regions=5)
        _check_against_brute(tr)


def _all_intervals(span):
    return [(s, e) for s in range(span + 1) for e in range(s, span + 1)]


@pytest.mark.parametrize("is_host", [False, True])
def test_exhaustive_three_interval_layouts(is_host):
    """Every multiset of 3 records (interval in [0,6), any kind) on one resource."""
    span = 6
    kinds = (tg.HOST_USEFUL, tg.HOST_OFFLOAD, tg.HOST_MPI) if is_host else (tg.DEV_KERNEL, tg.DEV_MEMOP)
    items = [(k, s, e) for k in kinds for (s, e) in _all_intervals(span)]
    combos = list(itertools.combinations_with_replacement(range(len(items)), 3))
    if is_host:
        combos = combos[::3]  # a third of the host multisets keeps the test short
    R = len(combos)
    res = np.repeat(np.arange(R, dtype=np.int32), 3)
    sel = np.array(combos).reshape(-1)
    arr = np.array(items, np.int64)[sel]
    kind, s, e = arr[:, 0].astype(np.int32), arr[:, 1], arr[:, 2]
    regions = [(0, 6), (1, 5), (2, 3), (-1, 7), (3, 6), (5, 9)]
    n, m = (R, 0) if is_host else (0, R)
    got = oracle.compute_arrays(n, m, res, kind, s, e, regions)
    # vectorised brute force: occupancy per resource and kind on [-1, 9)
    lo, hi = -1, 9
    occ = np.zeros((R, 5, hi - lo), bool)
    for i in range(s.size):
        occ[res[i], kind[i], s[i] - lo:e[i] - lo] = True
    for g, (t0, t1) in enumerate(regions):
        w = slice(t0 - lo, t1 - lo)
        E = t1 - t0
        if is_host:
            u = occ[:, 0, w]
            wo = occ[:, 1, w] & ~u
            mp = occ[:, 2, w] & ~u & ~wo
            want = np.stack([u.sum(1), wo.sum(1), mp.sum(1), E - u.sum(1) - wo.sum(1) - mp.sum(1)], 1)
        else:
            k = occ[:, 3, w]
            mm = occ[:, 4, w] & ~k
            want = np.stack([k.sum(1), mm.sum(1), E - k.sum(1) - mm.sum(1), np.zeros(R, np.int64)], 1)
        np.testing.assert_array_equal(got["times"][g], want)


# ---------------------------------------------------------------- paper tables

@pytest.mark.parametrize("case", pils.load(), ids=lambda c: c[0])
def test_pils_printed_tables(case):
    name, printed, t = case
    for variant in ({}, {"kernel_streams": 4}, {"hidden_memops": 5}, {"kernel_streams": 8, "hidden_memops": 3},
                    {"t0": tg.T0}):
        r = oracle.compute(pils.build_trace(t, **variant))
        got = r["ratios"][0]
        assert np.all(np.abs(got - np.array(printed)) <= 0.005 + 1e-12), (name, variant, got, printed)


def test_pils_variants_leave_integers_unchanged():
    for name, printed, t in pils.load():
        base = oracle.compute(pils.build_trace(t))
        for variant in ({"kernel_streams": 3}, {"hidden_memops": 7}, {"t0": 12345}):
            r = oracle.compute(pils.build_trace(t, **variant))
            np.testing.assert_array_equal(r["times"], base["times"])
            np.testing.assert_array_equal(r["ratios"], base["ratios"])


# ---------------------------------------------------------------- closed forms

def _uniform_trace(n, m, busy_host, busy_dev, E, streams=1, t0=0):
    chunks = []
    for r in range(n):
        u, w = busy_host[r]
        chunks.append(tg.Chunk(r, tg.HOST_USEFUL, np.array([t0]), np.array([t0 + u])))
        if w:
            chunks.append(tg.Chunk(r, tg.HOST_OFFLOAD, np.array([t0 + u]), np.array([t0 + u + w])))
        chunks.append(tg.Chunk(r, tg.HOST_MPI, np.array([t0 + u + w]), np.array([t0 + E])))
    for g in range(m):
        k, mem = busy_dev[g]
        s = np.full(streams, t0, np.int64)
        chunks.append(tg.Chunk(n + g, tg.DEV_KERNEL, s, s + k))
        if mem:
            chunks.append(tg.Chunk(n + g, tg.DEV_MEMOP, np.array([t0 + k]), np.array([t0 + k + mem])))
    return tg.Trace(n, m, chunks, [(t0, t0 + E)])


def test_balanced_gives_load_balance_one():
    tr = _uniform_trace(8, 8, [(300, 200)] * 8, [(700, 100)] * 8, 1000)
    q = oracle.compute(tr)["ratios"][0]
    assert q[2] == 1.0 and q[6] == 1.0
    assert q[3] == 0.5 and q[1] == 0.5  # max(U+W)/E and sum/(nE)


@pytest.mark.parametrize("f_num", [0, 1, 3, 5, 9])
def test_injected_idle_fraction(f_num):
    """idle fraction f = f_num/10 with (1-f)E integral: PE = OE = 1 - f exactly."""
    E = 1_000_000
    busy = E - (f_num * E) // 10
    tr = _uniform_trace(4, 4, [(busy, 0)] * 4, [(busy, 0)] * 4, E)
    q = oracle.compute(tr)["ratios"][0]
    want = busy / E
    assert q[0] == want and q[8] == want and q[5] == want and q[1] == want
    assert q[4] == 1.0 and q[6] == 1.0 and q[7] == 1.0


def test_hidden_memops_give_comm_efficiency_one():
    tr = pils.build_trace([1, 1, 0, 1, 1, 0, 6000, 0, 3000, 0], hidden_memops=50)
    q = oracle.compute(tr)["ratios"][0]
    assert q[7] == 1.0


def test_identical_kernels_on_many_streams_count_once():
    one = oracle.compute(_uniform_trace(1, 1, [(10, 0)], [(400, 0)], 1000, streams=1))
    many = oracle.compute(_uniform_trace(1, 1, [(10, 0)], [(400, 0)], 1000, streams=8))
    np.testing.assert_array_equal(one["times"], many["times"])
    assert many["times"][0, 1, 0] == 400


# ---------------------------------------------------------------- invariants

def test_invariants_on_generated_trace():
    tr = tg.make_trace(11, 3, 3, 4, 2000, 1000, w_range=(0.5, 1.5), regions="tiles", n_regions=9)
    base = oracle.compute(tr)
    lo, hi = tr.span()
    # permutation of records and splitting into many chunks
    rng = np.random.default_rng(0)
    chunks = []
    for c in tr.chunks:
        p = rng.permutation(c.start.size)
        for part in np.array_split(p, 5):
            chunks.append(tg.Chunk(c.resource, c.kind, c.start[part], c.end[part]))
    rng.shuffle(chunks)
    perm = oracle.compute(tg.Trace(tr.n_hosts, tr.n_devices, chunks, tr.regions))
    for k in ("times", "sums", "ratios", "mask"):
        np.testing.assert_array_equal(perm[k], base[k])
    # translation
    sh = 987_654_321
    moved = tg.Trace(tr.n_hosts, tr.n_devices,
                     [tg.Chunk(c.resource, c.kind, c.start + sh, c.end + sh) for c in tr.chunks],
                     [(a + sh, b + sh) for a, b in tr.regions])
    np.testing.assert_array_equal(oracle.compute(moved)["times"], base["times"])
    # additivity: regions 1..8 tile region 0, state times add exactly
    np.testing.assert_array_equal(base["times"][1:].sum(0), base["times"][0])
    # telescoping: PE_host = MPI_PE * OE, MPI_PE = LB * CE, PE_dev = LB * CE * OE
    q = base["ratios"]
    for row in q:
        assert abs(row[0] - row[1] * row[4]) <= 1e-15 * max(row[0], 1e-300) * 4
        assert abs(row[1] - row[2] * row[3]) <= 1e-15 * max(row[1], 1e-300) * 4
        assert abs(row[5] - row[6] * row[7] * row[8]) <= 1e-15 * max(row[5], 1e-300) * 6


def test_nested_regions_monotone():
    tr = tg.make_trace(5, 2, 2, 3, 3000, 800, regions="nested", n_regions=12)
    t = oracle.compute(tr)["times"]
    busy = t[:, :, :3].copy()
    busy[:, 2:, 2] = 0  # device idle is not a covered state
    assert np.all(np.diff(busy, axis=0) <= 0)


def test_zero_denominators_are_one_and_flagged():
    # no host ranks, a device with nothing at all
    tr = tg.Trace(0, 1, [], [(0, 100)])
    r = oracle.compute(tr)
    q, mk = r["ratios"][0], int(r["mask"][0])
    assert q[0] == 1.0 and q[1] == 1.0 and q[4] == 1.0  # 0/(0*E) host terms
    assert mk & 1 and mk & 2 and mk & 4 and mk & 16
    assert q[5] == 0.0 and q[6] == 1.0 and (mk >> 6) & 1 and q[7] == 1.0 and (mk >> 7) & 1
    assert q[8] == 0.0


def test_bad_interval_rejected():
    tr = tg.Trace(0, 1, [tg.Chunk(0, tg.DEV_KERNEL, np.array([5]), np.array([4]))], [(0, 10)])
    with pytest.raises(oracle.OracleError) as ei:
        oracle.compute(tr)
    assert ei.value.code == -4


def test_kind_resource_mismatch_rejected():
    tr = tg.Trace(1, 1, [tg.Chunk(0, tg.DEV_KERNEL, np.array([1]), np.array([4]))], [(0, 10)])
    with pytest.raises(oracle.OracleError):
        oracle.compute(tr)


def test_threads_give_identical_results():
    tr = tg.make_trace(3, 5, 5, 4, 3000, 1000, regions="tiles", n_regions=5)
    a = oracle.compute(tr, threads=1)
    b = oracle.compute(tr, threads=4)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
