"""The hpop_collect tool on a real HIP application (tests/apps/collect_app).

The application runs as a child process with the tool loaded through
ROCP_TOOL_LIBRARIES; this process never loads the tool itself. Checks:
the records match what the program did (kernel and copy counts, kernel
durations against HIP events, host busy time inside Useful, no uncovered
host time), the engine's trees over the collected trace equal the oracle's,
and, in live mode, every tree the in-process hpop server returned equals the
oracle's over the records submitted up to that region."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import paper_2603_26576_amd as hp
import tracegen as tg
from engine_util import assert_same, gpu_available, run_engine
from paper_2603_26576_amd import collect

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
APP = os.path.join(ROOT, "tests", "apps", "collect_app")
ITERS = 30


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")
    if not os.path.exists(APP):
        pytest.fail("tests/apps/collect_app is not built (run __graft_entry__.build())")


def run_app(tmp_path, live_every):
    prefix = str(tmp_path / ("app_live%d" % live_every))
    print("case: collect_app iters=%d live_every=%d" % (ITERS, live_every), flush=True)
    r = subprocess.run([APP, str(ITERS), str(live_every), prefix], env=collect.tool_env(), capture_output=True,
                       text=True, timeout=120)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("collect_app ")][-1]
    info = dict(kv.split("=") for kv in line.split()[1:])
    return prefix, {k: float(v) for k, v in info.items()}


def as_trace(tr, regions):
    chunks = [tg.Chunk(r, k, s, e) for r, k, s, e in tr["chunks"] if s.size]
    return tg.Trace(tr["n_hosts"], tr["n_devices"], chunks, regions)


def by_pair(tr):
    return {(r, k): (s, e) for r, k, s, e in tr["chunks"]}


def test_offline_trace_matches_the_program(tmp_path):
    prefix, info = run_app(tmp_path, 0)
    assert info["dropped"] == 0
    tr = collect.read_trace(prefix + ".trace")
    tb, te = tr["t_begin"], tr["t_end"]
    assert tr["n_hosts"] == 1 and tr["n_devices"] >= 1 and tb < te
    P = by_pair(tr)
    for (r, k), (s, e) in P.items():
        assert np.all(s <= e), (r, k)
        assert np.all(s >= tb) and np.all(e <= te), (r, k)
        assert (r == 0) == (k <= hp.HPOP_HOST_MPI)
    # device 0 of the process is resource 1: the two spin kernels of every iteration
    ks, ke = P[(1, hp.HPOP_DEV_KERNEL)]
    assert ks.size == 2 * ITERS
    # each fill (a runtime blit kernel) and each of the two copies is a memory operation
    assert P[(1, hp.HPOP_DEV_MEMOP)][0].size >= 3 * ITERS
    # at least 12 runtime calls per iteration (2 copies, 4 events, 2 launches, 2 error checks, a fill, a sync)
    assert P[(0, hp.HPOP_HOST_OFFLOAD)][0].size >= 12 * ITERS
    # kernel durations agree with HIP events around each kernel
    ev_ms = np.fromfile(prefix + ".kern", np.float32).astype(np.float64)
    assert ev_ms.size == 2 * ITERS
    rec_ms = (ke - ks) / 1e6
    assert abs(rec_ms.sum() - ev_ms.sum()) <= 0.1 * ev_ms.sum() + 0.02 * ks.size
    assert np.all(rec_ms > 0.02)
    # the whole span is classified: the host's Useful and Offload records leave nothing uncovered
    want = oracle.compute(as_trace(tr, [(tb, te)]))
    U, W, MPI, other = want["times"][0][0]
    assert other == 0 and MPI == 0 and U + W == te - tb
    assert U >= 0.95 * info["busy_ns"]
    K, M = want["times"][0][1][0], want["times"][0][1][1]
    assert K > 0 and M > 0


def test_offline_trace_engine_equals_oracle(tmp_path):
    prefix, _ = run_app(tmp_path, 0)
    tr = collect.read_trace(prefix + ".trace")
    tb, te = tr["t_begin"], tr["t_end"]
    rng = np.random.default_rng(5)
    cuts = np.sort(rng.integers(tb + 1, te, size=8))
    regions = [(tb, te)] + [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if a < b]
    trace = as_trace(tr, regions)
    assert_same(run_engine(trace), oracle.compute(trace), "collected trace")
    assert_same(run_engine(trace, device=True), oracle.compute(trace), "collected trace, device records")


def test_live_feed_equals_oracle(tmp_path):
    live_every = 5
    prefix, info = run_app(tmp_path, live_every)
    tr = collect.read_trace(prefix + ".trace")
    n_dev, tb = tr["n_devices"], tr["t_begin"]
    n_pairs = (1 + n_dev) * 5
    tsz = ctypes.sizeof(hp.hpop_metric_tree)
    raw = open(prefix + ".live", "rb").read()
    rec = 16 + 8 * n_pairs + 2 * tsz
    assert len(raw) % rec == 0
    n_regions = len(raw) // rec
    assert n_regions == int(info["regions"]) and n_regions >= ITERS // live_every
    P = by_pair(tr)
    # the server's own kernels ran on the device while the tool recorded: they are in the trace too
    assert P[(1, hp.HPOP_DEV_KERNEL)][0].size > 2 * ITERS
    prev_t1 = tb
    for j in range(n_regions):
        b = raw[j * rec:(j + 1) * rec]
        t0, t1 = np.frombuffer(b, np.int64, 2, 0)
        taken = np.frombuffer(b, np.int64, n_pairs, 16)
        reg = hp.hpop_metric_tree.from_buffer_copy(b, 16 + 8 * n_pairs)
        glob = hp.hpop_metric_tree.from_buffer_copy(b, 16 + 8 * n_pairs + tsz)
        assert t0 == prev_t1 and t0 < t1
        prev_t1 = t1
        chunks = []
        for (r, k), (s, e) in P.items():
            n = int(taken[r * 5 + k])
            assert n <= s.size
            if n:
                chunks.append(tg.Chunk(r, k, s[:n], e[:n]))
        frontier = max(int(c.end.max()) for c in chunks)
        want = oracle.compute(tg.Trace(1, n_dev, chunks, [(int(t0), int(t1)), (tb, frontier)]))
        for g, tree in ((0, reg), (1, glob)):
            np.testing.assert_array_equal(hp.tree_sums(tree), want["sums"][g], err_msg="region %d tree %d" % (j, g))
            np.testing.assert_array_equal(hp.tree_ratios(tree).view(np.int64), want["ratios"][g].view(np.int64),
                                          err_msg="region %d tree %d" % (j, g))
            assert tree.undefined_mask == want["mask"][g]
