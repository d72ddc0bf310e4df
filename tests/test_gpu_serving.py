"""Serving runtime on the GPU: every query's trees equal the oracle on the
records its session had received up to and including that query, whether the
query ran alone or batched with queries of other sessions."""
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


def make_queries(seed, n_sessions, ranks, n_queries, mean_events=3000, p_early=0.3):
    """Per session: a list of (chunks, t0, t1) continuing its own timeline."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_sessions):
        origin = tg.T0 + s * 10 ** 12
        frontier = origin
        prev_close = origin
        qs = []
        for q in range(n_queries):
            n_ev = int(rng.integers(mean_events // 4, mean_events * 2))
            chunks = tg.continue_trace(rng, ranks, ranks, 3, n_ev, frontier, p_early=p_early, early_back=300_000)
            hi = max(int(c.end.max()) for c in chunks)
            frontier = max(frontier, hi)
            qs.append((chunks, prev_close, frontier))
            prev_close = frontier
        out.append((origin, qs))
    return out


def expected(ranks, origin, qs, upto):
    chunks = [c for q in qs[:upto + 1] for c in q[0]]
    t0, t1 = qs[upto][1], qs[upto][2]
    frontier = max(int(c.end.max()) for c in chunks)
    tr = tg.Trace(ranks, ranks, chunks, [(t0, t1), (origin, frontier)])
    return oracle.compute(tr)


def as_payload(chunks, device):
    out = []
    for c in chunks:
        if device:
            import torch
            out.append((c.resource, c.kind, torch.from_numpy(c.start).cuda(), torch.from_numpy(c.end).cuda()))
        else:
            out.append((c.resource, c.kind, c.start, c.end))
    return out


def check_tree(tree, want, g, what):
    np.testing.assert_array_equal(hp.tree_sums(tree), want["sums"][g], err_msg=what)
    np.testing.assert_array_equal(hp.tree_ratios(tree).view(np.int64), want["ratios"][g].view(np.int64), err_msg=what)


@pytest.mark.parametrize("device", [False, True])
def test_mixed_equals_alone_equals_oracle(device):
    import torch
    ranks, n_sessions, n_queries = 3, 4, 6
    plan = make_queries(11 + device, n_sessions, ranks, n_queries)
    # in the mix: all queries submitted up front, interleaved across sessions
    srv = hp.hpop_server_create(max_sessions=8, max_inflight=8)
    keep = []
    try:
        sids = [hp.hpop_server_open_session(srv, ranks, ranks, origin) for origin, _ in plan]
        torch.cuda.synchronize()
        payloads = {(s, q): as_payload(plan[s][1][q][0], device) for q in range(n_queries)
                    for s in range(n_sessions)}
        keep.append(payloads)
        torch.cuda.synchronize()
        tickets = {}
        for q in range(n_queries):
            for s in range(n_sessions):
                chunks, t0, t1 = plan[s][1][q]
                tickets[(s, q)] = hp.hpop_server_submit(srv, sids[s], payloads[(s, q)],
                                                        hp.HPOP_MEM_DEVICE if device else hp.HPOP_MEM_HOST, t0, t1)
        mixed = {k: hp.hpop_server_wait(srv, t) for k, t in tickets.items()}
        stats = hp.hpop_server_get_stats(srv)
        assert stats.completed == n_sessions * n_queries
        assert stats.mean_batch > 1.0  # queries of different sessions shared device steps
    finally:
        hp.hpop_server_destroy(srv)
    for (s, q), (reg, glob) in mixed.items():
        origin, qs = plan[s]
        want = expected(ranks, origin, qs, q)
        check_tree(reg, want, 0, "session %d query %d region" % (s, q))
        check_tree(glob, want, 1, "session %d query %d global" % (s, q))
    # alone: one session at a time, each query waited for before the next
    srv = hp.hpop_server_create(max_sessions=8, max_inflight=1)
    try:
        for s in range(n_sessions):
            sid = hp.hpop_server_open_session(srv, ranks, ranks, plan[s][0])
            for q in range(n_queries):
                chunks, t0, t1 = plan[s][1][q]
                payload = as_payload(chunks, device)
                if device:
                    torch.cuda.synchronize()
                t = hp.hpop_server_submit(srv, sid, payload, hp.HPOP_MEM_DEVICE if device else hp.HPOP_MEM_HOST,
                                          t0, t1)
                reg, glob = hp.hpop_server_wait(srv, t)
                m_reg, m_glob = mixed[(s, q)]
                np.testing.assert_array_equal(hp.tree_sums(reg), hp.tree_sums(m_reg))
                np.testing.assert_array_equal(hp.tree_ratios(glob).view(np.int64),
                                              hp.tree_ratios(m_glob).view(np.int64))
    finally:
        hp.hpop_server_destroy(srv)


def test_large_batches_take_the_global_sort_path():
    ranks = 2
    plan = make_queries(23, 1, ranks, 3, mean_events=40000, p_early=1.0)
    srv = hp.hpop_server_create(max_sessions=2, max_inflight=4)
    try:
        origin, qs = plan[0]
        sid = hp.hpop_server_open_session(srv, ranks, ranks, origin)
        for q, (chunks, t0, t1) in enumerate(qs):
            t = hp.hpop_server_submit(srv, sid, as_payload(chunks, False), hp.HPOP_MEM_HOST, t0, t1)
            reg, glob = hp.hpop_server_wait(srv, t)
            want = expected(ranks, origin, qs, q)
            check_tree(reg, want, 0, "query %d region" % q)
            check_tree(glob, want, 1, "query %d global" % q)
    finally:
        hp.hpop_server_destroy(srv)


def test_large_host_payloads_copied_in_parts():
    """Host payloads of several MB (copied into page-locked memory by more
    than one thread) give the oracle's trees, query after query."""
    ranks = 2
    plan = make_queries(29, 1, ranks, 3, mean_events=400000, p_early=0.5)
    srv = hp.hpop_server_create(max_sessions=1, max_inflight=4)
    try:
        origin, qs = plan[0]
        sid = hp.hpop_server_open_session(srv, ranks, ranks, origin)
        for q, (chunks, t0, t1) in enumerate(qs):
            n = sum(len(c.start) for c in chunks)
            print("case: query %d, %d records (%.1f MB)" % (q, n, n * 16 / 2 ** 20), flush=True)
            t = hp.hpop_server_submit(srv, sid, as_payload(chunks, False), hp.HPOP_MEM_HOST, t0, t1)
            reg, glob = hp.hpop_server_wait(srv, t)
            want = expected(ranks, origin, qs, q)
            check_tree(reg, want, 0, "query %d region" % q)
            check_tree(glob, want, 1, "query %d global" % q)
    finally:
        hp.hpop_server_destroy(srv)


@pytest.mark.parametrize("device", [True, False])
def test_bad_record_rejected_and_state_unchanged(device):
    import torch
    ranks = 2
    plan = make_queries(31, 1, ranks, 2)
    srv = hp.hpop_server_create(max_sessions=2, max_inflight=4)
    try:
        origin, qs = plan[0]
        sid = hp.hpop_server_open_session(srv, ranks, ranks, origin)
        chunks, t0, t1 = qs[0]
        t = hp.hpop_server_submit(srv, sid, as_payload(chunks, False), hp.HPOP_MEM_HOST, t0, t1)
        hp.hpop_server_wait(srv, t)
        bad_s = np.array([origin + 5, origin + 9], np.int64)
        bad_e = np.array([origin + 6, origin + 1], np.int64)
        if device:
            bad_s, bad_e = torch.from_numpy(bad_s).cuda(), torch.from_numpy(bad_e).cuda()
            torch.cuda.synchronize()
        t = hp.hpop_server_submit(srv, sid, [(ranks, hp.HPOP_DEV_KERNEL, bad_s, bad_e)],
                                  hp.HPOP_MEM_DEVICE if device else hp.HPOP_MEM_HOST, t0, t1)
        with pytest.raises(hp.HpopError) as ei:
            hp.hpop_server_wait(srv, t)
        assert ei.value.status == hp.HPOP_E_BAD_INTERVAL
        chunks, t0, t1 = qs[1]
        t = hp.hpop_server_submit(srv, sid, as_payload(chunks, False), hp.HPOP_MEM_HOST, t0, t1)
        reg, glob = hp.hpop_server_wait(srv, t)
        want = expected(ranks, origin, qs, 1)
        check_tree(reg, want, 0, "after rejected query")
        check_tree(glob, want, 1, "after rejected query")
    finally:
        hp.hpop_server_destroy(srv)


def test_backpressure_busy():
    srv = hp.hpop_server_create(max_sessions=1, max_inflight=1, queue_capacity=1, mem_budget_bytes=1 << 20)
    try:
        sid = hp.hpop_server_open_session(srv, 1, 1, 0)
        s = np.arange(0, 200000, 10, dtype=np.int64)
        e = s + 5
        got_busy = False
        tickets = []
        for i in range(50):
            try:
                tickets.append(hp.hpop_server_submit(srv, sid, [(1, hp.HPOP_DEV_KERNEL, s + i * 10 ** 7,
                                                                 e + i * 10 ** 7)], hp.HPOP_MEM_HOST,
                                                     i * 10 ** 7, (i + 1) * 10 ** 7))
            except hp.HpopError as err:
                assert err.status == hp.HPOP_E_BUSY
                got_busy = True
        assert got_busy
        for t in tickets:
            hp.hpop_server_wait(srv, t)
    finally:
        hp.hpop_server_destroy(srv)


def test_host_staging_area_bounds_and_phase_statistics():
    """A 1 MiB page-locked staging area: a larger host payload is refused
    with HPOP_E_ARG; payloads that would overfill it while others are queued
    get HPOP_E_BUSY and fit again once those completed; the area is taken
    once, at creation; every query's trees still equal the oracle's; the step
    phases are measured."""
    ranks = 1
    srv = hp.hpop_server_create(max_sessions=1, max_inflight=1, queue_capacity=64, host_staging_mib=1)
    try:
        st0 = hp.hpop_server_get_stats(srv)
        assert st0.host_staging_bytes == 1 << 20 and st0.max_pinned_alloc_us > 0
        sid = hp.hpop_server_open_session(srv, ranks, ranks, 0)
        big = np.arange(0, 10 * 70000, 10, dtype=np.int64)  # 70000 records: 1.07 MiB with their ends
        with pytest.raises(hp.HpopError) as ei:
            hp.hpop_server_submit(srv, sid, [(1, hp.HPOP_DEV_KERNEL, big, big + 5)], hp.HPOP_MEM_HOST, 0, 10 ** 7)
        assert ei.value.status == hp.HPOP_E_ARG
        # a query of 60000 records (960 KB) holds nearly all of the area until
        # its step ends: a second one submitted right after it has to wait
        chunks_all, tickets, busy, q, step = [], [], 0, 0, 10 ** 6
        for rep in range(5):
            for n in (60000, 20000):
                s = np.arange(q * step, q * step + 10 * n, 10, dtype=np.int64)
                e = s + 7
                while True:
                    try:
                        t = hp.hpop_server_submit(srv, sid, [(1, hp.HPOP_DEV_KERNEL, s, e)], hp.HPOP_MEM_HOST,
                                                  q * step, (q + 1) * step)
                        break
                    except hp.HpopError as err:
                        assert err.status == hp.HPOP_E_BUSY
                        busy += 1
                        for tk, _ in tickets:  # the held area comes back once they completed
                            hp.hpop_server_wait(srv, tk)
                        tickets = []
                tickets.append((t, q))
                chunks_all.append(tg.Chunk(1, tg.DEV_KERNEL, s, e))
                q += 1
        for tk, _ in tickets:
            hp.hpop_server_wait(srv, tk)
        st = hp.hpop_server_get_stats(srv)
        assert st.host_staging_bytes == 1 << 20 and st.max_host_staging_used <= 1 << 20
        assert st.max_pinned_alloc_us == st0.max_pinned_alloc_us  # no second allocation
        assert st.completed == q
        for f in ("max_prep_us", "max_wait_us", "max_h2d_us", "max_build_us", "max_splice_us", "max_region_us"):
            assert getattr(st, f) > 0, f
            assert 0 < getattr(st, f.replace("max_", "mean_")) <= getattr(st, f), f
        # the longest enqueueing call: a site of the step, within the longest step
        assert 0 <= st.max_call_site < len(hp.HPOP_CALL_SITES) and 0 < st.max_call_us <= st.max_step_us
        hp.hpop_server_reset_stats(srv)
        st = hp.hpop_server_get_stats(srv)
        assert st.completed == 0 and st.device_steps == 0 and st.max_step_us == 0 and st.max_build_us == 0
        assert st.max_call_us == 0 and st.max_call_site == -1
        assert st.host_staging_bytes == 1 << 20
        # the session's lists hold every query's records: one more (empty) query reads them back
        frontier = max(int(c.end.max()) for c in chunks_all)
        tr = tg.Trace(ranks, ranks, chunks_all, [((q - 1) * step, q * step), (0, frontier)])
        t = hp.hpop_server_submit(srv, sid, [], hp.HPOP_MEM_HOST, (q - 1) * step, q * step)
        reg, glob = hp.hpop_server_wait(srv, t)
        want = oracle.compute(tr)
        check_tree(reg, want, 0, "last region")
        check_tree(glob, want, 1, "global")
    finally:
        hp.hpop_server_destroy(srv)
    assert busy >= 1


@pytest.mark.parametrize("heap", [0, 1 << 20, 64 << 20])
def test_replay_equals_oracle(heap):
    """The native load generator returns the same trees as submit/wait, with a
    latency per query and a wall time covering every completion; with the
    list heap grown on demand, taken too small at creation (lists then move
    into a new heap) and taken large enough for every list."""
    ranks, n_sessions, n_queries = 2, 3, 4
    plan = make_queries(41, n_sessions, ranks, n_queries)
    srv = hp.hpop_server_create(max_sessions=4, max_inflight=4, list_heap_bytes=heap)
    try:
        sids = [hp.hpop_server_open_session(srv, ranks, ranks, origin) for origin, _ in plan]
        queries, keys = [], []
        for q in range(n_queries):
            for s in range(n_sessions):
                chunks, t0, t1 = plan[s][1][q]
                queries.append((sids[s], as_payload(chunks, False), t0, t1, 200_000 * len(queries)))
                keys.append((s, q))
        reg, glob, lat, wall, busy = hp.hpop_server_replay(srv, queries, hp.HPOP_MEM_HOST)
    finally:
        hp.hpop_server_destroy(srv)
    assert busy == 0
    assert (lat > 0).all() and wall >= queries[-1][4] + lat[-1] - 1
    for (s, q), r, g in zip(keys, reg, glob):
        origin, qs = plan[s]
        want = expected(ranks, origin, qs, q)
        check_tree(r, want, 0, "replay session %d query %d region" % (s, q))
        check_tree(g, want, 1, "replay session %d query %d global" % (s, q))


def test_long_records_across_queries():
    """Records lasting 2^32-2^35 ns (ends far past their time bucket) in
    consecutive queries of one session: the serving splice must see their true
    ends, also when a later query's records fall under them."""
    rng = np.random.default_rng(57)
    ranks = 2
    origin = 1 << 40
    qs = []
    t = origin
    for q in range(4):
        chunks = []
        for r in range(2 * ranks):
            kinds = (tg.HOST_USEFUL, tg.HOST_OFFLOAD, tg.HOST_MPI) if r < ranks else (tg.DEV_KERNEL, tg.DEV_MEMOP)
            for kd in kinds:
                n = int(rng.integers(200, 2000))
                s = np.sort(t + rng.integers(-(1 << 30), 1 << 36, size=n)).astype(np.int64)
                s = np.maximum(s, origin)
                d = rng.integers(1, 50_000, size=n)
                far = rng.random(n) < 0.01
                d[far] = rng.integers(1 << 32, 1 << 35, size=int(far.sum()))
                chunks.append(tg.Chunk(r, kd, s, s + d))
        hi = max(int(c.end.max()) for c in chunks)
        qs.append((chunks, t, max(hi, t + 1)))
        t = max(hi, t + 1)
    srv = hp.hpop_server_create(max_sessions=2, max_inflight=4)
    try:
        sid = hp.hpop_server_open_session(srv, ranks, ranks, origin)
        for q, (chunks, t0, t1) in enumerate(qs):
            payload = as_payload(chunks, q % 2 == 1)  # kept alive until the query is done
            tk = hp.hpop_server_submit(srv, sid, payload, hp.HPOP_MEM_DEVICE if q % 2 else hp.HPOP_MEM_HOST, t0, t1)
            reg, glob = hp.hpop_server_wait(srv, tk)
            del payload
            want = expected(ranks, origin, qs, q)
            check_tree(reg, want, 0, "long records query %d region" % q)
            check_tree(glob, want, 1, "long records query %d global" % q)
    finally:
        hp.hpop_server_destroy(srv)
