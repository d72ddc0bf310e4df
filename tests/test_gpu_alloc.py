"""Caller-supplied device allocators (hpop_session_config.alloc / free).

The allocator here is hipMalloc / hipFree behind a byte budget: once the
budget is spent it returns NULL. A call that needed more memory then fails
with HPOP_E_OOM and leaves the session as it was (same records, same
results); with the budget raised the same call succeeds and the results
equal the oracle. At destroy every block the session took is given back.
"""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2603_26576_amd as hp
import tracegen as tg
from engine_util import assert_same, engine_results, gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")
    hp.lib()


class BudgetAllocator:
    def __init__(self, limit):
        import torch  # noqa: F401  (loads the HIP runtime the engine shares)
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.hip.hipFree.argtypes = [ctypes.c_void_p]
        self.hip.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        self.limit = limit
        self.live = {}
        self.refused = 0
        self.alloc_fn = hp.ALLOC_FN(self._alloc)
        self.free_fn = hp.FREE_FN(self._free)

    @property
    def used(self):
        return sum(self.live.values())

    def _alloc(self, ctx, nbytes, stream):
        if self.used + nbytes > self.limit:
            self.refused += 1
            return None
        p = ctypes.c_void_p()
        if self.hip.hipMalloc(ctypes.byref(p), nbytes) != 0 or not p.value:
            self.refused += 1
            return None
        self.live[p.value] = nbytes
        return p.value

    def _free(self, ctx, ptr, stream):
        if ptr:
            assert ptr in self.live, "free of a block the allocator never gave"
            del self.live[ptr]
            # the block may still be read by work queued on the session stream
            assert self.hip.hipStreamSynchronize(ctypes.c_void_p(stream)) == 0
            assert self.hip.hipFree(ctypes.c_void_p(ptr)) == 0


def split(trace):
    """The trace's chunks cut in two halves of each chunk (first half, second half)."""
    a, b = [], []
    for c in trace.chunks:
        h = len(c.start) // 2
        a.append((c.resource, c.kind, c.start[:h].copy(), c.end[:h].copy()))
        b.append((c.resource, c.kind, c.start[h:].copy(), c.end[h:].copy()))
    return a, b


def partial_trace(trace, chunks):
    return tg.Trace(trace.n_hosts, trace.n_devices,
                    [tg.Chunk(r, k, s, e) for r, k, s, e in chunks], list(trace.regions))


def test_refused_growth_leaves_the_session_unchanged():
    trace = tg.make_trace(21, 4, 4, 2, 20000, 5000, regions="tiles", n_regions=4)
    first, second = split(trace)
    A = BudgetAllocator(1 << 40)
    s = hp.hpop_session_create(trace.n_hosts, trace.n_devices, alloc=A.alloc_fn, free=A.free_fn)
    try:
        hp.add_chunks(s, first)
        for t0, t1 in trace.regions:
            hp.hpop_region_define(s, t0, t1)
        got = engine_results(s, trace)
        assert_same(got, oracle.compute(partial_trace(trace, first)), "first half")
        n0 = hp.hpop_session_get_info(s).n_events
        # no more memory: the second half needs a larger record arena
        A.limit = A.used
        with pytest.raises(hp.HpopError) as ei:
            hp.add_chunks(s, second)
        assert ei.value.status == hp.HPOP_E_OOM and A.refused >= 1
        assert hp.hpop_session_get_info(s).n_events == n0
        assert_same(engine_results(s, trace), got, "after the refused call")
        # memory again: the same call goes through and the results are the whole trace's
        A.limit = 1 << 40
        hp.add_chunks(s, second)
        assert hp.hpop_session_get_info(s).n_events == trace.n_events
        assert_same(engine_results(s, trace), oracle.compute(trace), "whole trace")
    finally:
        hp.hpop_session_destroy(s)
    assert A.live == {}, "blocks left after destroy"


def test_refused_workspace_then_compute_succeeds():
    trace = tg.make_trace(22, 3, 5, 4, 30000, 8000, regions="tiles", n_regions=3)
    A = BudgetAllocator(1 << 40)
    s = hp.hpop_session_create(trace.n_hosts, trace.n_devices, alloc=A.alloc_fn, free=A.free_fn)
    try:
        hp.add_chunks(s, [(c.resource, c.kind, c.start, c.end) for c in trace.chunks])
        for t0, t1 in trace.regions:
            hp.hpop_region_define(s, t0, t1)
        # the records fit; the build's workspace does not
        A.limit = A.used
        for _ in range(2):
            with pytest.raises(hp.HpopError) as ei:
                hp.hpop_metrics_compute_all(s)
            assert ei.value.status == hp.HPOP_E_OOM
        assert hp.hpop_session_get_info(s).n_events == trace.n_events
        A.limit = 1 << 40
        assert_same(engine_results(s, trace), oracle.compute(trace), "after the refused build")
    finally:
        hp.hpop_session_destroy(s)
    assert A.live == {}, "blocks left after destroy"


def test_allocator_pair_must_be_complete():
    A = BudgetAllocator(1 << 30)
    cfg = hp.hpop_session_config(1, 1, 0, ctypes.cast(A.alloc_fn, ctypes.c_void_p), None, None)
    h = ctypes.c_void_p()
    assert hp.lib().hpop_session_create(ctypes.byref(cfg), ctypes.byref(h)) == hp.HPOP_E_ARG
    assert not h.value
    np.testing.assert_equal(A.live, {})
