"""Python binding of libhpop, the MI355X engine for the heterogeneous POP
efficiency metrics (host and device trees of arXiv 2603.26576).

Argument marshalling only: every step of the reduction runs in the HIP
kernels of ``libhpop.so`` behind the C ABI in ``include/hpop.h``. The
functions keep the C names; they raise :class:`HpopError` on a non-zero
status. Arrays may be numpy arrays (host) or torch tensors (device); PyTorch
is used only for device memory and streams.

If ``libhpop.so`` has not been built, importing the binding succeeds but the
first call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhpop.so")

HPOP_OK = 0
HPOP_E_ARG = -1
HPOP_E_KIND = -2
HPOP_E_RESOURCE = -3
HPOP_E_BAD_INTERVAL = -4
HPOP_E_REGION = -5
HPOP_E_OVERFLOW = -6
HPOP_E_OOM = -7
HPOP_E_BUSY = -8
HPOP_E_HIP = -9
HPOP_E_TIMEOUT = -10
HPOP_E_STATE = -11

HPOP_HOST_USEFUL = 0
HPOP_HOST_OFFLOAD = 1
HPOP_HOST_MPI = 2
HPOP_DEV_KERNEL = 3
HPOP_DEV_MEMOP = 4

HPOP_MEM_HOST = 0
HPOP_MEM_DEVICE = 1
HPOP_FORCE_REBUILD = 1
HPOP_NO_GRAPH = 2

RATIO_FIELDS = ["host_pe", "host_mpi_pe", "host_mpi_lb", "host_mpi_ce", "host_oe",
                "dev_pe", "dev_lb", "dev_ce", "dev_oe"]
SUM_FIELDS = ["sumU", "sumW", "sumMPI", "sumOther", "sumUW", "maxUW", "sumK", "sumM", "maxK", "maxKM"]


class hpop_metric_tree(ctypes.Structure):
    _fields_ = ([("E", ctypes.c_int64), ("n", ctypes.c_int32), ("m", ctypes.c_int32)]
                + [(f, ctypes.c_int64) for f in SUM_FIELDS]
                + [(f, ctypes.c_double) for f in RATIO_FIELDS]
                + [("undefined_mask", ctypes.c_uint32), ("reserved", ctypes.c_uint32)])


class hpop_session_config(ctypes.Structure):
    _fields_ = [("n_hosts", ctypes.c_int32), ("n_devices", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("alloc", ctypes.c_void_p), ("free", ctypes.c_void_p), ("alloc_ctx", ctypes.c_void_p)]


class hpop_event_chunk(ctypes.Structure):
    _fields_ = [("resource", ctypes.c_int32), ("kind", ctypes.c_int32), ("start", ctypes.c_void_p),
                ("end", ctypes.c_void_p), ("count", ctypes.c_int64)]


class hpop_tuning(ctypes.Structure):
    _fields_ = [("bucket_target", ctypes.c_int32), ("bucket_cap", ctypes.c_int32),
                ("tile_elems", ctypes.c_int32), ("scatter_slots", ctypes.c_int32)]


class hpop_session_info(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_int64), ("n_chunks", ctypes.c_int64), ("n_buckets", ctypes.c_int64),
                ("n_oversized", ctypes.c_int64), ("n_components", ctypes.c_int64), ("n_regions", ctypes.c_int32),
                ("graph_replays", ctypes.c_int32), ("n_wide_components", ctypes.c_int64),
                ("n_wide_records", ctypes.c_int64)]


class hpop_server_config(ctypes.Structure):
    _fields_ = [("max_sessions", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("host_staging_mib", ctypes.c_int32),
                ("mem_budget_bytes", ctypes.c_int64), ("list_heap_bytes", ctypes.c_int64)]


class hpop_server_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("events", ctypes.c_int64), ("device_steps", ctypes.c_int64),
                ("mean_batch", ctypes.c_double), ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("max_submit_us", ctypes.c_double), ("max_step_us", ctypes.c_double),
                ("host_staging_bytes", ctypes.c_int64), ("max_pinned_alloc_us", ctypes.c_double),
                ("max_host_staging_used", ctypes.c_int64),
                ("max_prep_us", ctypes.c_double), ("max_grow_us", ctypes.c_double), ("max_wait_us", ctypes.c_double),
                ("max_h2d_us", ctypes.c_double), ("max_build_us", ctypes.c_double), ("max_move_us", ctypes.c_double),
                ("max_splice_us", ctypes.c_double), ("max_region_us", ctypes.c_double),
                ("mean_prep_us", ctypes.c_double), ("mean_grow_us", ctypes.c_double), ("mean_wait_us", ctypes.c_double),
                ("mean_h2d_us", ctypes.c_double), ("mean_build_us", ctypes.c_double),
                ("mean_move_us", ctypes.c_double), ("mean_splice_us", ctypes.c_double),
                ("mean_region_us", ctypes.c_double), ("max_call_us", ctypes.c_double),
                ("max_call_site", ctypes.c_int32), ("reserved", ctypes.c_int32)]


HPOP_CALL_SITES = ("event", "payload", "move", "build", "tables", "control", "splice", "region", "results")


class hpop_replay_query(ctypes.Structure):
    _fields_ = [("sid", ctypes.c_int32), ("n_chunks", ctypes.c_int32),
                ("chunks", ctypes.POINTER(hpop_event_chunk)), ("t0", ctypes.c_int64), ("t1", ctypes.c_int64),
                ("arrival_ns", ctypes.c_int64)]


class HpopError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("hpop status %d: %s" % (status, message))
        self.status = status
        self.message = message


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64

# C signatures: name -> (restype, argtypes)
_SIGS = {
    "hpop_status_string": (ctypes.c_char_p, [_I32]),
    "hpop_last_error": (ctypes.c_char_p, [_P]),
    "hpop_session_create": (_I32, [ctypes.POINTER(hpop_session_config), ctypes.POINTER(_P)]),
    "hpop_session_destroy": (_I32, [_P]),
    "hpop_add_events": (_I32, [_P, _I32, _I32, _P, _P, _I64, _I32]),
    "hpop_add_events_multi": (_I32, [_P, ctypes.POINTER(hpop_event_chunk), _I32, _I32]),
    "hpop_clear_events": (_I32, [_P]),
    "hpop_session_synchronize": (_I32, [_P]),
    "hpop_region_define": (_I32, [_P, _I64, _I64, ctypes.POINTER(_I32)]),
    "hpop_region_define_multi": (_I32, [_P, _P, _P, _P, _I64, ctypes.POINTER(_I32)]),
    "hpop_num_regions": (_I32, [_P, ctypes.POINTER(_I32)]),
    "hpop_metrics_compute": (_I32, [_P, _I32, ctypes.POINTER(hpop_metric_tree)]),
    "hpop_metrics_compute_all": (_I32, [_P, _U32, ctypes.POINTER(hpop_metric_tree)]),
    "hpop_resource_times": (_I32, [_P, _I32, _I32, ctypes.POINTER(_I64)]),
    "hpop_batch_compute": (_I32, [ctypes.POINTER(_P), _I32, _U32, ctypes.POINTER(hpop_metric_tree)]),
    "hpop_session_get_info": (_I32, [_P, ctypes.POINTER(hpop_session_info)]),
    "hpop_session_set_tuning": (_I32, [_P, ctypes.POINTER(hpop_tuning)]),
    "hpop_session_get_tuning": (_I32, [_P, ctypes.POINTER(hpop_tuning)]),
    "hpop_session_enable_timing": (_I32, [_P, _I32]),
    "hpop_session_time_stage": (_I32, [_P, ctypes.c_char_p]),
    "hpop_session_stage_times": (_I32, [_P, _I32, ctypes.POINTER(ctypes.c_char_p),
                                        ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_I32)]),
    "hpop_autotune": (_I32, [ctypes.POINTER(_P), _I32, ctypes.c_char_p, ctypes.POINTER(hpop_tuning)]),
    "hpop_server_create": (_I32, [ctypes.POINTER(hpop_server_config), ctypes.POINTER(_P)]),
    "hpop_server_destroy": (_I32, [_P]),
    "hpop_server_open_session": (_I32, [_P, _I32, _I32, _I64, ctypes.POINTER(_I32)]),
    "hpop_server_submit": (_I32, [_P, _I32, ctypes.POINTER(hpop_event_chunk), _I32, _I32, _I64, _I64,
                                  ctypes.POINTER(_U64)]),
    "hpop_server_wait": (_I32, [_P, _U64, _I64, ctypes.POINTER(hpop_metric_tree),
                                ctypes.POINTER(hpop_metric_tree)]),
    "hpop_server_get_stats": (_I32, [_P, ctypes.POINTER(hpop_server_stats)]),
    "hpop_server_reset_stats": (_I32, [_P]),
    "hpop_server_last_error": (ctypes.c_char_p, [_P]),
    "hpop_tree_format": (_I32, [ctypes.POINTER(hpop_metric_tree), _I32, ctypes.c_char_p, _I64, ctypes.POINTER(_I64)]),
    "hpop_region_format": (_I32, [_P, _I32, _I32, ctypes.c_char_p, _I64, ctypes.POINTER(_I64)]),
    "hpop_metrics_compute_static": (_I32, [_I32, _I32, ctypes.POINTER(hpop_event_chunk), _I32,
                                           ctypes.POINTER(_I64), ctypes.POINTER(_I64), _I32, _P,
                                           ctypes.POINTER(hpop_metric_tree), ctypes.POINTER(_I64)]),
    "hpop_session_set_streams": (_I32, [_P, _P]),
    "hpop_add_stream_events": (_I32, [_P, _I32, _I32, _P, _P, _I64, _I32]),
    "hpop_stream_metrics": (_I32, [_P, _U32, ctypes.c_void_p, _P]),
    "hpop_server_replay": (_I32, [_P, ctypes.POINTER(hpop_replay_query), _I32, _I32,
                                  ctypes.POINTER(hpop_metric_tree), ctypes.POINTER(hpop_metric_tree),
                                  ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
}

_lib = None


def lib():
    """The loaded libhpop.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhpop.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status, handle=None):
    if status != HPOP_OK:
        msg = lib().hpop_last_error(handle)
        raise HpopError(status, (msg or b"").decode(errors="replace"))


def _ptr(x):
    """Address and memory space of a numpy array or torch tensor (int64, contiguous)."""
    if isinstance(x, np.ndarray):
        if x.dtype != np.int64 or not x.flags["C_CONTIGUOUS"]:
            raise ValueError("need a contiguous int64 array")
        return x.ctypes.data, HPOP_MEM_HOST
    import torch  # device memory comes from torch tensors
    if isinstance(x, torch.Tensor):
        if x.dtype != torch.int64 or not x.is_contiguous():
            raise ValueError("need a contiguous int64 tensor")
        return x.data_ptr(), (HPOP_MEM_DEVICE if x.is_cuda else HPOP_MEM_HOST)
    raise TypeError(type(x))


# ---------------------------------------------------------------------------
# the C calls, same names
# ---------------------------------------------------------------------------

def hpop_status_string(status):
    return lib().hpop_status_string(status).decode()


# hpop_alloc_fn / hpop_free_fn of include/hpop.h (the caller keeps the objects alive)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def hpop_session_create(n_hosts, n_devices, stream=None, alloc=None, free=None, alloc_ctx=None):
    """alloc / free: optional ALLOC_FN / FREE_FN objects for every device allocation."""
    cfg = hpop_session_config(n_hosts, n_devices, stream or 0,
                              ctypes.cast(alloc, ctypes.c_void_p) if alloc else None,
                              ctypes.cast(free, ctypes.c_void_p) if free else None, alloc_ctx)
    h = _P()
    _check(lib().hpop_session_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def hpop_session_destroy(s):
    _check(lib().hpop_session_destroy(s))


def hpop_add_events(s, resource, kind, start, end):
    ps, ms = _ptr(start)
    pe, me = _ptr(end)
    if ms != me or len(start) != len(end):
        raise ValueError("start and end must have the same length and memory space")
    _check(lib().hpop_add_events(s, resource, kind, ps, pe, len(start), ms), s)


def hpop_add_events_multi(s, chunks, mem_space):
    """chunks: iterable of (resource, kind, start, end)."""
    arr = (hpop_event_chunk * max(1, len(chunks)))()
    keep = []
    for i, (r, k, st, en) in enumerate(chunks):
        ps, _ = _ptr(st)
        pe, _ = _ptr(en)
        keep.append((st, en))
        arr[i] = hpop_event_chunk(r, k, ps, pe, len(st))
    _check(lib().hpop_add_events_multi(s, arr, len(chunks), mem_space), s)


def hpop_session_synchronize(s):
    _check(lib().hpop_session_synchronize(s), s)


def hpop_clear_events(s):
    _check(lib().hpop_clear_events(s), s)


def hpop_region_define(s, t0, t1):
    out = _I32()
    _check(lib().hpop_region_define(s, int(t0), int(t1), ctypes.byref(out)), s)
    return out.value


def hpop_region_define_multi(s, intervals):
    """A region entered repeatedly: intervals = [(resource, t0, t1), ...]."""
    r = np.ascontiguousarray([int(x[0]) for x in intervals], np.int32)
    a = np.ascontiguousarray([int(x[1]) for x in intervals], np.int64)
    b = np.ascontiguousarray([int(x[2]) for x in intervals], np.int64)
    out = _I32()
    _check(lib().hpop_region_define_multi(s, r.ctypes.data, a.ctypes.data, b.ctypes.data, len(intervals),
                                          ctypes.byref(out)), s)
    return out.value


class hpop_stream_tree(ctypes.Structure):
    _fields_ = [("busy", ctypes.c_int64), ("stream_time", ctypes.c_int64), ("capacity", ctypes.c_int64),
                ("m", ctypes.c_int32), ("n_streams", ctypes.c_int32), ("stream_eff", ctypes.c_double),
                ("mean_active", ctypes.c_double), ("undefined_mask", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


def hpop_session_set_streams(s, n_streams):
    """Declare the streams of every device: n_streams[g] for device g."""
    arr = np.ascontiguousarray(n_streams, np.int32)
    _check(lib().hpop_session_set_streams(s, arr.ctypes.data if arr.size else None), s)


def hpop_add_stream_events(s, resource, stream, start, end):
    ps, ms = _ptr(start)
    pe, me = _ptr(end)
    if ms != me or len(start) != len(end):
        raise ValueError("start and end must have the same length and memory space")
    _check(lib().hpop_add_stream_events(s, resource, stream, ps, pe, len(start), ms), s)


def hpop_stream_metrics(s, flags=0, n_devices=None):
    """Stream trees of every region; given the session's n_devices, also the
    int64 array [region][device][3] of (busy, stream time, streams)."""
    n = hpop_num_regions(s)
    out = (hpop_stream_tree * max(1, n))()
    per = np.zeros((max(1, n), max(1, n_devices), 3), np.int64) if n_devices is not None else None
    _check(lib().hpop_stream_metrics(s, flags, ctypes.cast(out, ctypes.c_void_p),
                                     per.ctypes.data if per is not None else None), s)
    trees = list(out[:n])
    return (trees, per[:n, :n_devices]) if per is not None else trees


def hpop_num_regions(s):
    out = _I32()
    _check(lib().hpop_num_regions(s, ctypes.byref(out)), s)
    return out.value


def hpop_metrics_compute(s, region):
    t = hpop_metric_tree()
    _check(lib().hpop_metrics_compute(s, region, ctypes.byref(t)), s)
    return t


def hpop_metrics_compute_all(s, flags=0):
    n = hpop_num_regions(s)
    out = (hpop_metric_tree * max(1, n))()
    _check(lib().hpop_metrics_compute_all(s, flags, out), s)
    return list(out[:n])


HPOP_STATIC_SCRATCH_BYTES = 256 << 20


def hpop_metrics_compute_static(n_hosts, n_devices, chunks, regions, stream=None, times=False):
    """One-shot evaluation without allocation: chunks are (resource, kind, start, end)
    device tensors, regions (t0, t1) pairs. Returns the trees (a ctypes array),
    and with times=True also an int64 array [regions][n_hosts + n_devices][4]."""
    arr = (hpop_event_chunk * max(1, len(chunks)))()
    for i, (r, k, st, en) in enumerate(chunks):
        ps, _ = _ptr(st)
        pe, _ = _ptr(en)
        if len(st) != len(en):
            raise ValueError("start and end must have the same length")
        arr[i] = hpop_event_chunk(r, k, ps, pe, len(st))
    nreg = len(regions)
    t0 = (_I64 * max(1, nreg))(*[a for a, _ in regions])
    t1 = (_I64 * max(1, nreg))(*[b for _, b in regions])
    out = (hpop_metric_tree * max(1, nreg))()
    tout = np.zeros((nreg, n_hosts + n_devices, 4), np.int64) if times else None
    _check(lib().hpop_metrics_compute_static(
        n_hosts, n_devices, arr, len(chunks), t0, t1, nreg, stream or 0, out,
        tout.ctypes.data_as(ctypes.POINTER(_I64)) if times else None))
    return (out, tout) if times else out


def hpop_resource_times(s, region, resource):
    out = (_I64 * 4)()
    _check(lib().hpop_resource_times(s, region, resource, out), s)
    return list(out)


def hpop_batch_compute(sessions, flags=0):
    """Trees of every region of every session, in order (a ctypes array)."""
    k = len(sessions)
    arr = (_P * k)(*sessions)
    total = sum(hpop_num_regions(s) for s in sessions)
    out = (hpop_metric_tree * max(1, total))()
    _check(lib().hpop_batch_compute(arr, k, flags, out))
    return out if total else []


def hpop_session_get_info(s):
    out = hpop_session_info()
    _check(lib().hpop_session_get_info(s, ctypes.byref(out)), s)
    return out


def hpop_session_set_tuning(s, bucket_target=0, bucket_cap=0, tile_elems=0, scatter_slots=0):
    t = hpop_tuning(bucket_target, bucket_cap, tile_elems, scatter_slots)
    _check(lib().hpop_session_set_tuning(s, ctypes.byref(t)), s)


def hpop_session_get_tuning(s):
    t = hpop_tuning()
    _check(lib().hpop_session_get_tuning(s, ctypes.byref(t)), s)
    return t


def hpop_session_enable_timing(s, on=True):
    _check(lib().hpop_session_enable_timing(s, 1 if on else 0), s)


def hpop_session_time_stage(s, stage=None):
    _check(lib().hpop_session_time_stage(s, stage.encode() if stage else None), s)


def hpop_session_stage_times(s):
    names = (ctypes.c_char_p * 32)()
    ms = (ctypes.c_float * 32)()
    n = _I32()
    _check(lib().hpop_session_stage_times(s, 32, names, ms, ctypes.byref(n)), s)
    return [(names[i].decode(), ms[i]) for i in range(n.value)]


def hpop_autotune(sessions, cache_path=None):
    k = len(sessions)
    arr = (_P * k)(*sessions)
    out = hpop_tuning()
    _check(lib().hpop_autotune(arr, k, cache_path.encode() if cache_path else None, ctypes.byref(out)))
    return out


def hpop_server_create(max_sessions=64, max_inflight=64, queue_capacity=4096, mem_budget_bytes=8 << 30,
                       host_staging_mib=0, list_heap_bytes=0):
    cfg = hpop_server_config(max_sessions, max_inflight, queue_capacity, host_staging_mib, mem_budget_bytes,
                             list_heap_bytes)
    h = _P()
    _check(lib().hpop_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def _check_srv(status, srv):
    if status != HPOP_OK:
        msg = lib().hpop_server_last_error(srv)
        raise HpopError(status, (msg or b"").decode(errors="replace"))


def hpop_server_destroy(srv):
    _check_srv(lib().hpop_server_destroy(srv), None)


def hpop_server_open_session(srv, n_hosts, n_devices, t_origin):
    out = _I32()
    _check_srv(lib().hpop_server_open_session(srv, n_hosts, n_devices, int(t_origin), ctypes.byref(out)), srv)
    return out.value


def hpop_server_submit(srv, sid, chunks, mem_space, t0, t1):
    """chunks: list of (resource, kind, start, end); returns the ticket."""
    arr = (hpop_event_chunk * max(1, len(chunks)))()
    for i, (r, k, st, en) in enumerate(chunks):
        ps, _ = _ptr(st)
        pe, _ = _ptr(en)
        arr[i] = hpop_event_chunk(r, k, ps, pe, len(st))
    tk = _U64()
    _check_srv(lib().hpop_server_submit(srv, sid, arr, len(chunks), mem_space, int(t0), int(t1),
                                        ctypes.byref(tk)), srv)
    return tk.value


def hpop_server_wait(srv, ticket, timeout_ns=-1):
    a = hpop_metric_tree()
    b = hpop_metric_tree()
    _check_srv(lib().hpop_server_wait(srv, ticket, timeout_ns, ctypes.byref(a), ctypes.byref(b)), srv)
    return a, b


def hpop_server_get_stats(srv):
    out = hpop_server_stats()
    _check_srv(lib().hpop_server_get_stats(srv, ctypes.byref(out)), srv)
    return out


def hpop_server_reset_stats(srv):
    _check_srv(lib().hpop_server_reset_stats(srv), srv)


def hpop_server_replay(srv, queries, mem_space):
    """queries: list of (sid, chunks, t0, t1, arrival_ns), chunks either a list of
    (resource, kind, start, end) or a (hpop_event_chunk array, count) pair.
    Returns (region trees, global trees, latency_ns array, wall_ns, busy)."""
    n = len(queries)
    arr = (hpop_replay_query * max(1, n))()
    keep = []
    for i, (sid, chunks, t0, t1, arrival) in enumerate(queries):
        if isinstance(chunks, tuple):
            ca, cnt = chunks
        else:
            cnt = len(chunks)
            ca = (hpop_event_chunk * max(1, cnt))()
            for j, (r, k, st, en) in enumerate(chunks):
                ca[j] = hpop_event_chunk(r, k, _ptr(st)[0], _ptr(en)[0], len(st))
        keep.append(ca)
        arr[i] = hpop_replay_query(sid, cnt, ctypes.cast(ca, ctypes.POINTER(hpop_event_chunk)), int(t0), int(t1),
                                   int(arrival))
    reg = (hpop_metric_tree * max(1, n))()
    glob = (hpop_metric_tree * max(1, n))()
    lat = np.zeros(max(1, n), np.int64)
    wall = _I64()
    busy = _I64()
    _check_srv(lib().hpop_server_replay(srv, arr, n, mem_space, reg, glob,
                                        lat.ctypes.data_as(ctypes.POINTER(_I64)), ctypes.byref(wall),
                                        ctypes.byref(busy)), srv)
    return list(reg)[:n], list(glob)[:n], lat[:n], wall.value, busy.value


# ---------------------------------------------------------------------------
# conveniences over the calls above
# ---------------------------------------------------------------------------

HPOP_FORMAT_TEXT = 0
HPOP_FORMAT_JSON = 1


def hpop_tree_format(t, fmt=HPOP_FORMAT_TEXT):
    """The tree as indented text or as a JSON object (a str)."""
    need = _I64()
    _check(lib().hpop_tree_format(ctypes.byref(t), fmt, None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(int(need.value))
    _check(lib().hpop_tree_format(ctypes.byref(t), fmt, buf, need.value, None))
    return buf.value.decode()


def hpop_region_format(s, region, fmt=HPOP_FORMAT_TEXT):
    """A region's report (its trees and every resource's state times) as text or JSON (a str)."""
    need = _I64()
    _check(lib().hpop_region_format(s, region, fmt, None, 0, ctypes.byref(need)), s)
    buf = ctypes.create_string_buffer(int(need.value))
    _check(lib().hpop_region_format(s, region, fmt, buf, need.value, None), s)
    return buf.value.decode()


def tree_ratios(t):
    return np.array([getattr(t, f) for f in RATIO_FIELDS], np.float64)


def tree_sums(t):
    return np.array([getattr(t, f) for f in SUM_FIELDS], np.int64)


def add_chunks(s, chunks, device=False):
    """Add (resource, kind, start, end) chunks; device=True copies them to torch
    device tensors first and hands device pointers to the engine."""
    if device:
        import torch
        dev = [(r, k, torch.from_numpy(np.ascontiguousarray(a, np.int64)).cuda(),
                torch.from_numpy(np.ascontiguousarray(b, np.int64)).cuda()) for r, k, a, b in chunks]
        torch.cuda.synchronize()
        hpop_add_events_multi(s, dev, HPOP_MEM_DEVICE)
        hpop_session_synchronize(s)  # the copies have left the tensors
        return dev
    host = [(r, k, np.ascontiguousarray(a, np.int64), np.ascontiguousarray(b, np.int64)) for r, k, a, b in chunks]
    hpop_add_events_multi(s, host, HPOP_MEM_HOST)
    return host
