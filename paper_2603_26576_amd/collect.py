"""Python binding of libhpop_collect, the rocprofiler-sdk tool that records
host and device states inside a running HIP application (include/hpop_collect.h).

Argument marshalling only. The functions keep the C names; they work in a
process whose HIP runtime started with the tool loaded: either the process
was launched with the environment of :func:`tool_env`, or the library was
linked in. :func:`read_trace` parses the trace file the tool writes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import HpopError, HPOP_OK, hpop_status_string

_HERE = os.path.dirname(os.path.abspath(__file__))
COLLECT_LIB_PATH = os.path.join(_HERE, "libhpop_collect.so")
TRACE_MAGIC = b"HPOPTRC1"

_lib = None


def collect_lib():
    global _lib
    if _lib is None:
        if not os.path.exists(COLLECT_LIB_PATH):
            raise HpopError(-11, "libhpop_collect.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(COLLECT_LIB_PATH)
        i32, i64, p64 = ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)
        for name, res, args in [
            ("hpop_collect_active", i32, []),
            ("hpop_collect_devices", i32, []),
            ("hpop_collect_now", i64, []),
            ("hpop_collect_begin", i64, []),
            ("hpop_collect_poll", i32, [p64]),
            ("hpop_collect_flush", i32, []),
            ("hpop_collect_count", i64, [i32, i32]),
            ("hpop_collect_copy", i32, [i32, i32, i64, i64, ctypes.c_void_p, ctypes.c_void_p]),
            ("hpop_collect_write", i32, [ctypes.c_char_p]),
            ("hpop_collect_dropped", i64, []),
        ]:
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _check(st):
    if st != HPOP_OK:
        raise HpopError(st, hpop_status_string(st))


def tool_env(out_path=None, base=None):
    """Environment for a child process that loads the tool when its HIP
    runtime starts and, if out_path is given, writes its trace there at exit."""
    env = dict(os.environ if base is None else base)
    env["ROCP_TOOL_LIBRARIES"] = COLLECT_LIB_PATH
    if out_path:
        env["HPOP_COLLECT_OUT"] = out_path
    return env


def hpop_collect_active():
    return int(collect_lib().hpop_collect_active())


def hpop_collect_devices():
    return int(collect_lib().hpop_collect_devices())


def hpop_collect_now():
    return int(collect_lib().hpop_collect_now())


def hpop_collect_begin():
    return int(collect_lib().hpop_collect_begin())


def hpop_collect_poll():
    f = ctypes.c_int64(0)
    _check(collect_lib().hpop_collect_poll(ctypes.byref(f)))
    return f.value


def hpop_collect_flush():
    _check(collect_lib().hpop_collect_flush())


def hpop_collect_count(resource, kind):
    return int(collect_lib().hpop_collect_count(resource, kind))


def hpop_collect_copy(resource, kind, first, count):
    s = np.empty(count, np.int64)
    e = np.empty(count, np.int64)
    _check(collect_lib().hpop_collect_copy(resource, kind, first, count, s.ctypes.data, e.ctypes.data))
    return s, e


def hpop_collect_write(path):
    _check(collect_lib().hpop_collect_write(os.fsencode(path)))


def hpop_collect_dropped():
    return int(collect_lib().hpop_collect_dropped())


def read_trace(path):
    """The trace file of hpop_collect_write: dict with n_hosts, n_devices,
    t_begin, t_end and chunks [(resource, kind, start, end)] (int64 arrays)."""
    raw = open(path, "rb").read()
    if raw[:8] != TRACE_MAGIC:
        raise ValueError("%s is not an hpop trace file" % path)
    pos = 8
    n_hosts, n_devices = np.frombuffer(raw, np.int32, 2, pos)
    pos += 8
    t_begin, t_end = np.frombuffer(raw, np.int64, 2, pos)
    pos += 16
    (n_chunks,) = np.frombuffer(raw, np.int32, 1, pos)
    pos += 4
    chunks = []
    for _ in range(int(n_chunks)):
        resource, kind = np.frombuffer(raw, np.int32, 2, pos)
        pos += 8
        (count,) = np.frombuffer(raw, np.int64, 1, pos)
        pos += 8
        count = int(count)
        start = np.frombuffer(raw, np.int64, count, pos).copy()
        pos += 8 * count
        end = np.frombuffer(raw, np.int64, count, pos).copy()
        pos += 8 * count
        chunks.append((int(resource), int(kind), start, end))
    if pos != len(raw):
        raise ValueError("%s: %d trailing bytes" % (path, len(raw) - pos))
    return {"n_hosts": int(n_hosts), "n_devices": int(n_devices), "t_begin": int(t_begin), "t_end": int(t_end),
            "chunks": chunks}
