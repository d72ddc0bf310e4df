"""Python access to the CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package. The product path (``paper_2603_26576_amd``)
never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hpop_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RATIO_NAMES = ["host_pe", "host_mpi_pe", "host_mpi_lb", "host_mpi_ce", "host_oe",
               "dev_pe", "dev_lb", "dev_ce", "dev_oe"]
SUM_NAMES = ["sumU", "sumW", "sumMPI", "sumOther", "sumUW", "maxUW", "sumK", "sumM", "maxK", "maxKM"]

_lib = None


def load_library(path):
    """ctypes handle with the oracle's signatures (also used to load rebuilt variants)."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.oracle_union_measure.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, P, P, P]
    lib.oracle_union_measure.restype = ctypes.c_int
    lib.oracle_compute.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P, P, P, P,
                                   ctypes.c_int32, P, P, ctypes.c_int32, P, P, P, P]
    lib.oracle_compute.restype = ctypes.c_int
    return lib


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load_library(_LIB)
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def union_measure(s, e, regions):
    lib = _load()
    s = np.ascontiguousarray(s, np.int64)
    e = np.ascontiguousarray(e, np.int64)
    t0 = np.ascontiguousarray([r[0] for r in regions], np.int64)
    t1 = np.ascontiguousarray([r[1] for r in regions], np.int64)
    out = np.zeros(len(regions), np.int64)
    rc = lib.oracle_union_measure(_ptr(s), _ptr(e), s.size, len(regions), _ptr(t0), _ptr(t1), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_union_measure failed: %d" % rc)
    return out


class OracleError(ValueError):
    def __init__(self, code):
        super().__init__("oracle_compute returned %d" % code)
        self.code = code


def compute_arrays(n_hosts, n_devices, resource, kind, start, end, regions, threads=1, lib=None):
    lib = lib or _load()
    resource = np.ascontiguousarray(resource, np.int32)
    kind = np.ascontiguousarray(kind, np.int32)
    start = np.ascontiguousarray(start, np.int64)
    end = np.ascontiguousarray(end, np.int64)
    nreg = len(regions)
    t0 = np.ascontiguousarray([r[0] for r in regions], np.int64)
    t1 = np.ascontiguousarray([r[1] for r in regions], np.int64)
    R = n_hosts + n_devices
    times = np.zeros((nreg, R, 4), np.int64)
    sums = np.zeros((nreg, 10), np.int64)
    ratios = np.zeros((nreg, 9), np.float64)
    mask = np.zeros(nreg, np.uint32)
    rc = lib.oracle_compute(n_hosts, n_devices, start.size, _ptr(resource), _ptr(kind), _ptr(start),
                            _ptr(end), nreg, _ptr(t0), _ptr(t1), int(threads), _ptr(times), _ptr(sums),
                            _ptr(ratios), _ptr(mask))
    if rc != 0:
        raise OracleError(rc)
    return {"times": times, "sums": sums, "ratios": ratios, "mask": mask}


def compute(trace, threads=1, regions=None, lib=None):
    """Evaluate a tracegen.Trace: dict with times, sums, ratios, mask arrays."""
    res, kind, s, e = trace.flat()
    return compute_arrays(trace.n_hosts, trace.n_devices, res, kind, s, e,
                          trace.regions if regions is None else regions, threads, lib)
