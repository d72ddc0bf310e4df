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


HOST_LEVELS = [(0,), (0, 1), (0, 1, 2)]   # {U}, {U, W}, {U, W, MPI} by kind
DEVICE_LEVELS = [(3,), (3, 4)]            # {K}, {K, M}


def _ratio(num, den, bit, mask):
    """One IEEE division of two exact integers; 0/0 := 1, flagged (as the C oracle)."""
    if den == 0:
        mask[0] |= 1 << bit
        return 1.0
    return float(num) / float(den)


def compute_multi(trace, regions):
    """Regions entered repeatedly, each resource on its own clock: regions[g] is
    a list of (resource, a, b) with disjoint [a, b) per resource.

    Plain definition: for resource r and nested level l, D_l(r) is the sum over
    r's intervals of the union measure of the level's records inside it (the
    C union_measure); E_r is r's own time in the region. Host: U = D_0,
    W = D_1 - D_0, MPI = D_2 - D_1, Other = E_r - D_2; device: K = D_0,
    M = D_1 - D_0, Idle = E_r - D_1. E follows eq. 1 literally: the largest
    E_r over host processes (over devices when no host process is in the
    region). Aggregates and ratios as eqs. 4-12, each ratio one IEEE division.
    """
    n, m = trace.n_hosts, trace.n_devices
    R = n + m
    res, kind, s, e = trace.flat()
    nreg = len(regions)
    times = np.zeros((nreg, R, 4), np.int64)
    sums = np.zeros((nreg, 10), np.int64)
    ratios = np.zeros((nreg, 9), np.float64)
    masks = np.zeros(nreg, np.uint32)
    Es = np.zeros(nreg, np.int64)
    for g, ivls in enumerate(regions):
        per = [[] for _ in range(R)]
        for r, a, b in ivls:
            per[r].append((int(a), int(b)))
        Er = np.array([sum(b - a for a, b in per[r]) for r in range(R)], np.int64)
        E = int(Er[:n].max()) if n and Er[:n].max() > 0 else (int(Er[n:].max()) if m else 0)
        Es[g] = E
        for r in range(R):
            levels = HOST_LEVELS if r < n else DEVICE_LEVELS
            D = []
            for kinds in levels:
                sel = (res == r) & np.isin(kind, kinds)
                D.append(int(union_measure(s[sel], e[sel], per[r]).sum()) if per[r] else 0)
            if r < n:
                times[g, r] = [D[0], D[1] - D[0], D[2] - D[1], Er[r] - D[2]]
            else:
                times[g, r] = [D[0], D[1] - D[0], Er[r] - D[1], 0]
        h, d = times[g, :n], times[g, n:]
        sU, sW, sMPI, sO = (int(h[:, i].sum()) for i in range(4))
        sUW = sU + sW
        mUW = int((h[:, 0] + h[:, 1]).max()) if n else 0
        sK, sM = int(d[:, 0].sum()), int(d[:, 1].sum())
        mK = int(d[:, 0].max()) if m else 0
        mKM = int((d[:, 0] + d[:, 1]).max()) if m else 0
        sums[g] = [sU, sW, sMPI, sO, sUW, mUW, sK, sM, mK, mKM]
        mk = [0]
        ratios[g] = [_ratio(sU, n * E, 0, mk), _ratio(sUW, n * E, 1, mk), _ratio(sUW, n * mUW, 2, mk),
                     _ratio(mUW, E, 3, mk), _ratio(sU, sUW, 4, mk), _ratio(sK, m * E, 5, mk),
                     _ratio(sK, m * mK, 6, mk), _ratio(mK, mKM, 7, mk), _ratio(mKM, E, 8, mk)]
        masks[g] = mk[0]
    return {"times": times, "sums": sums, "ratios": ratios, "mask": masks, "E": Es}


def compute_streams(n_streams, chunks, regions):
    """Stream concurrency of the devices (the stream-level row; the paper
    leaves streams to its future Device Computational Efficiency branch,
    Sec. 4.1, so the definition is this engine's reading).

    n_streams[g]: streams declared on device g (all count, busy or not).
    chunks: (device g, stream s, start, end) kernel records, s < n_streams[g].
    regions: [(t0, t1)].

    Plain definition, per region and device g: U_gs = union measure of the
    records of stream s inside the region (the C union_measure); B_g = union
    measure of all records of g; ST_g = sum_s U_gs (the stream time: the
    integral of the number of active streams). Aggregates over devices:
    busy = sum_g B_g, stream_time = sum_g ST_g, capacity = sum_g S_g B_g;
    efficiency = stream_time / capacity (bit 0 when 0/0), mean_active =
    stream_time / busy (bit 1). Each ratio one IEEE division; 0/0 := 1.
    Returns per_device [region][g] = (B_g, ST_g, S_g), sums [region] =
    (busy, stream_time, capacity), ratios, mask.
    """
    m = len(n_streams)
    nreg = len(regions)
    per = np.zeros((nreg, m, 3), np.int64)
    sums = np.zeros((nreg, 3), np.int64)
    ratios = np.zeros((nreg, 2), np.float64)
    masks = np.zeros(nreg, np.uint32)
    for g in range(m):
        sel = [c for c in chunks if c[0] == g]
        s_all = np.concatenate([np.asarray(c[2], np.int64) for c in sel]) if sel else np.zeros(0, np.int64)
        e_all = np.concatenate([np.asarray(c[3], np.int64) for c in sel]) if sel else np.zeros(0, np.int64)
        B = union_measure(s_all, e_all, regions) if nreg else np.zeros(0, np.int64)
        ST = np.zeros(nreg, np.int64)
        for st in range(int(n_streams[g])):
            cs = [c for c in sel if c[1] == st]
            if not cs:
                continue
            ss = np.concatenate([np.asarray(c[2], np.int64) for c in cs])
            ee = np.concatenate([np.asarray(c[3], np.int64) for c in cs])
            ST += union_measure(ss, ee, regions)
        per[:, g, 0] = B
        per[:, g, 1] = ST
        per[:, g, 2] = int(n_streams[g])
    for r in range(nreg):
        busy = int(per[r, :, 0].sum())
        stream_time = int(per[r, :, 1].sum())
        capacity = int((per[r, :, 0] * per[r, :, 2]).sum())
        sums[r] = [busy, stream_time, capacity]
        mk = [0]
        ratios[r] = [_ratio(stream_time, capacity, 0, mk), _ratio(stream_time, busy, 1, mk)]
        masks[r] = mk[0]
    return {"per_device": per, "sums": sums, "ratios": ratios, "mask": masks}
