"""Seeded synthetic trace generator (host states and device activity).

This module only *produces inputs*: timestamped intervals of host states and
device activity, and the time regions to evaluate. It holds none of the
method's arithmetic (no union, no clipping, no metric formulas), so both the
oracle and the GPU path may consume what it generates.

Kinds follow the paper's state classification: on the host, Useful,
Device Offloading and MPI (Section 4.1, host states); on the device, Kernel
computation and Memory operations (Section 4.1, device states; idle time is
whatever no record covers). Timestamps are int64 nanoseconds; every interval
is half-open [start, end).

Workload recipe (shared by tests and the benchmark):

* time origin T0 = 1.7e18 ns, so keys exercise the full 64-bit range;
* kernel and host-compute durations: lognormal(mu = ln 50 us, sigma = 0.5)
  times a per-rank work factor w;
* gaps: exponential with mean 20 us;
* memory operations: probability 0.2, duration 2 us + size / 25 B/ns with
  size log-uniform in [4 KiB, 64 MiB];
* device streams: an event overlaps the previous one (starts inside it, on
  another stream) with probability 0.3 when the device has more than one
  stream; at most `streams` events overlap in one group, so streams never
  have to serialise;
* host ranks: cycles of Useful followed by a gap labelled Offloading or MPI
  (equal odds), optionally an injected MPI idle interval per cycle, and a
  final MPI barrier up to the end of the whole trace, so each rank's states
  partition the trace span;
* delivery order: device records in completion (end-time) order, host
  records in time order, one chunk per (resource, kind).

Every resource draws from its own child of ``SeedSequence(seed)`` so the
result does not depend on generation order.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

HOST_USEFUL = 0
HOST_OFFLOAD = 1
HOST_MPI = 2
DEV_KERNEL = 3
DEV_MEMOP = 4

T0 = 1_700_000_000_000_000_000

KERNEL_MU = float(np.log(50_000.0))
KERNEL_SIGMA = 0.5
GAP_MEAN = 20_000.0
P_MEMOP = 0.2
P_OVERLAP = 0.3
MEMOP_MIN_BYTES = 4096.0
MEMOP_MAX_BYTES = 64.0 * 1024 * 1024
MEMOP_BYTES_PER_NS = 25.0
MEMOP_LATENCY_NS = 2000


@dataclasses.dataclass
class Chunk:
    resource: int
    kind: int
    start: np.ndarray  # int64
    end: np.ndarray  # int64


@dataclasses.dataclass
class Trace:
    n_hosts: int
    n_devices: int
    chunks: List[Chunk]
    regions: List[Tuple[int, int]]
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def n_events(self) -> int:
        return int(sum(c.start.size for c in self.chunks))

    def flat(self):
        """Concatenate all chunks: (resource, kind, start, end) arrays."""
        if not self.chunks:
            z = np.zeros(0, np.int64)
            return np.zeros(0, np.int32), np.zeros(0, np.int32), z, z
        res = np.concatenate([np.full(c.start.size, c.resource, np.int32) for c in self.chunks])
        kind = np.concatenate([np.full(c.start.size, c.kind, np.int32) for c in self.chunks])
        s = np.concatenate([c.start for c in self.chunks]).astype(np.int64)
        e = np.concatenate([c.end for c in self.chunks]).astype(np.int64)
        return res, kind, s, e

    def span(self) -> Tuple[int, int]:
        lo = min(int(c.start.min()) for c in self.chunks if c.start.size)
        hi = max(int(c.end.max()) for c in self.chunks if c.end.size)
        return lo, hi


# ----------------------------------------------------------------------------
# per-resource timelines
# ----------------------------------------------------------------------------

def _durations(rng, n, w):
    d = rng.lognormal(KERNEL_MU, KERNEL_SIGMA, size=n) * w
    return np.maximum(1, np.rint(d)).astype(np.int64)


def _gaps(rng, n):
    return np.rint(rng.exponential(GAP_MEAN, size=n)).astype(np.int64)


def device_timeline(rng, n_events: int, streams: int, w: float, t0: int,
                    p_memop: float = P_MEMOP, p_overlap: float = P_OVERLAP, return_streams: bool = False):
    """One device's activity: returns (start, end, kind, realised overlap fraction),
    and with return_streams also the stream of every event.

    Events form launch groups. The first event of a group starts a gap after
    the previous group's last end; each further event of the group starts
    inside its predecessor (at a uniform fraction of the predecessor's
    duration), as a launch on another stream would. A group holds at most
    `streams` events, on distinct streams (rotating from group to group), so
    no stream runs two events at once.
    """
    n = int(n_events)
    if n == 0:
        z = np.zeros(0, np.int64)
        out = (z, z, np.zeros(0, np.int32), 0.0)
        return out + (np.zeros(0, np.int32),) if return_streams else out
    is_mem = rng.random(n) < p_memop
    kdur = _durations(rng, n, w)
    size = np.exp(rng.uniform(np.log(MEMOP_MIN_BYTES), np.log(MEMOP_MAX_BYTES), size=n))
    mdur = MEMOP_LATENCY_NS + np.rint(size / MEMOP_BYTES_PER_NS).astype(np.int64)
    d = np.where(is_mem, mdur, kdur).astype(np.int64)
    kind = np.where(is_mem, DEV_MEMOP, DEV_KERNEL).astype(np.int32)

    if streams > 1:
        ov = rng.random(n) < p_overlap
    else:
        ov = np.zeros(n, bool)
    ov[0] = False
    frac = rng.random(n)

    def groups(flags):
        first = np.flatnonzero(~flags)
        gid = np.cumsum(~flags) - 1
        pos = np.arange(n) - first[gid]
        return first, gid, pos

    first, gid, pos = groups(ov)
    # at most `streams` events share a group, so no stream runs two at once
    ov = ov & (pos % max(streams, 1) != 0)
    first, gid, pos = groups(ov)

    step = np.zeros(n, np.int64)
    step[1:] = np.floor(frac[1:] * d[:-1]).astype(np.int64)
    step[~ov] = 0
    cs = np.cumsum(step)
    off = cs - cs[first[gid]]
    rel_end = off + d
    extent = np.maximum.reduceat(rel_end, first)
    g = first.size
    gap = _gaps(rng, g)
    prev_extent = np.concatenate([[0], extent[:-1]]).astype(np.int64)
    gstart = t0 + np.cumsum(gap + prev_extent)
    s = gstart[gid] + off
    e = s + d
    out = (s.astype(np.int64), e.astype(np.int64), kind, float(ov.mean()))
    if return_streams:
        return out + (((gid + pos) % max(streams, 1)).astype(np.int32),)
    return out


def host_timeline(rng, n_events: int, w: float, t0: int, idle_frac: Optional[float] = None):
    """One host rank's states as back-to-back intervals (before the final barrier).

    Returns (start, end, kind). Each cycle is Useful then a gap labelled
    Offloading or MPI; with `idle_frac` f an extra MPI interval of length
    f/(1-f) times the cycle is appended to each cycle.
    """
    per_cycle = 2 if idle_frac is None else 3
    cycles = max(1, int(n_events) // per_cycle)
    u = _durations(rng, cycles, w)
    gap = np.maximum(1, _gaps(rng, cycles))
    gap_kind = np.where(rng.random(cycles) < 0.5, HOST_OFFLOAD, HOST_MPI).astype(np.int32)
    parts_d = [u, gap]
    parts_k = [np.full(cycles, HOST_USEFUL, np.int32), gap_kind]
    if idle_frac is not None:
        f = float(idle_frac)
        idle = np.maximum(1, np.rint(f / (1.0 - f) * (u + gap))).astype(np.int64)
        parts_d.append(idle)
        parts_k.append(np.full(cycles, HOST_MPI, np.int32))
    d = np.stack(parts_d, axis=1).reshape(-1)
    k = np.stack(parts_k, axis=1).reshape(-1)
    s = t0 + np.concatenate([[0], np.cumsum(d)[:-1]])
    e = s + d
    return s.astype(np.int64), e.astype(np.int64), k


def _device_chunks(resource, s, e, kind):
    order = np.argsort(e, kind="stable")  # completion order
    s, e, kind = s[order], e[order], kind[order]
    out = []
    for k in (DEV_KERNEL, DEV_MEMOP):
        sel = kind == k
        if sel.any():
            out.append(Chunk(resource, k, np.ascontiguousarray(s[sel]), np.ascontiguousarray(e[sel])))
    return out


def _host_chunks(resource, s, e, kind):
    out = []
    for k in (HOST_USEFUL, HOST_OFFLOAD, HOST_MPI):
        sel = kind == k
        if sel.any():
            out.append(Chunk(resource, k, np.ascontiguousarray(s[sel]), np.ascontiguousarray(e[sel])))
    return out


def make_trace(seed: int, n_ranks: int, n_devices: int, streams: int,
               dev_events: int, host_events: int,
               w_range: Tuple[float, float] = (1.0, 1.0),
               idle_range: Optional[Tuple[float, float]] = None,
               p_memop: float = P_MEMOP, t0: int = T0,
               regions: str = "global", n_regions: int = 1,
               seed_seq: Optional[np.random.SeedSequence] = None) -> Trace:
    """Build one trace. `regions` is "global", "nested" or "tiles"."""
    ss = seed_seq if seed_seq is not None else np.random.SeedSequence(seed)
    kids = ss.spawn(1 + n_ranks + n_devices)
    prng = np.random.default_rng(kids[0])
    w = prng.uniform(w_range[0], w_range[1], size=max(n_ranks, n_devices))
    idle = None
    if idle_range is not None:
        idle = prng.uniform(idle_range[0], idle_range[1], size=n_ranks)
    streams_s = streams

    chunks: List[Chunk] = []
    ov_fracs = []
    dev_parts = []
    for g in range(n_devices):
        rng = np.random.default_rng(kids[1 + n_ranks + g])
        s, e, k, ovf = device_timeline(rng, dev_events, streams_s, float(w[g]), t0, p_memop)
        dev_parts.append((s, e, k))
        ov_fracs.append(ovf)
    host_parts = []
    for r in range(n_ranks):
        rng = np.random.default_rng(kids[1 + r])
        s, e, k = host_timeline(rng, host_events, float(w[r]), t0,
                                None if idle is None else float(idle[r]))
        host_parts.append((s, e, k))
    t_end = t0 + 1
    for s, e, _ in dev_parts + host_parts:
        if e.size:
            t_end = max(t_end, int(e.max()))
    for r, (s, e, k) in enumerate(host_parts):
        last = int(e[-1]) if e.size else t0
        if last < t_end:  # final MPI barrier up to the end of the trace
            s = np.concatenate([s, [last]]).astype(np.int64)
            e = np.concatenate([e, [t_end]]).astype(np.int64)
            k = np.concatenate([k, [HOST_MPI]]).astype(np.int32)
        chunks.extend(_host_chunks(r, s, e, k))
    for g, (s, e, k) in enumerate(dev_parts):
        chunks.extend(_device_chunks(n_ranks + g, s, e, k))

    L = t_end - t0
    regs: List[Tuple[int, int]]
    if regions == "global":
        regs = [(t0, t_end)]
    elif regions == "nested":
        q = L // 34
        regs = [(t0 + k * q, t_end - k * q) for k in range(n_regions)]
    elif regions == "tiles":
        tiles = n_regions - 1
        bounds = [t0 + (j * L) // tiles for j in range(tiles)] + [t_end]
        regs = [(t0, t_end)] + [(bounds[j], bounds[j + 1]) for j in range(tiles)]
    elif regions == "halving":
        regs = [(t0, t_end)]
        for frac_den in (2, 4, 8):
            half = L // (2 * frac_den)
            mid = t0 + L // 2
            regs.append((mid - half, mid + half))
        regs = regs[:n_regions]
    else:
        raise ValueError(regions)
    info = {"t0": t0, "t_end": t_end, "overlap_fraction": float(np.mean(ov_fracs)) if ov_fracs else 0.0,
            "streams": streams}
    return Trace(n_ranks, n_devices, chunks, regs, info)


# ----------------------------------------------------------------------------
# the workload configurations
# ----------------------------------------------------------------------------

def stream_kernels(seed: int, n_devices: int, streams: int, events_per_device: int, t0: int = T0,
                   w_range=(0.5, 1.5), p_overlap: float = 0.5):
    """Kernel records per (device, stream) with the launch-group shape of
    device_timeline: returns (streams per device, [(device, stream, start, end)])."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(w_range[0], w_range[1], size=n_devices)
    chunks = []
    for g in range(n_devices):
        s, e, _, _, st = device_timeline(rng, events_per_device, streams, float(w[g]), t0, p_memop=0.0,
                                         p_overlap=p_overlap, return_streams=True)
        for k in range(streams):
            sel = st == k
            if sel.any():
                chunks.append((g, k, s[sel], e[sel]))
    return [streams] * n_devices, chunks


def small(seed: int = 1001) -> Trace:
    """4 ranks, one device each, 2 streams, 10^4 events per resource, 1 region."""
    return make_trace(seed, 4, 4, 2, 10_000, 10_000, regions="global")


def mid(seed: int = 1002, scale: float = 1.0) -> Trace:
    """64 ranks x 64 devices x 8 streams, 10^7 device events, 16 nested regions."""
    dev = max(1, int(round(156_250 * scale)))
    host = max(2, int(round(39_062 * scale)))
    return make_trace(seed, 64, 64, 8, dev, host, w_range=(0.8, 1.2),
                      regions="nested", n_regions=16)


def large(seed: int = 1003, scale: float = 1.0, ranks: int = 256) -> Trace:
    """256 ranks x 256 devices x 4 streams, 10^8 device events, host-idle 0.1-0.4, 64 regions."""
    dev = max(1, int(round(390_625 * scale)))
    host = max(3, int(round(97_656 * scale)))
    return make_trace(seed, ranks, ranks, 4, dev, host, w_range=(0.5, 1.5),
                      idle_range=(0.1, 0.4), regions="tiles", n_regions=64)


def batched(seed: int = 1004, n_traces: int = 1000, max_events: float = 1e6,
            min_events: float = 1e3) -> List[Trace]:
    """Independent traces of log-uniform size, 1-128 ranks, 1-8 streams, 4 nested regions."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(n_traces)
    out = []
    for i in range(n_traces):
        rng = np.random.default_rng(kids[i].spawn(1)[0])
        n_ev = int(np.rint(10 ** rng.uniform(np.log10(min_events), np.log10(max_events))))
        ranks = int(rng.integers(1, 129))
        streams = int(rng.integers(1, 9))
        dev_total = (4 * n_ev) // 5
        host_total = n_ev - dev_total
        dev_per = max(1, dev_total // ranks)
        host_per = max(2, host_total // ranks)
        out.append(make_trace(0, ranks, ranks, streams, dev_per, host_per, w_range=(0.8, 1.2),
                              regions="halving", n_regions=4, seed_seq=kids[i]))
    return out


def serving_sessions(seed: int = 1005, n_sessions: int = 32, ranks: int = 16, streams: int = 4,
                     warm_events: int = 1_000_000):
    """Warm state for the serving workload: one trace per session, no regions yet."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(n_sessions)
    out = []
    per_res = max(2, warm_events // (2 * ranks))
    for i in range(n_sessions):
        out.append(make_trace(0, ranks, ranks, streams, (4 * per_res) // 2 + per_res // 2,
                              per_res // 2, w_range=(0.8, 1.2), seed_seq=kids[i]))
    return out


def continue_trace(rng, n_ranks: int, n_devices: int, streams: int, n_events: int,
                   frontier: int, p_early: float = 0.01, early_back: int = 200_000) -> List[Chunk]:
    """New records for one serving query, continuing a session after `frontier`.

    With probability `p_early` the batch starts up to `early_back` ns before
    the frontier (records completing out of order).
    """
    start = frontier
    if rng.random() < p_early:
        start = frontier - int(rng.integers(1, early_back))
    dev_total = (4 * n_events) // 5
    host_total = n_events - dev_total
    chunks: List[Chunk] = []
    dev_per = max(1, dev_total // n_devices)
    host_per = max(2, host_total // n_ranks)
    w = 1.0
    ends = []
    parts = []
    for g in range(n_devices):
        s, e, k, _ = device_timeline(rng, dev_per, streams, w, start)
        parts.append(("d", n_ranks + g, s, e, k))
        ends.append(int(e.max()))
    for r in range(n_ranks):
        s, e, k = host_timeline(rng, host_per, w, start)
        parts.append(("h", r, s, e, k))
        ends.append(int(e.max()))
    t_end = max(ends)
    for typ, res, s, e, k in parts:
        if typ == "h":
            last = int(e[-1])
            if last < t_end:
                s = np.concatenate([s, [last]]).astype(np.int64)
                e = np.concatenate([e, [t_end]]).astype(np.int64)
                k = np.concatenate([k, [HOST_MPI]]).astype(np.int32)
            chunks.extend(_host_chunks(res, s, e, k))
        else:
            chunks.extend(_device_chunks(res, s, e, k))
    return chunks


def random_tiny(rng, max_span: int = 64, max_events: int = 12, n_hosts: Optional[int] = None,
                n_devices: Optional[int] = None, n_regions: int = 3, t0: int = 0,
                allow_empty: bool = True) -> Trace:
    """Small random traces with arbitrary overlaps, for brute-force comparison."""
    n = int(rng.integers(0, 4)) if n_hosts is None else n_hosts
    m = int(rng.integers(0, 4)) if n_devices is None else n_devices
    if n + m == 0:
        m = 1
    chunks = []
    for r in range(n + m):
        kinds = (HOST_USEFUL, HOST_OFFLOAD, HOST_MPI) if r < n else (DEV_KERNEL, DEV_MEMOP)
        for k in kinds:
            c = int(rng.integers(0, max_events + 1))
            if c == 0:
                continue
            s = rng.integers(0, max_span, size=c)
            ln = rng.integers(0 if allow_empty else 1, max(2, max_span // 3), size=c)
            e = np.minimum(s + ln, max_span)
            chunks.append(Chunk(r, k, (s + t0).astype(np.int64), (e + t0).astype(np.int64)))
    regs = []
    for _ in range(n_regions):
        a = int(rng.integers(-2, max_span + 1))
        b = int(rng.integers(a + 1, max_span + 4))
        regs.append((a + t0, b + t0))
    return Trace(n, m, chunks, regs)
