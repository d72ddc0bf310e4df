"""Brute-force, per-nanosecond reading of the paper's state classification.

Independent of the oracle (no shared code): for every nanosecond t of a small
trace it decides each resource's state directly from the paper's rules and
counts nanoseconds.

* device (Section 4.1 device states, Section 4.2 post-processing): a
  nanosecond covered by any kernel record is Kernel (overlap between
  computation and communication counts as computation; overlapping kernels
  count once), else Memory if covered by a memory record, else Idle;
* host (Section 4.1 host states): Useful if covered by a Useful record, else
  Offloading if covered by an Offloading record, else MPI if covered by an
  MPI record, else Other.

The metric formulas below are typed from eqs. 6-12 (and eqs. 4-5 for the MPI
children with Useful+Offloading as the useful state), with 0/0 taken as 1.
"""
from __future__ import annotations

import numpy as np

HOST_USEFUL, HOST_OFFLOAD, HOST_MPI, DEV_KERNEL, DEV_MEMOP = 0, 1, 2, 3, 4


def occupancy_times(trace):
    """times[region][resource][4] by counting nanoseconds."""
    n, m = trace.n_hosts, trace.n_devices
    R = n + m
    pts = [t for r in trace.regions for t in r]
    for c in trace.chunks:
        if c.start.size:
            pts += [int(c.start.min()), int(c.end.max())]
    lo, hi = min(pts), max(pts)
    T = hi - lo
    assert T <= 1 << 22, "brute force is for tiny traces"
    occ = np.zeros((R, 5, T), bool)
    for c in trace.chunks:
        for s, e in zip(c.start.tolist(), c.end.tolist()):
            occ[c.resource, c.kind, s - lo:e - lo] = True
    out = np.zeros((len(trace.regions), R, 4), np.int64)
    for g, (t0, t1) in enumerate(trace.regions):
        w = slice(t0 - lo, t1 - lo)
        E = t1 - t0
        for r in range(R):
            if r < n:
                u = occ[r, HOST_USEFUL, w]
                wo = occ[r, HOST_OFFLOAD, w] & ~u
                mp = occ[r, HOST_MPI, w] & ~u & ~wo
                out[g, r] = [u.sum(), wo.sum(), mp.sum(), E - u.sum() - wo.sum() - mp.sum()]
            else:
                k = occ[r, DEV_KERNEL, w]
                mm = occ[r, DEV_MEMOP, w] & ~k
                out[g, r] = [k.sum(), mm.sum(), E - k.sum() - mm.sum(), 0]
    return out


def _div(a, b):
    return 1.0 if b == 0 else a / b


def tree_from_times(times, n, m, regions):
    """Aggregates and the two metric trees from per-resource state times."""
    sums, ratios, masks = [], [], []
    for g, (t0, t1) in enumerate(regions):
        E = t1 - t0
        h = times[g, :n]
        d = times[g, n:]
        U = [int(x) for x in h[:, 0]]
        W = [int(x) for x in h[:, 1]]
        UW = [u + w for u, w in zip(U, W)]
        K = [int(x) for x in d[:, 0]]
        KM = [int(k) + int(x) for k, x in zip(K, d[:, 1])]
        s = [sum(U), sum(W), int(h[:, 2].sum()), int(h[:, 3].sum()), sum(UW), max(UW, default=0),
             sum(K), int(d[:, 1].sum()), max(K, default=0), max(KM, default=0)]
        pairs = [
            (sum(U), n * E),                   # host hybrid PE
            (sum(UW), n * E),                  # MPI PE
            (sum(UW), n * max(UW, default=0)),  # MPI load balance
            (max(UW, default=0), E),           # MPI communication efficiency
            (sum(U), sum(UW)),                 # device offload efficiency
            (sum(K), m * E),                   # device PE
            (sum(K), m * max(K, default=0)),   # device load balance
            (max(K, default=0), max(KM, default=0)),  # device communication efficiency
            (max(KM, default=0), E),           # orchestration efficiency
        ]
        mask = 0
        vals = []
        for j, (a, b) in enumerate(pairs):
            if b == 0:
                assert a == 0
                mask |= 1 << j
            vals.append(_div(a, b))
        sums.append(s)
        ratios.append(vals)
        masks.append(mask)
    return np.array(sums, np.int64), np.array(ratios, np.float64), np.array(masks, np.uint32)
