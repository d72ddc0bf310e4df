"""Loads the PILS use-case fixtures (printed tables plus reconstructed traces)."""
import os

import numpy as np

import tracegen as tg

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "pils_usecases.txt")
E = 10_000


def load():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, host, dev, trace = [p.strip() for p in line.split("|")]
            h = [float(x) for x in host.split()]
            d = [float(x) for x in dev.split()]
            t = [int(x) for x in trace.split()]
            # printed order PE, MPI_PE, CE, LB, OE -> ratio order PE, MPI_PE, LB, CE, OE
            printed = [h[0], h[1], h[3], h[2], h[4], d[0], d[1], d[2], d[3]]
            cases.append((name, printed, t))
    return cases


def build_trace(t, kernel_streams=1, hidden_memops=0, t0=0):
    """Trace of one PILS case. kernel_streams > 1 splits each kernel interval
    into overlapping pieces on several streams (same union); hidden_memops
    adds memory records lying entirely under kernels."""
    chunks = []
    for r in range(2):
        u, w, mpi = t[3 * r:3 * r + 3]
        bounds = np.cumsum([0, u, w, mpi])
        for k, (a, b) in zip((tg.HOST_USEFUL, tg.HOST_OFFLOAD, tg.HOST_MPI), zip(bounds[:-1], bounds[1:])):
            if b > a:
                chunks.append(tg.Chunk(r, k, np.array([a + t0], np.int64), np.array([b + t0], np.int64)))
    for g in range(2):
        K, M = t[6 + 2 * g:8 + 2 * g]
        res = 2 + g
        if K > 0:
            if kernel_streams <= 1:
                ks, ke = [0], [K]
            else:
                # pieces [j*K/S - ov, (j+1)*K/S + ov) clipped to [0, K): union is [0, K)
                S = kernel_streams
                ks = [max(0, (j * K) // S - 7) for j in range(S)]
                ke = [min(K, ((j + 1) * K) // S + 5) for j in range(S)]
            chunks.append(tg.Chunk(res, tg.DEV_KERNEL, np.array(ks, np.int64) + t0, np.array(ke, np.int64) + t0))
            if hidden_memops:
                hs = np.linspace(0, max(0, K - 2), hidden_memops).astype(np.int64)
                he = np.minimum(hs + 2, K)
                chunks.append(tg.Chunk(res, tg.DEV_MEMOP, hs + t0, he + t0))
        if M > 0:
            chunks.append(tg.Chunk(res, tg.DEV_MEMOP, np.array([K + t0], np.int64), np.array([K + M + t0], np.int64)))
    return tg.Trace(2, 2, chunks, [(t0, t0 + E)])
