"""Benchmark: trace records reduced to the full host and device metric trees per second.

One step = one full build and reduction of the whole workload on the GPU:
validation and per-resource statistics, time-bucket histogram and scatter,
LDS sort and flattening of every state level, region clipping of every
(region, resource) pair, reductions and the FP64 ratios of every region, and
the copy of the trees to the host. The records are resident in HBM (in the
session) when the timed region starts.

Default workload: 256 host ranks x 256 devices x 4 streams, 10^8 device
records plus 2.5x10^7 host records (2.0 GB of int64 start/end), host-idle
fraction 0.1-0.4 per rank, 64 regions (the whole span and 63 tiles of it).

Prints one JSON line. Extra legs (regions entered repeatedly, batched
traces, serving, stream concurrency, the live collector on its test
application) are reported as sub-objects of the same
line; the CPU baseline times the oracle on a bounded sample of the same
workload.
"""
import argparse
import hashlib
import json
import os
import re
import shutil
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
COLLECT_APP = os.path.join(ROOT, "tests", "apps", "collect_app")
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ALGO_BYTES_PER_RECORD = 16  # each record's start and end, read once
METRIC = "trace events/sec reduced to full metric tree"

# algorithmic bytes per unit of each build kernel (a unit is a record, except
# where noted); the minimum each kernel must move for its role
ALGO_BYTES = {
    "stats": 8,          # read start
    "hist": 16,          # read start + end (exact-count fallback only)
    "scatter": None,     # read start + end, write the 8 B bucketed form (16 B form: +8)
    "merge_wave": None,  # read the 8 B bucketed form (16 B: +8), write 8 B per merged
                         # interval and level (16 B on resources with buckets wider than 2^30 ns)
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the sources that define the build kernels (their code, launch shapes and data layout)
KERNEL_SOURCES = ("hpop_kernels.hip", "hpop_kernels.h", "hpop_device.h", "hpop_geom.h", "hpop_internal.h")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_26576_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this
    kernel and workload (its own record, else its line in the record of every
    build kernel), if it was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (kernel, workload))
    whole = not os.path.exists(p)
    if whole:
        p = os.path.join(ROOT, "profiles", "traffic_path_%s.txt" % workload)
        if not os.path.exists(p):
            return None
    d = {}
    for line in open(p):
        if ":" in line and not line.startswith("#"):
            k, v = line.rsplit(":", 1) if line.startswith("kernel ") else line.split(":", 1)
            d[k.strip()] = v.strip()
    if d.get("source_hash") != kernel_source_hash():
        return None
    try:
        if not whole:
            return int(d["bytes_per_launch"])
        # "kernel <name>: bytes", the name with its template arguments (one
        # instantiation runs per build)
        pat = re.compile(r"::k_%s(<|$)" % re.escape(kernel))
        hits = [int(v) for k, v in d.items() if k.startswith("kernel ") and pat.search(k)]
        return hits[0] if len(hits) == 1 else None
    except (KeyError, ValueError):
        return None


def upload_session(hp, trace):
    import torch
    s = hp.hpop_session_create(trace.n_hosts, trace.n_devices)
    dev = []
    for c in trace.chunks:
        dev.append((c.resource, c.kind, torch.from_numpy(c.start).cuda(), torch.from_numpy(c.end).cuda()))
    torch.cuda.synchronize()
    hp.hpop_add_events_multi(s, dev, hp.HPOP_MEM_DEVICE)
    hp.hpop_session_synchronize(s)
    del dev
    for a, b in trace.regions:
        hp.hpop_region_define(s, a, b)
    return s


def save_trace_cache(path, trace):
    arrs = {"meta": np.array([trace.n_hosts, trace.n_devices, len(trace.chunks)], np.int64),
            "regions": np.array(trace.regions, np.int64),
            "info": np.array([trace.info["t0"], trace.info["t_end"]], np.int64),
            "ovf": np.array([trace.info["overlap_fraction"]])}
    for i, c in enumerate(trace.chunks):
        arrs["c%d" % i] = np.array([c.resource, c.kind], np.int64)
        arrs["s%d" % i] = c.start
        arrs["e%d" % i] = c.end
    np.savez(path, **arrs)


def load_trace_cache(path, tg):
    if not os.path.exists(path):
        return None
    z = np.load(path)
    n, m, nc = (int(x) for x in z["meta"])
    chunks = [tg.Chunk(int(z["c%d" % i][0]), int(z["c%d" % i][1]), z["s%d" % i], z["e%d" % i]) for i in range(nc)]
    info = {"t0": int(z["info"][0]), "t_end": int(z["info"][1]), "overlap_fraction": float(z["ovf"][0]), "streams": 4}
    return tg.Trace(n, m, chunks, [tuple(int(v) for v in r) for r in z["regions"]], info)


def bench_single(hp, trace, steps, warmup, workload, tune_cache=None):
    import torch
    s = upload_session(hp, trace)
    n_events = trace.n_events
    try:
        t = time.time()
        tun = hp.hpop_autotune([s], tune_cache)  # bucket size, on-chip capacity, tile; cached per size class
        log("autotune: %.1f s -> target %d cap %d tile %d slots %d" % (time.time() - t, tun.bucket_target,
                                                                   tun.bucket_cap, tun.tile_elems, tun.scatter_slots))
        for _ in range(warmup):
            hp.hpop_metrics_compute_all(s, hp.HPOP_FORCE_REBUILD)
        # every stage's device time, from untimed steps with a HIP event after
        # each stage; the longest stage is the dominant kernel
        hp.hpop_session_enable_timing(s, True)
        cal_steps = max(3, steps // 2)
        stage_tot = {}
        for _ in range(cal_steps):
            hp.hpop_metrics_compute_all(s, hp.HPOP_FORCE_REBUILD)
            for name, ms in hp.hpop_session_stage_times(s):
                stage_tot[name] = stage_tot.get(name, 0.0) + ms
        stage_ms = {k: v / cal_steps for k, v in stage_tot.items()}
        dom = max((k for k in stage_ms if k in ALGO_BYTES), key=lambda k: stage_ms[k])
        # the timed steps: HIP events only right around the dominant kernel,
        # on the session stream it runs on (its launch duration, live)
        hp.hpop_session_time_stage(s, dom)
        dom_tot = 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            trees = hp.hpop_metrics_compute_all(s, hp.HPOP_FORCE_REBUILD)
            for name, ms in hp.hpop_session_stage_times(s):
                if name == dom:
                    dom_tot += ms
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        hp.hpop_session_time_stage(s, None)
        hp.hpop_session_enable_timing(s, False)
        stage_ms[dom] = dom_tot / steps
        info = hp.hpop_session_get_info(s)
        # graph-replayed steps (no per-kernel events) for the launch-overhead view
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            hp.hpop_metrics_compute_all(s, hp.HPOP_FORCE_REBUILD)
        torch.cuda.synchronize()
        dt_graph = (time.perf_counter() - t1) / steps
    finally:
        hp.hpop_session_destroy(s)
    # algorithmic bytes of one launch: 16 B per record (its start and end,
    # read once) times the records one launch processes (all of them)
    algo = ALGO_BYTES_PER_RECORD * n_events
    achieved = algo / (stage_ms[dom] * 1e-3) / 1e9
    # beside it, the minimum bytes of the kernel's own role (its reads and
    # writes in the engine's data layout)
    if dom == "merge_wave":
        role = 8 * n_events + 8 * info.n_wide_records + 8 * info.n_components + 8 * info.n_wide_components
    elif dom == "scatter":
        role = 24 * n_events + 8 * info.n_wide_records
    else:
        role = ALGO_BYTES[dom] * n_events
    role_gbs = role / (stage_ms[dom] * 1e-3) / 1e9
    traffic = load_traffic(dom, workload)
    roof = {"bound": "hbm", "kernel": "k_" + dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": int(algo), "bytes_per_unit": ALGO_BYTES_PER_RECORD,
            "units_per_launch": int(n_events), "avg_launch_ms": round(stage_ms[dom], 4),
            "kernel_role_bytes_per_launch": int(role), "kernel_role_GBps": round(role_gbs, 1),
            "kernel_role_frac": round(role_gbs / HBM_PEAK_GBS, 4),
            "timing": "HIP events around k_%s in each timed step" % dom}
    tuning = {"bucket_target": tun.bucket_target, "bucket_cap": tun.bucket_cap, "tile_elems": tun.tile_elems}
    return {"tuning": tuning, "ms_per_step": dt * 1e3, "ms_per_step_graph": dt_graph * 1e3, "events": n_events,
            "value": n_events / dt, "value_graph": n_events / dt_graph, "stage_ms": stage_ms, "roofline": roof,
            "components": int(info.n_components), "wide_components": int(info.n_wide_components),
            "wide_records": int(info.n_wide_records),
            "buckets": int(info.n_buckets),
            "oversized_buckets": int(info.n_oversized), "trees": trees}


def small_leg(hp, reps=20):
    """Small trace (4 ranks x 4 devices x 2 streams, 8e4 records, the whole
    span as one region): latency of one full rebuild and reduction, with the
    records resident in HBM, median of `reps` calls of the C entry points
    (arguments prepared once): kernels launched one by one, the captured HIP
    graph replayed, and the entry point that allocates nothing; the sum of
    the kernels' HIP-event times; the oracle timed beside it (one warm-up,
    median of 5)."""
    import ctypes

    import oracle
    import torch
    import tracegen as tg
    tr = tg.small()
    L = hp.lib()
    nreg = len(tr.regions)
    out = (hp.hpop_metric_tree * nreg)()
    s = upload_session(hp, tr)

    def med_us(fn):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return round(float(np.median(ts)) * 1e6, 1)

    def call(flags):
        def f():
            st = L.hpop_metrics_compute_all(s, flags, out)
            if st != hp.HPOP_OK:
                raise hp.HpopError(st, hp.hpop_status_string(st))
        return f

    try:
        for _ in range(3):
            call(hp.HPOP_FORCE_REBUILD)()
        direct_us = med_us(call(hp.HPOP_FORCE_REBUILD | hp.HPOP_NO_GRAPH))
        graph_us = med_us(call(hp.HPOP_FORCE_REBUILD))
        hp.hpop_session_enable_timing(s, True)
        ks = []
        for _ in range(reps):
            call(hp.HPOP_FORCE_REBUILD)()
            ks.append(sum(ms for _, ms in hp.hpop_session_stage_times(s)))
        hp.hpop_session_enable_timing(s, False)
        kernel_us = round(float(np.median(ks)) * 1e3, 1)
        want = [bytes(t) for t in hp.hpop_metrics_compute_all(s)]
    finally:
        hp.hpop_session_destroy(s)
    # the same records and region through the entry point that allocates nothing
    dev = [(c.resource, c.kind, torch.from_numpy(c.start).cuda(), torch.from_numpy(c.end).cuda()) for c in tr.chunks]
    torch.cuda.synchronize()
    arr = (hp.hpop_event_chunk * len(dev))(*[hp.hpop_event_chunk(r, k, a.data_ptr(), b.data_ptr(), a.numel())
                                              for r, k, a, b in dev])
    t0s = (ctypes.c_int64 * nreg)(*[a for a, _ in tr.regions])
    t1s = (ctypes.c_int64 * nreg)(*[b for _, b in tr.regions])
    sout = (hp.hpop_metric_tree * nreg)()

    def static_call():
        st = L.hpop_metrics_compute_static(tr.n_hosts, tr.n_devices, arr, len(dev), t0s, t1s, nreg, None, sout, None)
        if st != hp.HPOP_OK:
            raise hp.HpopError(st, hp.hpop_status_string(st))

    static_us = med_us(static_call)
    if [bytes(t) for t in sout] != want:
        raise RuntimeError("the entry point without allocation disagrees with the session path")
    del dev
    ora1 = timed_median(lambda: oracle.compute(tr, threads=1))
    thr = oracle_threads()
    oran = timed_median(lambda: oracle.compute(tr, threads=thr))
    n = tr.n_events
    return {"workload": "small trace", "ranks": 4, "devices": 4, "streams": 2, "regions": nreg, "events": n,
            "timing": "median of %d calls after warm-up" % reps,
            "us_per_compute": direct_us, "us_per_compute_graph": graph_us, "us_per_compute_no_alloc": static_us,
            "kernel_us": kernel_us, "events_per_s": n / (graph_us * 1e-6),
            "oracle": {"us_per_compute": round(ora1 * 1e6, 1), "cores": 1,
                       "us_per_compute_threads": round(oran * 1e6, 1), "threads": thr,
                       "timing": "1 warm-up, median of 5"}}


def mid_leg(hp, steps, warmup, tune_cache=None):
    """Mid trace (64 ranks x 64 devices x 8 streams, 1.25e7 records, 16
    nested regions): the single-trace leg at that size, its whole-path HBM
    figures (the records, 200 MB, and much of the build's traffic fit the
    256 MB last-level cache, so the counter fraction is flagged as
    cache-resident) and the oracle beside it."""
    import tracegen as tg
    t = time.time()
    tr = tg.mid()
    log("mid: generated %d records in %.1f s" % (tr.n_events, time.time() - t))
    r = bench_single(hp, tr, steps, warmup, "mid", tune_cache)
    out = {"workload": "mid trace", "ranks": 64, "devices": 64, "streams": 8, "regions": len(tr.regions),
           "events": tr.n_events, "ms_per_step": round(r["ms_per_step"], 4), "events_per_s": r["value"],
           "graph_replay": {"ms_per_step": round(r["ms_per_step_graph"], 4), "events_per_s": r["value_graph"]},
           "stage_ms": {k: round(v, 4) for k, v in r["stage_ms"].items()}, "roofline": r["roofline"],
           "tuning": r["tuning"]}
    ph = path_hbm(r, "mid")
    ph["cache_resident"] = True
    out["path_hbm"] = ph
    out["cpu_baseline"] = cpu_baseline(tr)
    return out


def bench_batched(hp, traces, steps, warmup, tune_cache=None):
    import torch
    sessions = [upload_session(hp, tr) for tr in traces]
    try:
        n_events = sum(tr.n_events for tr in traces)
        t = time.time()
        hp.hpop_autotune(sessions, tune_cache)  # picks bucket size, on-chip capacity, tile; cached per size class
        log("autotune: %.1f s" % (time.time() - t))
        # the C entry point with its arrays allocated once: the timed loop holds
        # no per-session Python work
        import ctypes
        arr = (ctypes.c_void_p * len(sessions))(*sessions)
        total = sum(hp.hpop_num_regions(s) for s in sessions)
        out = (hp.hpop_metric_tree * max(1, total))()
        L = hp.lib()

        def step():
            st = L.hpop_batch_compute(arr, len(sessions), hp.HPOP_FORCE_REBUILD, out)
            if st != hp.HPOP_OK:
                raise hp.HpopError(st, hp.hpop_status_string(st))

        for _ in range(max(1, warmup)):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        # per-stage device times, from separate steps with HIP-event timing on
        hp.hpop_session_enable_timing(sessions[0], True)
        stage = {}
        for _ in range(steps):
            step()
            for k, ms in hp.hpop_session_stage_times(sessions[0]):
                stage.setdefault(k, []).append(ms)
        hp.hpop_session_enable_timing(sessions[0], False)
        segs = sum(tr.n_hosts + tr.n_devices for tr in traces)
        tun = hp.hpop_session_get_tuning(sessions[0])
    finally:
        for s in sessions:
            hp.hpop_session_destroy(s)
    return {"traces": len(traces), "events": n_events, "segments": segs, "ms_per_step": round(dt * 1e3, 3),
            "events_per_s": n_events / dt,
            "stage_ms": {k: round(float(np.mean(v)), 4) for k, v in stage.items()},
            "tuning": {"bucket_target": tun.bucket_target, "bucket_cap": tun.bucket_cap, "tile_elems": tun.tile_elems}}


def entered_regions(trace, n_regions=16, entries=32, seed=1007):
    """Regions entered repeatedly, each resource on its own clock: region q
    gives every resource `entries` intervals, one in each of `entries` equal
    windows of the span, at a per-resource offset and length."""
    rng = np.random.default_rng(seed)
    lo, hi = trace.info["t0"], trace.info["t_end"]
    w = (hi - lo) // entries
    R = trace.n_hosts + trace.n_devices
    out = []
    for q in range(n_regions):
        off = rng.integers(0, w // 4, size=(R, 1)) + q * (w // (4 * n_regions))
        ln = rng.integers(w // 4, w // 2, size=(R, 1))
        a = lo + np.arange(entries)[None, :] * w + off
        res = np.repeat(np.arange(R), entries)
        out.append(list(zip(res.tolist(), a.ravel().tolist(), (a + ln).ravel().tolist())))
    return out


def entered_regions_leg(hp, trace, reps=20):
    """Region evaluation alone (the merged lists already built): the 64 plain
    regions of the workload, then regions entered repeatedly (every resource
    32 times per region, 16 regions)."""
    import torch
    regions = entered_regions(trace)
    res = {}
    for name, multi in (("plain", False), ("entered", True)):
        s = upload_session(hp, trace) if not multi else None
        if multi:
            s = hp.hpop_session_create(trace.n_hosts, trace.n_devices)
            dev = [(c.resource, c.kind, torch.from_numpy(c.start).cuda(), torch.from_numpy(c.end).cuda())
                   for c in trace.chunks]
            torch.cuda.synchronize()
            hp.hpop_add_events_multi(s, dev, hp.HPOP_MEM_DEVICE)
            hp.hpop_session_synchronize(s)
            del dev
            for ivls in regions:
                hp.hpop_region_define_multi(s, ivls)
        try:
            hp.hpop_session_set_tuning(s, 256, 2048, 2048)
            hp.hpop_metrics_compute_all(s)  # build once
            hp.hpop_metrics_compute_all(s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                hp.hpop_metrics_compute_all(s)  # nothing changed: the region kernels only
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t0) / reps
        finally:
            hp.hpop_session_destroy(s)
    n_ivl = sum(len(r) for r in regions)
    return {"plain_regions": len(trace.regions), "plain_ms_per_pass": round(res["plain"] * 1e3, 4),
            "entered_regions": len(regions), "intervals": n_ivl,
            "entered_ms_per_pass": round(res["entered"] * 1e3, 4),
            "intervals_per_s": n_ivl / res["entered"]}


def streams_workload(n_devices=256, streams=4, per_device=100_000, n_regions=16, seed=1006):
    """Stream-tagged kernel records of every device and the regions the
    streams leg reduces: the whole span, then n_regions - 1 tiles of it."""
    import tracegen as tg
    n_streams, chunks = tg.stream_kernels(seed, n_devices, streams, per_device)
    lo = min(int(c[2].min()) for c in chunks)
    hi = max(int(c[3].max()) for c in chunks)
    # exact integer cuts (float64 cannot hold ns timestamps near 1.7e18)
    cuts = [lo + (hi - lo) * i // (n_regions - 1) for i in range(n_regions)]
    regions = [(lo, hi)] + list(zip(cuts[:-1], cuts[1:]))
    return n_streams, chunks, regions


def streams_leg(hp, steps, warmup, n_devices=256, streams=4, per_device=100_000, n_regions=16, seed=1006):
    """Stream concurrency of every device (hpop_stream_metrics): kernel records
    tagged by stream, in the launch-group shape of the main workload's
    devices, resident in HBM; each step rebuilds the per-stream and per-device
    merged lists and reduces all regions (the whole span and tiles of it)."""
    import torch
    n_streams, chunks, regions = streams_workload(n_devices, streams, per_device, n_regions, seed)
    n_rec = sum(int(c[2].size) for c in chunks)
    s = hp.hpop_session_create(0, n_devices)
    try:
        hp.hpop_session_set_tuning(s, 256, 2048, 2048)
        hp.hpop_session_set_streams(s, n_streams)
        dev = [(g, k, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for g, k, a, b in chunks]
        torch.cuda.synchronize()
        for g, k, a, b in dev:
            hp.hpop_add_stream_events(s, g, k, a, b)
        hp.hpop_session_synchronize(s)
        del dev
        for t0, t1 in regions:
            hp.hpop_region_define(s, t0, t1)
        for _ in range(max(1, warmup)):
            trees = hp.hpop_stream_metrics(s, hp.HPOP_FORCE_REBUILD)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            trees = hp.hpop_stream_metrics(s, hp.HPOP_FORCE_REBUILD)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
    finally:
        hp.hpop_session_destroy(s)
    return {"devices": n_devices, "streams_per_device": streams, "records": n_rec, "regions": len(regions),
            "ms_per_step": round(dt * 1e3, 3), "records_per_s": n_rec / dt,
            "stream_eff": trees[0].stream_eff, "mean_active": trees[0].mean_active}


# device memory taken up front for the serving sessions' lists: every
# component of a run (about 1.5 per record over the levels, 16 B each, for
# 2000 queries of 2.2e5 records and 3.2e7 warm records) with room for lists
# that move as they grow
SERVING_LIST_HEAP = 32 << 30


def serving_workload(n_queries, seed=1005, n_sessions=32, ranks=16, streams=4, warm=1_000_000, device=True):
    """Record streams of the serving workload: per session one trace of
    `ranks` hosts and devices, long enough for its warm-up slice and every
    query that targets it; query sizes log-uniform 10^4-10^6 records, owners
    uniform over the sessions. With device=True each chunk is also uploaded
    to the GPU (device-resident payloads)."""
    import tracegen as tg
    rng = np.random.default_rng(seed)
    sizes = np.rint(10 ** rng.uniform(4, 6, size=n_queries)).astype(np.int64)
    owner = rng.integers(0, n_sessions, size=n_queries)
    kids = np.random.SeedSequence(seed).spawn(n_sessions)

    def gen(i):
        need = warm + int(sizes[owner == i].sum())
        per_res = max(4, need // (2 * ranks))
        return tg.make_trace(0, ranks, ranks, streams, (8 * per_res) // 5, (2 * per_res) // 5 + 3,
                             w_range=(0.8, 1.2), seed_seq=kids[i])

    # sessions are independent (a seed each): generated on the host's threads
    import concurrent.futures
    with concurrent.futures.ThreadPoolExecutor(max_workers=oracle_threads()) as ex:
        traces = list(ex.map(gen, range(n_sessions)))
    sess = []
    for i, tr in enumerate(traces):
        chunks = []
        for c in tr.chunks:
            if device:
                import torch
                ds, de = torch.from_numpy(c.start).cuda(), torch.from_numpy(c.end).cuda()
            else:
                ds = de = None
            chunks.append((c.resource, c.kind, ds, de, np.maximum.accumulate(c.end), c.start, c.end))
        sess.append({"origin": tr.info["t0"], "chunks": chunks, "total": tr.n_events})
    if device:
        import torch
        torch.cuda.synchronize()
    return {"rng": rng, "sizes": sizes, "owner": owner, "sess": sess, "n_sessions": n_sessions, "ranks": ranks,
            "streams": streams, "warm": warm}


def serving_slices(hp, W, sidx, n_rec, cursor, host):
    """hpop_event_chunk array for the next n_rec records of a session (spread
    over its chunks in proportion), the number of chunks used and the largest
    end among them; advances cursor."""
    S = W["sess"][sidx]
    arr = (hp.hpop_event_chunk * len(S["chunks"]))()
    frontier = S["origin"]
    k = 0
    for j, (r, kind, st, en, pmax, hst, hen) in enumerate(S["chunks"]):
        ln = hst.size
        a = cursor[j]
        b = min(ln, a + max(1, int(round(n_rec * ln / S["total"]))))
        if b > a:
            ps = hst.ctypes.data if host else st.data_ptr()
            pe = hen.ctypes.data if host else en.data_ptr()
            arr[k] = hp.hpop_event_chunk(r, kind, ps + 8 * a, pe + 8 * a, b - a)
            k += 1
            frontier = max(frontier, int(pmax[b - 1]))
        cursor[j] = b
    return arr, k, frontier


def cgroup_throttle():
    """(times throttled, throttled us) of this process's cgroup CPU quota, or None."""
    for path, scale in (("/sys/fs/cgroup/cpu.stat", 1.0), ("/sys/fs/cgroup/cpu,cpuacct/cpu.stat", 1e-3),
                        ("/sys/fs/cgroup/cpu/cpu.stat", 1e-3)):
        try:
            kv = dict(line.split() for line in open(path) if len(line.split()) == 2)
        except (OSError, ValueError):
            continue
        if "nr_throttled" in kv:
            us = float(kv.get("throttled_usec", kv.get("throttled_time", 0))) * scale
            return int(kv["nr_throttled"]), us
    return None


def serving_run(hp, W, lam, host, keep=False):
    """One Poisson run of the serving workload at `lam` queries/s: a fresh
    server, every session warmed with its first W["warm"] records (untimed, in
    the run's own memory space), then the queries replayed natively. With
    keep=True also returns, per warm-up and per query, (session, t0, t1,
    record count per chunk so far) and the trees the server answered."""
    import ctypes
    lib = hp.lib()
    n_sessions, ranks = W["n_sessions"], W["ranks"]
    sizes, owner = W["sizes"], W["owner"]
    n_queries = int(sizes.size)
    mem = hp.HPOP_MEM_HOST if host else hp.HPOP_MEM_DEVICE
    srv = hp.hpop_server_create(max_sessions=n_sessions, max_inflight=n_sessions, queue_capacity=1 << 16,
                                mem_budget_bytes=64 << 30, list_heap_bytes=SERVING_LIST_HEAP)
    kept = {"warm": [], "queries": []}
    try:
        sids = [hp.hpop_server_open_session(srv, ranks, ranks, S["origin"]) for S in W["sess"]]
        cursors = [[0] * len(S["chunks"]) for S in W["sess"]]
        closes = [S["origin"] for S in W["sess"]]
        warm_t = []
        for i in range(n_sessions):
            # a host run also fills the server's page-locked pool here (blocks as large as any query)
            arr, k, fr = serving_slices(hp, W, i, W["warm"], cursors[i], host)
            tk = ctypes.c_uint64()
            t1 = max(fr, closes[i] + 1)
            rc = lib.hpop_server_submit(srv, sids[i], arr, k, mem, closes[i], t1, ctypes.byref(tk))
            if rc != hp.HPOP_OK:
                raise hp.HpopError(rc, "warm-up submission of session %d" % i)
            warm_t.append(tk.value)
            kept["warm"].append((i, closes[i], t1, list(cursors[i])))
            closes[i] = t1
        warm_trees = [hp.hpop_server_wait(srv, t) for t in warm_t]
        hp.hpop_server_reset_stats(srv)  # the figures below cover the timed queries only
        base = hp.hpop_server_get_stats(srv)
        plan = []
        for q in range(n_queries):
            i = int(owner[q])
            arr, k, fr = serving_slices(hp, W, i, int(sizes[q]), cursors[i], host)
            t1 = max(fr, closes[i] + 1)
            plan.append((sids[i], arr, k, closes[i], t1))
            kept["queries"].append((i, closes[i], t1, list(cursors[i])))
            closes[i] = t1
        arrivals = np.cumsum(W["rng"].exponential(1.0 / lam, size=n_queries))
        queries = [(sid, (arr, k), a, b, int(arrivals[q] * 1e9)) for q, (sid, arr, k, a, b) in enumerate(plan)]
        thr0 = cgroup_throttle()
        reg, glob, lat_ns, wall_ns, busy = hp.hpop_server_replay(srv, queries, mem)
        thr1 = cgroup_throttle()
        st = hp.hpop_server_get_stats(srv)
    finally:
        hp.hpop_server_destroy(srv)
    wall = wall_ns * 1e-9
    ev = int(sizes.sum())
    lat_us = np.sort(lat_ns) * 1e-3
    steps_run = max(1, st.device_steps - base.device_steps)
    res = {"lambda_req_s": lam, "payload": "host" if host else "device", "queries": n_queries,
           "events": ev,
           "offered_events_per_s": ev / float(arrivals[-1]),
           "events_per_s": ev / wall,
           "achieved_req_s": n_queries / wall,
           "p50_us": round(float(np.percentile(lat_us, 50)), 1),
           "p99_us": round(float(np.percentile(lat_us, 99)), 1),
           "max_us": round(float(lat_us[-1]), 1),
           "mean_batch": round((st.mean_batch * st.device_steps - base.mean_batch * base.device_steps)
                               / steps_run, 2),
           "busy_retries": busy,
           # over the timed queries (statistics restarted after the warm-up)
           "max_submit_us": round(st.max_submit_us, 1), "max_step_us": round(st.max_step_us, 1),
           "host_staging_bytes": int(st.host_staging_bytes),
           "max_host_staging_used": int(st.max_host_staging_used),
           "staging_alloc_us": round(st.max_pinned_alloc_us, 1),
           # longest time of each phase of a device step, in us
           "max_phase_us": {k: round(getattr(st, "max_%s_us" % k), 1)
                            for k in ("prep", "grow", "wait", "h2d", "build", "move", "splice", "region")},
           "mean_phase_us": {k: round(getattr(st, "mean_%s_us" % k), 1)
                             for k in ("prep", "grow", "wait", "h2d", "build", "move", "splice", "region")},
           # longest single runtime call while enqueueing a step, and which
           "max_call_us": round(st.max_call_us, 1),
           "max_call_site": hp.HPOP_CALL_SITES[st.max_call_site] if 0 <= st.max_call_site < len(hp.HPOP_CALL_SITES)
           else None}
    if thr0 and thr1:
        # CPU quota throttling of the process's cgroup during the replay (stalls every thread)
        res["cpu_throttled"] = {"times": thr1[0] - thr0[0], "ms": round((thr1[1] - thr0[1]) * 1e-3, 1)}
    if keep:
        kept["warm_trees"] = warm_trees
        kept["query_trees"] = list(zip(reg, glob))
        return res, kept
    return res


def serving_expected_trace(W, entry):
    """The records a session had received up to and including one query, with
    that query's region and the session's global region: (session, t0, t1,
    records per chunk so far) -> tracegen.Trace for the oracle."""
    import tracegen as tg
    i, t0, t1, cur = entry
    S = W["sess"][i]
    chunks = []
    gmax = S["origin"]
    for (r, kind, _, _, pmax, hst, hen), b in zip(S["chunks"], cur):
        if b > 0:
            chunks.append(tg.Chunk(r, kind, hst[:b], hen[:b]))
            gmax = max(gmax, int(pmax[b - 1]))
    return tg.Trace(W["ranks"], W["ranks"], chunks, [(t0, t1), (S["origin"], gmax)])


def serving_leg(hp, lambdas, n_queries, seed=1005, n_sessions=32, ranks=16, streams=4, warm=1_000_000,
                host_lambdas=()):
    """Poisson region-close queries against device-resident sessions.

    Each session's record stream is generated once and uploaded to the GPU;
    its first `warm` records are applied untimed, then every query takes the
    next slice of its session's stream (log-uniform 10^4-10^6 records, spread
    over all resources in proportion) and closes the region
    [previous close, new frontier). With device-resident payloads latency and
    throughput measure the serving runtime and kernels; the runs at
    `host_lambdas` hand the same slices over from host memory (copied at
    submission, staged through pinned memory), so they include PCIe.
    """
    W = serving_workload(n_queries, seed, n_sessions, ranks, streams, warm)
    results = []
    for lam, host in [(l, False) for l in lambdas] + [(l, True) for l in host_lambdas]:
        results.append(serving_run(hp, W, lam, host))
        log("serving lambda=%d %s: %s" % (lam, "host" if host else "device", results[-1]))
    return {"sessions": n_sessions, "ranks": ranks, "devices": ranks, "streams": streams,
            "warm_events_per_session": warm, "list_heap_bytes": SERVING_LIST_HEAP,
            "payload": "device-resident, or host memory (copied at submission) where a run says so",
            "latency": "scheduled arrival to trees on the host",
            "runs": results}


def cpu_model():
    """The host CPU's model name and logical CPU count (Linux)."""
    name = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": name, "logical_cpus": os.cpu_count()}


def timed_median(fn, reps=5):
    """One untimed warm-up call, then the median wall time of `reps` calls."""
    fn()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def oracle_threads():
    """The oracle's threads: the host's CPUs, at most 16 (one GPU's share of its host)."""
    return max(1, min(16, os.cpu_count() or 1))


def cpu_baseline(trace, target_s=2.5, target_1_s=1.5):
    """Oracle on a bounded sample: a subset of the resources, all regions; one
    warm-up and the median of 5 runs, with the host's threads and on one thread."""
    import oracle
    import tracegen as tg
    threads = oracle_threads()
    n, m = trace.n_hosts, trace.n_devices

    def subset(k):
        hosts = list(range(min(n, k)))
        devs = list(range(n, n + min(m, k)))
        keep = set(hosts + devs)
        remap = {r: i for i, r in enumerate(hosts)}
        remap.update({r: len(hosts) + i for i, r in enumerate(devs)})
        chunks = [tg.Chunk(remap[c.resource], c.kind, c.start, c.end) for c in trace.chunks if c.resource in keep]
        return tg.Trace(len(hosts), len(devs), chunks, trace.regions)

    def sized(k, thr, target):
        # grow the sample until one run takes about `target` seconds
        sub = subset(k)
        t0 = time.perf_counter()
        oracle.compute(sub, threads=thr)
        dt = time.perf_counter() - t0
        while dt < target / 2 and k < max(n, m):
            k = min(max(n, m), k * 2)
            sub = subset(k)
            t0 = time.perf_counter()
            oracle.compute(sub, threads=thr)
            dt = time.perf_counter() - t0
        return sub

    sub = sized(max(1, min(n, m, threads)), threads, target_s)
    dt = timed_median(lambda: oracle.compute(sub, threads=threads))
    sub1 = sized(1, 1, target_1_s)
    dt1 = timed_median(lambda: oracle.compute(sub1, threads=1))
    return {"value": sub.n_events / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(), "timing": "1 warm-up, median of 5",
            "sample": "%d host ranks + %d devices of the workload (%d records), all %d regions, %.2f s per run"
                      % (sub.n_hosts, sub.n_devices, sub.n_events, len(trace.regions), dt),
            "single_thread": {"value": sub1.n_events / dt1, "unit": "events/s", "cores": 1,
                              "sample": "%d host ranks + %d devices (%d records), all %d regions, %.2f s per run"
                                        % (sub1.n_hosts, sub1.n_devices, sub1.n_events, len(trace.regions), dt1)}}


CALIB_BYTES = 1 << 30  # plain copy of 1 GiB: reads 1 GiB, writes 1 GiB


def timed_copy(reps=5):
    """ms per plain device copy of CALIB_BYTES (reads and writes that many bytes)."""
    import torch
    a = torch.ones(CALIB_BYTES // 8, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.copy_(a)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del a, b
    torch.cuda.empty_cache()
    return ms


def calibrate_copy(reps=5):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    ms = timed_copy(reps)
    print(json.dumps({"calibration_copy_bytes": CALIB_BYTES, "reps": reps, "ms_per_copy": round(ms, 4),
                      "read_plus_write_GBs": round(2 * CALIB_BYTES / (ms * 1e-3) / 1e9, 1)}))


def _pmc_rows(path, counter):
    """(kernel name, value) per dispatch from a rocprofv3 counter_collection.csv."""
    import csv
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") == counter:
                rows.append((r.get("Kernel_Name", ""), float(r["Counter_Value"])))
    return rows


def import_traffic(kernel, workload, fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, out_dir):
    """HBM bytes per launch of `kernel` from two counter runs, each scaled by the
    same counter's reading for the calibration copy (FETCH_SIZE and WRITE_SIZE
    are in KiB per dispatch)."""
    def mean_for(rows, name):
        v = [x for k, x in rows if name in k]
        return sum(v) / len(v) if v else None
    cal_f = max((x for k, x in _pmc_rows(cal_fetch_csv, "FETCH_SIZE") if "copy" in k.lower() or "elementwise" in k.lower()),
                default=None)
    cal_w = max((x for k, x in _pmc_rows(cal_write_csv, "WRITE_SIZE") if "copy" in k.lower() or "elementwise" in k.lower()),
                default=None)
    f = mean_for(_pmc_rows(fetch_csv, "FETCH_SIZE"), kernel)
    w = mean_for(_pmc_rows(write_csv, "WRITE_SIZE"), kernel)
    if None in (cal_f, cal_w, f, w):
        raise SystemExit("missing counter rows (%s %s %s %s)" % (cal_f, cal_w, f, w))
    sf = (CALIB_BYTES / 1024.0) / cal_f
    sw = (CALIB_BYTES / 1024.0) / cal_w
    rec = {"kernel": kernel, "workload": workload, "source_hash": kernel_source_hash(),
           "fetch_kib_per_launch": f, "write_kib_per_launch": w,
           "calibration_fetch_kib": cal_f, "calibration_write_kib": cal_w,
           "fetch_scale": sf, "write_scale": sw,
           "bytes_per_launch": int(f * 1024 * sf + w * 1024 * sw)}
    path = os.path.join(out_dir, "traffic_%s_%s.txt" % (kernel.replace("k_", ""), workload))
    with open(path, "w") as fo:
        fo.write("# HBM traffic of %s on the %s workload, from rocprofv3 FETCH_SIZE and WRITE_SIZE\n" % (kernel, workload))
        fo.write("# (KiB per dispatch), each scaled by the same counter's reading for a plain 1 GiB copy\n")
        for k, v in rec.items():
            fo.write("%s: %s\n" % (k, v))
    print(path, rec)
    # every build kernel of the same runs: the whole path's bytes per step
    fr, wr = _pmc_rows(fetch_csv, "FETCH_SIZE"), _pmc_rows(write_csv, "WRITE_SIZE")
    names = sorted({k.split("(")[0] for k, _ in fr if "hpop::k_" in k})
    per = {}
    for n in names:
        fm, wm = mean_for(fr, n + "("), mean_for(wr, n + "(")
        per[n] = int((fm or 0) * 1024 * sf + (wm or 0) * 1024 * sw)
    path = os.path.join(out_dir, "traffic_path_%s.txt" % workload)
    with open(path, "w") as fo:
        fo.write("# HBM traffic of every build kernel on the %s workload (bytes per launch; each kernel\n" % workload)
        fo.write("# runs once per build), from the same FETCH_SIZE and WRITE_SIZE runs and scales\n")
        fo.write("workload: %s\nsource_hash: %s\n" % (workload, kernel_source_hash()))
        for n, v in per.items():
            fo.write("kernel %s: %d\n" % (n, v))
        fo.write("bytes_per_step: %d\n" % sum(per.values()))
    print(path, sum(per.values()))


def load_path_traffic(workload):
    """Counter-measured HBM bytes of one build (all build kernels), if taken on
    the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic_path_%s.txt" % workload)
    if not os.path.exists(p):
        return None
    d = {}
    for line in open(p):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            d[k.strip()] = v.strip()
    if d.get("source_hash") != kernel_source_hash():
        return None
    try:
        return int(d["bytes_per_step"])
    except (KeyError, ValueError):
        return None


def path_hbm(r, workload):
    """Whole-path HBM figures of the single-trace leg: counter-measured bytes of a
    build over the sum of the kernels' stage times, against the chip's peak and
    a plain copy on the same GPU; and the algorithmic fraction (16 B per record
    at the measured record rate)."""
    kernel_ms = sum(r["stage_ms"].values())
    copy_ms = timed_copy()
    copy_gbs = 2 * CALIB_BYTES / (copy_ms * 1e-3) / 1e9
    b = load_path_traffic(workload)
    out = {"kernel_ms_per_step": round(kernel_ms, 4), "peak_GBps": HBM_PEAK_GBS,
           "plain_copy_GBps": round(copy_gbs, 1),
           "algorithmic_bytes_per_record": ALGO_BYTES_PER_RECORD,
           "algorithmic_frac": round(ALGO_BYTES_PER_RECORD * r["value"] / (HBM_PEAK_GBS * 1e9), 4),
           "counter_bytes_per_step": b, "achieved_GBps": None, "frac": None, "frac_of_plain_copy": None}
    if b is not None:
        ach = b / (kernel_ms * 1e-3) / 1e9
        out.update({"achieved_GBps": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                    "frac_of_plain_copy": round(ach / copy_gbs, 4)})
    return out


def run_collect_app(iters, live_every, prefix, with_tool):
    from paper_2603_26576_amd import collect
    env = collect.tool_env() if with_tool else dict(os.environ, HPOP_APP_ALLOW_INACTIVE="1")
    if not with_tool:
        env.pop("ROCP_TOOL_LIBRARIES", None)
    r = subprocess.run([COLLECT_APP, str(iters), str(live_every), prefix], env=env, capture_output=True, text=True,
                       timeout=300)
    if r.returncode != 0:
        raise RuntimeError("collect_app failed (%d): %s" % (r.returncode, r.stderr[-1000:]))
    line = [l for l in r.stdout.splitlines() if l.startswith("collect_app ")][-1]
    return {k: float(v) for k, v in (kv.split("=") for kv in line.split()[1:])}


def collector_leg(hp, iters=400, live_every=20):
    """The live collector on its test application (a real HIP program): the
    tracing cost per runtime call and per iteration (with the tool against
    without it), and the latency of each live region (poll, copy, submit to
    an in-process hpop server, wait for its trees)."""
    if not os.path.exists(COLLECT_APP):
        return {"skipped": "tests/apps/collect_app is not built"}
    tmp = tempfile.mkdtemp(prefix="hpop_collect_")
    try:
        base = run_collect_app(iters, 0, os.path.join(tmp, "plain"), False)
        traced = run_collect_app(iters, 0, os.path.join(tmp, "traced"), True)
        live = run_collect_app(iters, live_every, os.path.join(tmp, "live"), True)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return {"app": "tests/apps/collect_app: per iteration 150 us of host work, 2 copies of 4 MiB, a 1 MiB fill, "
                   "2 kernels on 2 streams, a device synchronisation",
            "iters": iters, "call_ns_without_tool": base["call_ns"], "call_ns_traced": traced["call_ns"],
            "iter_us_without_tool": base["iter_us"], "iter_us_traced": traced["iter_us"],
            "iter_us_live": live["iter_us"], "live_regions": int(live["regions"]),
            "live_every_iters": live_every, "live_records_per_region": round(live["live_records"] / max(1, live["regions"]), 1),
            "live_p50_us": live["live_p50_us"], "live_max_us": live["live_max_us"],
            "live_poll_p50_us": live["live_poll_p50_us"],
            "dropped": int(traced["dropped"] + live["dropped"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["large", "mid", "small"])
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the workload's records (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-traces", type=int, default=1000)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-only", action="store_true", help="profiling aid: run only the serving leg")
    ap.add_argument("--serving-queries", type=int, default=2000)
    ap.add_argument("--serving-lambdas", default="2000,5000,10000,20000")
    ap.add_argument("--serving-host-lambdas", default="2000,5000,10000,20000",
                    help="runs with payloads in host memory (0: none)")
    ap.add_argument("--no-small", action="store_true", help="skip the small-trace latency leg")
    ap.add_argument("--no-mid", action="store_true", help="skip the mid-trace leg")
    ap.add_argument("--no-entered", action="store_true", help="skip the regions-entered-repeatedly leg")
    ap.add_argument("--no-streams", action="store_true")
    ap.add_argument("--streams-only", action="store_true", help="run only the stream concurrency leg")
    ap.add_argument("--no-collector", action="store_true")
    ap.add_argument("--collector-only", action="store_true", help="run only the collector leg")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (JSON)")
    ap.add_argument("--trace-cache", default=None, help="npz file to reuse the generated workload")
    ap.add_argument("--calibrate-copy", action="store_true", help="only run the plain copy used to scale counters")
    ap.add_argument("--import-traffic", nargs=6, metavar=("KERNEL", "WORKLOAD", "FETCH_CSV", "WRITE_CSV",
                                                          "CAL_FETCH_CSV", "CAL_WRITE_CSV"))
    args = ap.parse_args()
    if args.import_traffic:
        import_traffic(*args.import_traffic, out_dir=os.path.join(ROOT, "profiles"))
        return
    if args.gpus != 1:
        print("this engine runs on one GPU; the per-resource sharding across GPUs is a design note only "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2603_26576_amd as hp
    import tracegen as tg
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        calibrate_copy()
        return
    hp.lib()

    if args.streams_only:
        print(json.dumps({"streams": streams_leg(hp, args.steps, args.warmup)}), flush=True)
        return
    if args.collector_only:
        print(json.dumps({"collector": collector_leg(None)}), flush=True)
        return
    if args.serving_only:
        lams = [int(x) for x in args.serving_lambdas.split(",") if x]
        host_lams = [int(x) for x in args.serving_host_lambdas.split(",") if x and int(x) > 0]
        print(json.dumps({"serving": serving_leg(hp, lams, args.serving_queries, host_lambdas=host_lams)}), flush=True)
        return
    log("generating workload %s (scale %g)" % (args.workload, args.scale))
    t = time.time()
    if args.workload == "large":
        trace = load_trace_cache(args.trace_cache, tg) if args.trace_cache else None
        if trace is None:
            trace = tg.large(scale=args.scale)
            if args.trace_cache:
                save_trace_cache(args.trace_cache, trace)
        cfg = {"workload": "large imbalance sweep", "ranks": 256, "devices": 256, "streams": 4, "regions": 64,
               "device_events": 10 ** 8, "host_events": 25 * 10 ** 6}
    elif args.workload == "mid":
        trace = tg.mid(scale=args.scale)
        cfg = {"workload": "mid trace", "ranks": 64, "devices": 64, "streams": 8, "regions": 16}
    else:
        trace = tg.small()
        cfg = {"workload": "small trace", "ranks": 4, "devices": 4, "streams": 2, "regions": 1}
    cfg["events"] = trace.n_events
    cfg["overlap_fraction"] = round(trace.info["overlap_fraction"], 4)
    log("generated %d records in %.1f s" % (trace.n_events, time.time() - t))

    log("single-trace leg: %d warmup + %d timed steps" % (args.warmup, args.steps))
    r = bench_single(hp, trace, args.steps, args.warmup, args.workload, args.tune_cache)
    log("single-trace: %.3f ms/step, %.3e events/s, stages %s" % (r["ms_per_step"], r["value"],
                                                                  {k: round(v, 3) for k, v in r["stage_ms"].items()}))
    out = {"metric": METRIC, "value": r["value"], "unit": "events/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic", "config": cfg,
           "roofline": r["roofline"],
           "stage_ms": {k: round(v, 4) for k, v in r["stage_ms"].items()},
           "graph_replay": {"ms_per_step": round(r["ms_per_step_graph"], 4), "events_per_s": r["value_graph"]},
           "components": r["components"], "wide_components": r["wide_components"],
           "wide_records": r["wide_records"], "buckets": r["buckets"],
           "oversized_buckets": r["oversized_buckets"],
           "tuning": r["tuning"]}
    out["path_hbm"] = path_hbm(r, args.workload)
    log("path HBM: %s" % out["path_hbm"])
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a sample)")
        out["cpu_baseline"] = cpu_baseline(trace)
        log("cpu baseline: %s" % out["cpu_baseline"])
    if not args.no_small:
        log("small-trace leg")
        out["small"] = small_leg(hp)
        log("small: %s" % out["small"])
    if not args.no_mid:
        log("mid-trace leg")
        out["mid"] = mid_leg(hp, args.steps, args.warmup, args.tune_cache)
        log("mid: %s" % {k: v for k, v in out["mid"].items() if k != "stage_ms"})
    if not args.no_entered:
        log("regions entered repeatedly")
        out["entered_regions"] = entered_regions_leg(hp, trace)
        log("entered regions: %s" % out["entered_regions"])
    del trace
    if not args.no_batched and args.batched_traces > 0:
        log("batched leg: generating %d traces" % args.batched_traces)
        t = time.time()
        traces = tg.batched(n_traces=args.batched_traces)
        log("generated %d records in %.1f s" % (sum(x.n_events for x in traces), time.time() - t))
        out["batched"] = bench_batched(hp, traces, max(3, args.steps // 2), 1, args.tune_cache)
        log("batched: %s" % out["batched"])
    if not args.no_serving and args.serving_queries > 0:
        lams = [int(x) for x in args.serving_lambdas.split(",") if x]
        host_lams = [int(x) for x in args.serving_host_lambdas.split(",") if x and int(x) > 0]
        log("serving leg: lambdas %s, %d queries each" % (lams, args.serving_queries))
        out["serving"] = serving_leg(hp, lams, args.serving_queries, host_lambdas=host_lams)
    if not args.no_streams:
        log("stream concurrency leg")
        out["streams"] = streams_leg(hp, args.steps, args.warmup)
        log("streams: %s" % out["streams"])
    if not args.no_collector:
        log("collector leg")
        out["collector"] = collector_leg(hp)
        log("collector: %s" % out["collector"])
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
