"""Host-side pieces of bench.py, CPU only: the one-GPU refusal, the oracle
baseline object, the traffic records' source check, and the synthetic
workloads of the regions-entered and stream legs (their shape is what the
oracle and the engine assume)."""
import os
import shutil
import subprocess
import sys
import time

import numpy as np

import bench
import tracegen as tg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


def test_cpu_baseline_object():
    tr = tg.small()
    out = bench.cpu_baseline(tr, target_s=0.3, target_1_s=0.1)
    assert out["kind"] == "oracle" and out["unit"] == "events/s"
    assert out["cores"] >= 1 and out["value"] > 0 and isinstance(out["sample"], str)
    assert out["timing"] == "1 warm-up, median of 5"
    assert out["cpu"]["logical_cpus"] == os.cpu_count() and out["cpu"]["model"]
    one = out["single_thread"]
    assert one["cores"] == 1 and one["value"] > 0


def test_timed_median_warms_up_then_takes_the_median():
    calls = []

    def fn():
        calls.append(time.perf_counter())
        time.sleep(0.02 if len(calls) == 1 else 0.001)  # a slow first (warm-up) call

    dt = bench.timed_median(fn, reps=5)
    assert len(calls) == 6 and dt < 0.015


def test_traffic_records_are_tied_to_the_kernel_sources(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    for b in (bench.load_traffic("merge_wave", "large"), bench.load_path_traffic("large")):
        assert b is None or b > 0
    # a record taken on other sources is not used
    prof = tmp_path / "profiles"
    prof.mkdir()
    shutil.copy(os.path.join(ROOT, "profiles", "traffic_merge_wave_large.txt"), prof)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("merge_wave", "large") is None
    assert bench.load_traffic("merge_wave", "absent") is None


def test_entered_regions_are_disjoint_per_resource():
    tr = tg.make_trace(5, 3, 2, 2, 2000, 500, regions="tiles", n_regions=2)
    R = tr.n_hosts + tr.n_devices
    regions = bench.entered_regions(tr, n_regions=4, entries=8)
    assert len(regions) == 4
    lo, hi = tr.info["t0"], tr.info["t_end"]
    for ivls in regions:
        assert len(ivls) == 8 * R
        per = {}
        for r, a, b in ivls:
            assert 0 <= r < R and lo <= a < b <= hi
            per.setdefault(r, []).append((a, b))
        for lst in per.values():
            lst.sort()
            assert all(b0 <= a1 for (_, b0), (a1, _) in zip(lst, lst[1:]))


def test_streams_workload_tiles_its_span():
    n_streams, chunks, regions = bench.streams_workload(n_devices=3, streams=2, per_device=500, n_regions=5)
    assert n_streams == [2, 2, 2]
    lo = min(int(c[2].min()) for c in chunks)
    hi = max(int(c[3].max()) for c in chunks)
    assert regions[0] == (lo, hi) and len(regions) == 5
    tiles = np.array(regions[1:])
    assert tiles[0, 0] == lo and tiles[-1, 1] == hi and (tiles[1:, 0] == tiles[:-1, 1]).all()
    for g, k, s, e in chunks:
        assert 0 <= g < 3 and 0 <= k < 2 and (s <= e).all()


def test_serving_slices_are_consecutive_prefixes():
    """The serving workload's queries take consecutive slices of each session's
    chunks, and the oracle's input for a query is exactly the prefix its
    session had received up to it (with the query's region and the global one)."""
    import paper_2603_26576_amd as hp
    W = bench.serving_workload(12, n_sessions=3, ranks=2, streams=2, warm=3000, device=False)
    assert W["sizes"].size == 12 and ((W["sizes"] >= 10 ** 4) & (W["sizes"] <= 10 ** 6)).all()
    cursors = [[0] * len(S["chunks"]) for S in W["sess"]]
    closes = [S["origin"] for S in W["sess"]]
    for q in [None] * 3 + list(range(12)):
        i = int(W["owner"][q]) if q is not None else sum(1 for c in closes if c != W["sess"][0]["origin"]) % 3
        before = list(cursors[i])
        arr, k, fr = bench.serving_slices(hp, W, i, 3000 if q is None else int(W["sizes"][q]), cursors[i], True)
        S = W["sess"][i]
        j = 0
        for c, (r, kind, _, _, pmax, hst, hen) in enumerate(S["chunks"]):
            assert before[c] <= cursors[i][c] <= hst.size
            if cursors[i][c] > before[c]:
                got = arr[j]
                assert (got.resource, got.kind, got.count) == (r, kind, cursors[i][c] - before[c])
                assert got.start == hst.ctypes.data + 8 * before[c] and got.end == hen.ctypes.data + 8 * before[c]
                assert fr >= int(hen[:cursors[i][c]].max())
                j += 1
        assert j == k
        t1 = max(fr, closes[i] + 1)
        tr = bench.serving_expected_trace(W, (i, closes[i], t1, list(cursors[i])))
        assert tr.regions[0] == (closes[i], t1) and tr.regions[1][0] == S["origin"]
        want_n = sum(cursors[i])
        assert tr.n_events == want_n
        if want_n:
            assert tr.regions[1][1] == max(int(c.end.max()) for c in tr.chunks)
        closes[i] = t1


def test_traffic_of_any_build_kernel_from_the_path_record(tmp_path, monkeypatch):
    """A kernel without a record of its own takes its line of the record of
    every build kernel (template arguments in the name; k_stats is not
    k_stats_small)."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_path_w.txt").write_text(
        "# test\nworkload: w\nsource_hash: abcd\n"
        "kernel hpop::k_merge_wave: 100\n"
        "kernel void hpop::k_scatter<512, 4, false>: 300\n"
        "kernel void hpop::k_stats<256, false>: 50\n"
        "kernel void hpop::k_stats_small<true>: 7\n"
        "bytes_per_step: 457\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abcd")
    assert bench.load_traffic("scatter", "w") == 300
    assert bench.load_traffic("merge_wave", "w") == 100
    assert bench.load_traffic("stats", "w") == 50
    assert bench.load_traffic("region_part", "w") is None
    assert bench.load_path_traffic("w") == 457
    # a kernel templated on a flag (the merge with fixed slots) and a fused one
    (prof / "traffic_path_w.txt").write_text(
        "# test\nworkload: w\nsource_hash: abcd\n"
        "kernel void hpop::k_merge_wave<true>: 120\n"
        "kernel void hpop::k_scan_carry<false>: 9\n"
        "bytes_per_step: 129\n")
    assert bench.load_traffic("merge_wave", "w") == 120
    assert bench.load_traffic("scan", "w") is None
    assert bench.load_traffic("scan_carry", "w") == 9
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "ffff")
    assert bench.load_traffic("scatter", "w") is None
