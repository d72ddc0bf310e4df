"""The collector library in a process without a GPU runtime, and its trace
file format (CPU only). The reader is also checked on files laid out by hand
from the format that include/hpop_collect.h documents."""
import ctypes
import os
import struct
import subprocess
import sys
import time

import numpy as np
import pytest

import paper_2603_26576_amd as hp
from paper_2603_26576_amd import collect

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _without_gpu_runtime(out_dir):
    """Run in a fresh interpreter: the tool is loaded first, then the HIP
    runtime library (through libhpop), which hands rocprofiler-sdk the tool's
    configuration entry. With no GPU agent and no HIP call, the only records
    are the Useful gaps the polls make final: they tile [begin, last frontier)."""
    import os
    a = collect.hpop_collect_now()
    assert 0 < a <= collect.hpop_collect_now()  # rocprofiler's clock, configured or not
    assert collect.hpop_collect_active() == 0
    # raw status codes: the binding's error message would load libhpop, and with it the HIP runtime
    L = collect.collect_lib()
    f = ctypes.c_int64(0)
    assert L.hpop_collect_poll(ctypes.byref(f)) == hp.HPOP_E_STATE
    assert L.hpop_collect_flush() == hp.HPOP_E_STATE
    assert collect.hpop_collect_active() == 0
    hp.lib()  # loads the HIP runtime library
    t = time.time() + 10
    while not collect.hpop_collect_active() and time.time() < t:
        time.sleep(0.01)
    assert collect.hpop_collect_active() == 1
    assert collect.hpop_collect_devices() == 0
    collect.hpop_collect_flush()  # no GPU agent: nothing to deliver
    b = collect.hpop_collect_begin()
    assert b > 0
    f1 = collect.hpop_collect_poll()
    time.sleep(0.01)
    f2 = collect.hpop_collect_poll()
    assert b <= f1 < f2
    n = collect.hpop_collect_count(0, hp.HPOP_HOST_USEFUL)
    assert n >= 2
    s, e = collect.hpop_collect_copy(0, hp.HPOP_HOST_USEFUL, 0, n)
    assert s[0] == b and e[-1] == f2
    assert np.all(s <= e) and np.all(s[1:] == e[:-1])
    assert f1 in e
    for k in (hp.HPOP_HOST_OFFLOAD, hp.HPOP_HOST_MPI):
        assert collect.hpop_collect_count(0, k) == 0
    assert collect.hpop_collect_count(1, hp.HPOP_DEV_KERNEL) == 0  # no such resource
    assert L.hpop_collect_copy(1, hp.HPOP_DEV_KERNEL, 0, 0, None, None) == hp.HPOP_E_RESOURCE
    assert L.hpop_collect_copy(0, hp.HPOP_DEV_KERNEL, 0, 0, None, None) == hp.HPOP_E_KIND
    assert L.hpop_collect_copy(0, hp.HPOP_HOST_USEFUL, n, 1, s.ctypes.data, e.ctypes.data) == hp.HPOP_E_REGION
    # the C writer and the Python reader agree on the file format
    path = os.path.join(out_dir, "self.trace")
    collect.hpop_collect_write(path)
    t = collect.read_trace(path)
    assert (t["n_hosts"], t["n_devices"], t["t_begin"]) == (1, 0, b)
    assert t["t_end"] >= f2
    assert [(r, k) for r, k, _, _ in t["chunks"]] == [(0, hp.HPOP_HOST_USEFUL)]
    s3, e3 = t["chunks"][0][2], t["chunks"][0][3]
    np.testing.assert_array_equal(s3[:n], s)
    np.testing.assert_array_equal(e3[:n], e)
    assert e3[-1] == t["t_end"]
    with pytest.raises(hp.HpopError) as err:
        collect.hpop_collect_write(os.path.join(out_dir, "no", "such", "dir.trace"))
    assert err.value.status == hp.HPOP_E_ARG
    print("child ok", n)


def _threads_and_polls(out_dir):
    """Run in a fresh interpreter: four threads make HIP runtime calls (traced
    even with no GPU: each returns an error) while this thread polls. Every
    Useful gap must be disjoint from every offload call, and gaps plus calls
    must cover [begin, last frontier) exactly: a gap may never be made final
    over a call that was still running when the poll took its frontier."""
    import ctypes
    import threading
    collect.collect_lib()  # the tool first: the HIP runtime configures it when it starts
    hip = ctypes.CDLL("libamdhip64.so")
    n = ctypes.c_int(0)
    hip.hipGetDeviceCount(ctypes.byref(n))  # starts the runtime, which configures the tool
    t = time.time() + 10
    while not collect.hpop_collect_active() and time.time() < t:
        time.sleep(0.01)
    assert collect.hpop_collect_active() == 1
    stop = threading.Event()

    def worker():
        m = ctypes.c_int(0)
        while not stop.is_set():
            for _ in range(50):
                hip.hipGetDeviceCount(ctypes.byref(m))
            time.sleep(0.0002)

    ths = [threading.Thread(target=worker) for _ in range(4)]
    for th in ths:
        th.start()
    frontiers = []
    t_end = time.time() + 0.5
    while time.time() < t_end:  # half a second of polls, as often as possible
        frontiers.append(collect.hpop_collect_poll())
    stop.set()
    for th in ths:
        th.join()
    last = collect.hpop_collect_poll()
    frontiers.append(last)
    assert all(a <= b for a, b in zip(frontiers, frontiers[1:]))
    b = collect.hpop_collect_begin()
    nu = collect.hpop_collect_count(0, hp.HPOP_HOST_USEFUL)
    nw = collect.hpop_collect_count(0, hp.HPOP_HOST_OFFLOAD)
    us, ue = collect.hpop_collect_copy(0, hp.HPOP_HOST_USEFUL, 0, nu)
    ws, we = collect.hpop_collect_copy(0, hp.HPOP_HOST_OFFLOAD, 0, nw)
    assert nw > 1000 and nu > 10, (nw, nu)
    assert np.all(us < ue) and np.all(ws <= we)
    # the gaps are made final in time order and never overlap each other
    assert np.all(us[1:] >= ue[:-1])
    # union of the offload calls, clipped to [b, last)
    o = np.argsort(ws, kind="stable")
    cs, ce = [], []
    for a0, a1 in zip(ws[o], we[o]):
        a0, a1 = max(int(a0), b), min(int(a1), last)
        if a0 >= a1:
            continue
        if cs and a0 <= ce[-1]:
            ce[-1] = max(ce[-1], a1)
        else:
            cs.append(a0)
            ce.append(a1)
    cs, ce = np.array(cs, np.int64), np.array(ce, np.int64)
    # no gap overlaps a call: a gap [u0, u1) meets the union iff some call starts before u1 and ends after u0
    k = np.searchsorted(cs, ue, side="left")  # calls starting before each gap's end
    prev_end = np.where(k > 0, ce[np.maximum(k - 1, 0)], np.iinfo(np.int64).min)
    assert np.all(prev_end <= us), "a Useful gap overlaps an offload call"
    # gaps and calls tile [b, last)
    covered = int((ue - us).sum()) + int((ce - cs).sum())
    assert covered == last - b, (covered, last - b)
    print("child ok", nu, nw)


def test_concurrent_calls_and_polls(tmp_path):
    env = dict(os.environ)
    env["PYTHONPATH"] = os.pathsep.join([ROOT] + [p for p in env.get("PYTHONPATH", "").split(os.pathsep) if p])
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "threads", str(tmp_path)], capture_output=True,
                       text=True, timeout=180, cwd=ROOT, env=env)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert "child ok" in r.stdout


def test_without_gpu_runtime(tmp_path):
    env = dict(os.environ)
    env["PYTHONPATH"] = os.pathsep.join([ROOT] + [p for p in env.get("PYTHONPATH", "").split(os.pathsep) if p])
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "single", str(tmp_path)], capture_output=True,
                       text=True, timeout=120, cwd=ROOT, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "child ok" in r.stdout


def test_tool_configured_before_its_constructors(tmp_path):
    """Regression: a library initialised before the tool starts the HIP
    runtime, so rocprofiler-sdk configures the tool before the tool library's
    static constructors run. The state must still be valid, every call
    recorded, and the exit clean (this once ended in a segmentation fault)."""
    apps = os.path.join(ROOT, "tests", "apps")
    inc = ["-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include"]
    early = str(tmp_path / "libcollect_early.so")
    main = str(tmp_path / "collect_early")
    subprocess.run(["g++", "-std=c++17", "-fPIC", "-shared"] + inc + [os.path.join(apps, "collect_early_lib.cpp"),
                    "-o", early, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    pkg = os.path.dirname(collect.COLLECT_LIB_PATH)
    subprocess.run(["g++", "-std=c++17"] + inc + [os.path.join(apps, "collect_early_main.cpp"), "-o", main,
                    "-Wl,--no-as-needed", "-L" + str(tmp_path), "-lcollect_early", "-L" + pkg, "-lhpop_collect",
                    "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath," + pkg,
                    "-Wl,-rpath,/opt/rocm/lib"], check=True)
    r = subprocess.run([main], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr[-2000:])
    assert "HIP started from a constructor" in r.stderr
    assert "active=1 poll=0" in r.stdout


def test_bad_arguments_rejected_first():
    L = collect.collect_lib()
    assert L.hpop_collect_poll(None) == hp.HPOP_E_ARG
    assert L.hpop_collect_copy(0, 1, -1, 0, None, None) == hp.HPOP_E_ARG
    assert L.hpop_collect_copy(0, 1, 0, 2, None, None) == hp.HPOP_E_ARG
    assert L.hpop_collect_write(None) == hp.HPOP_E_ARG


def test_tool_env():
    env = collect.tool_env("/tmp/t_%p.trace", base={"PATH": "/bin"})
    assert env["ROCP_TOOL_LIBRARIES"] == collect.COLLECT_LIB_PATH
    assert env["HPOP_COLLECT_OUT"] == "/tmp/t_%p.trace"
    assert env["PATH"] == "/bin"
    assert "HPOP_COLLECT_OUT" not in collect.tool_env(base={})


def write_by_hand(path, n_devices, t_begin, t_end, chunks):
    with open(path, "wb") as f:
        f.write(b"HPOPTRC1")
        f.write(struct.pack("<ii", 1, n_devices))
        f.write(struct.pack("<qq", t_begin, t_end))
        f.write(struct.pack("<i", len(chunks)))
        for r, k, s, e in chunks:
            f.write(struct.pack("<iiq", r, k, len(s)))
            f.write(struct.pack("<%dq" % len(s), *s))
            f.write(struct.pack("<%dq" % len(e), *e))


def test_read_trace(tmp_path):
    chunks = [(0, hp.HPOP_HOST_USEFUL, [10, 40], [20, 50]), (0, hp.HPOP_HOST_OFFLOAD, [20], [40]),
              (1, hp.HPOP_DEV_KERNEL, [25, 26, 1 << 61], [30, 35, (1 << 61) + 7]), (2, hp.HPOP_DEV_MEMOP, [], [])]
    p = tmp_path / "a.trace"
    write_by_hand(p, 2, 10, 50, chunks)
    t = collect.read_trace(p)
    assert (t["n_hosts"], t["n_devices"], t["t_begin"], t["t_end"]) == (1, 2, 10, 50)
    assert len(t["chunks"]) == len(chunks)
    for (r, k, s, e), (r2, k2, s2, e2) in zip(chunks, t["chunks"]):
        assert (r, k) == (r2, k2)
        assert s2.dtype == np.int64 and e2.dtype == np.int64
        np.testing.assert_array_equal(s2, np.array(s, np.int64))
        np.testing.assert_array_equal(e2, np.array(e, np.int64))


def test_read_trace_rejects_damage(tmp_path):
    p = tmp_path / "b.trace"
    write_by_hand(p, 1, 0, 5, [(1, hp.HPOP_DEV_KERNEL, [1, 2], [3, 4])])
    raw = p.read_bytes()
    (tmp_path / "bad_magic").write_bytes(b"XPOPTRC1" + raw[8:])
    with pytest.raises(ValueError):
        collect.read_trace(tmp_path / "bad_magic")
    (tmp_path / "trailing").write_bytes(raw + b"\0")
    with pytest.raises(ValueError):
        collect.read_trace(tmp_path / "trailing")
    (tmp_path / "short").write_bytes(raw[:-8])
    with pytest.raises(ValueError):
        collect.read_trace(tmp_path / "short")


if __name__ == "__main__":
    if sys.argv[1] == "threads":
        _threads_and_polls(sys.argv[2])
    else:
        _without_gpu_runtime(sys.argv[2])
