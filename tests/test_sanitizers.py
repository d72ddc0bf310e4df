"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* the C oracle, rebuilt with both sanitizers into a stand-alone driver, must
  still pass its pins (the per-nanosecond brute force on random tiny traces,
  the PILS tables of Sec. 5.1), agree bit for bit with the normal build on a
  generated trace with threads, and reject bad input with its error codes;
* the autotuner's cache reader must read what the writer's format allows and
  reject truncated, garbled or out-of-range files with a clean error;
* the tree renderings (hpop_tree_format and the region report) must write
  within every buffer size, for trees holding extreme values.

A sanitizer report makes the driver exit non-zero (no recovery), which fails
the test.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle
import pils
import tracegen as tg
from brute import occupancy_times, tree_from_times

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2603_26576_amd", "csrc")
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")


def _build(tmp, name, cmd):
    exe = os.path.join(str(tmp), name)
    r = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        if "sanitizer" in (r.stderr + r.stdout).lower() and "cannot find" in (r.stderr + r.stdout).lower():
            pytest.skip("sanitizer runtime not installed")
        raise AssertionError(r.stderr + r.stdout)
    return exe


def _run(args):
    r = subprocess.run(args, capture_output=True, text=True, env=ENV, timeout=120)
    assert r.returncode == 0, "exit %d\n%s%s" % (r.returncode, r.stdout, r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.fixture(scope="module")
def oracle_exe(tmp_path_factory):
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    tmp = tmp_path_factory.mktemp("san_oracle")
    return _build(tmp, "oracle_san", ["gcc", "-std=c11"] + SAN + ["-I", os.path.join(ROOT, "oracle"),
                                                                  os.path.join(ROOT, "oracle", "hpop_oracle.c"),
                                                                  os.path.join(NATIVE, "oracle_main.c"),
                                                                  "-lpthread"])


def run_oracle(exe, tmp, n, m, res, kind, s, e, regions, threads=1):
    inp, out = os.path.join(str(tmp), "in.bin"), os.path.join(str(tmp), "out.bin")
    with open(inp, "wb") as f:
        f.write(struct.pack("<iiq", n, m, len(s)))
        f.write(np.asarray(res, "<i4").tobytes() + np.asarray(kind, "<i4").tobytes())
        f.write(np.asarray(s, "<i8").tobytes() + np.asarray(e, "<i8").tobytes())
        f.write(struct.pack("<i", len(regions)))
        f.write(np.array([r[0] for r in regions], "<i8").tobytes() + np.array([r[1] for r in regions], "<i8").tobytes())
        f.write(struct.pack("<i", threads))
    _run([exe, inp, out])
    raw = open(out, "rb").read()
    rc = struct.unpack_from("<i", raw)[0]
    if rc != 0:
        return rc, None
    G, R = len(regions), n + m
    o = 4
    times = np.frombuffer(raw, "<i8", G * R * 4, o).reshape(G, R, 4)
    o += 8 * G * R * 4
    sums = np.frombuffer(raw, "<i8", G * 10, o).reshape(G, 10)
    o += 8 * G * 10
    ratios = np.frombuffer(raw, "<f8", G * 9, o).reshape(G, 9)
    o += 8 * G * 9
    mask = np.frombuffer(raw, "<u4", G, o)
    return 0, {"times": times, "sums": sums, "ratios": ratios, "mask": mask}


def test_sanitized_oracle_brute_force_pins(oracle_exe, tmp_path):
    for seed in range(40):
        rng = np.random.default_rng(9000 + seed)
        tr = tg.random_tiny(rng, max_span=int(rng.integers(2, 80)), max_events=int(rng.integers(1, 16)))
        res, kind, s, e = tr.flat()
        rc, got = run_oracle(oracle_exe, tmp_path, tr.n_hosts, tr.n_devices, res, kind, s, e, tr.regions)
        assert rc == 0
        want = occupancy_times(tr)
        np.testing.assert_array_equal(got["times"], want)
        sums, ratios, mask = tree_from_times(want, tr.n_hosts, tr.n_devices, tr.regions)
        np.testing.assert_array_equal(got["sums"], sums)
        np.testing.assert_array_equal(got["ratios"], ratios)
        np.testing.assert_array_equal(got["mask"], mask)


def test_sanitized_oracle_pils_tables(oracle_exe, tmp_path):
    for name, printed, t in pils.load():
        tr = pils.build_trace(t, kernel_streams=4, hidden_memops=3)
        rc, got = run_oracle(oracle_exe, tmp_path, tr.n_hosts, tr.n_devices, *tr.flat(), tr.regions)
        assert rc == 0
        assert ["%.2f" % x for x in got["ratios"][0]] == ["%.2f" % x for x in printed], name


def test_sanitized_oracle_threads_equal_normal_build(oracle_exe, tmp_path):
    tr = tg.make_trace(17, 6, 5, 3, 4000, 1500, w_range=(0.5, 1.5), idle_range=(0.1, 0.4), regions="tiles",
                       n_regions=7)
    rc, got = run_oracle(oracle_exe, tmp_path, tr.n_hosts, tr.n_devices, *tr.flat(), tr.regions, threads=4)
    assert rc == 0
    want = oracle.compute(tr)
    for k in ("times", "sums", "mask"):
        np.testing.assert_array_equal(got[k], want[k])
    np.testing.assert_array_equal(got["ratios"].view(np.int64), want["ratios"].view(np.int64))


def test_sanitized_oracle_rejects_bad_input(oracle_exe, tmp_path):
    one = ([0], [tg.DEV_KERNEL])
    rc_interval = run_oracle(oracle_exe, tmp_path, 0, 1, *one, [5], [4], [(0, 10)])[0]
    rc_kind = run_oracle(oracle_exe, tmp_path, 1, 0, [0], [tg.DEV_KERNEL], [1], [2], [(0, 10)])[0]
    rc_region = run_oracle(oracle_exe, tmp_path, 0, 1, *one, [1], [2], [(10, 10)])[0]
    rc_resource = run_oracle(oracle_exe, tmp_path, 0, 1, [3], [tg.DEV_KERNEL], [1], [2], [(0, 10)])[0]
    assert rc_interval == -4 and rc_kind == -2 and rc_region == -5 and rc_resource < 0
    assert run_oracle(oracle_exe, tmp_path, 0, 1, [], [], [], [], [(0, 10)])[0] == 0


@pytest.fixture(scope="module")
def cache_exe(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("no g++")
    tmp = tmp_path_factory.mktemp("san_cache")
    return _build(tmp, "cache_san", ["g++", "-std=c++17"] + SAN + ["-I", CSRC,
                                                                  os.path.join(NATIVE, "tune_cache_main.cpp")])


GOOD = '{\n  "ev2^27_res2^9_k2^0": [256, 2048, 2048],\n  "ev2^27_res2^17_k2^10": [256, 2048, 512]\n}\n'

BAD = {
    "empty file": "",
    "truncated in a key": GOOD[:12],
    "truncated in a list": GOOD[:40],
    "truncated before the brace": GOOD.rstrip()[:-1],
    "two values": '{"a": [256, 2048]}',
    "four values": '{"a": [256, 2048, 512, 1]}',
    "not a number": '{"a": [256, x, 512]}',
    "huge number": '{"a": [25600000000000000000000, 2048, 512]}',
    "target too small": '{"a": [8, 2048, 512]}',
    "negative target": '{"a": [-256, 2048, 512]}',
    "bad capacity": '{"a": [256, 3000, 512]}',
    "bad tile": '{"a": [256, 2048, 1000]}',
    "escaped key": '{"a\\"b": [256, 2048, 512]}',
    "duplicate key": '{"a": [256, 2048, 512], "a": [128, 2048, 512]}',
    "trailing data": '{"a": [256, 2048, 512]} x',
    "missing comma": '{"a": [256, 2048, 512] "b": [256, 2048, 512]}',
    "array at top": '[["a", 256, 2048, 512]]',
    "binary": "\x00\xff\x01{",
    "float": '{"a": [256.5, 2048, 512]}',
}


def test_cache_reader_accepts_the_format(cache_exe, tmp_path):
    p = tmp_path / "c.json"
    p.write_text(GOOD)
    out = _run([cache_exe, str(p)]).splitlines()
    assert out == ["ok 2", "ev2^27_res2^17_k2^10 256 2048 512", "ev2^27_res2^9_k2^0 256 2048 2048"]
    p.write_text("{}")
    assert _run([cache_exe, str(p)]).splitlines() == ["ok 0"]
    assert _run([cache_exe, str(tmp_path / "absent.json")]).splitlines() == ["ok 0"]


@pytest.mark.parametrize("name", sorted(BAD))
def test_cache_reader_rejects_damage(cache_exe, tmp_path, name):
    p = tmp_path / "c.json"
    p.write_bytes(BAD[name].encode("latin-1"))
    out = _run([cache_exe, str(p)])
    assert out.startswith("error malformed tuning cache "), (name, out)


def test_cache_reader_every_truncation(cache_exe, tmp_path):
    p = tmp_path / "c.json"
    body = GOOD.rstrip()
    for k in range(len(body)):
        p.write_text(body[:k])
        out = _run([cache_exe, str(p)])
        assert out.startswith("error malformed"), (k, out)


def test_tree_rendering_within_every_buffer(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("no g++")
    exe = _build(tmp_path, "format_san", ["g++", "-std=c++17"] + SAN + [
        "-I", os.path.join(ROOT, "include"), "-x", "c++", os.path.join(CSRC, "hpop_format.hip"), "-x", "none",
        os.path.join(NATIVE, "format_main.cpp")])
    assert _run([exe]).startswith("ok 60")
