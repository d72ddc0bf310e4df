"""Time-bucket geometry of the engine's build (csrc/hpop_geom.h), on the CPU:
the native driver checks, for segment ranges from empty to 2^62 ns and
bucket counts from 1 to 2^24, that each probed start falls in the bucket
floor(((start - min) >> s0) / wx), inside that bucket's [lo, lo + width),
in time order, with times past the range clamped to the last bucket. Built
with AddressSanitizer and UndefinedBehaviorSanitizer when g++ has them."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("san", [False, True])
def test_bucket_geometry(tmp_path, san):
    if not shutil.which("g++"):
        pytest.skip("no g++")
    exe = str(tmp_path / "geom")
    flags = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"] if san else ["-O2"]
    r = subprocess.run(["g++", "-std=c++17"] + flags + ["-I", os.path.join(ROOT, "paper_2603_26576_amd", "csrc"),
                        os.path.join(ROOT, "tests", "native", "geom_main.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
