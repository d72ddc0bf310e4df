"""Builds libhpop.so (the HIP engine behind include/hpop.h) for gfx950 with hipcc."""
import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhpop.so")
OBJ = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    return obj, out


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    for _, out in results:
        if verbose and out.strip():
            print(out)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results] + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


COLLECT_SRC = os.path.join(PKG, "collect", "hpop_collect.cpp")
COLLECT_LIB = os.path.join(PKG, "libhpop_collect.so")
ROCM_INCLUDE = "/opt/rocm/include"
ROCM_LIB = "/opt/rocm/lib"
APP_SRC = os.path.join(ROOT, "tests", "apps", "collect_app.hip")
APP_BIN = os.path.join(ROOT, "tests", "apps", "collect_app")


def build_collect():
    """libhpop_collect.so: the rocprofiler-sdk tool (host code only, no HIP call)."""
    tmp = COLLECT_LIB + ".tmp%d" % os.getpid()
    cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE,
           "-I", ROCM_INCLUDE, COLLECT_SRC, "-o", tmp, "-L" + ROCM_LIB, "-lrocprofiler-sdk",
           "-Wl,-rpath," + ROCM_LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("collector build failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, COLLECT_LIB)
    return COLLECT_LIB


def build_app():
    """The collector's test application, linked to both libraries of the package."""
    tmp = APP_BIN + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + [APP_SRC, "-o", tmp, "-L" + PKG, "-lhpop", "-lhpop_collect",
                             "-Wl,-rpath," + PKG, "-Wl,-rpath,$ORIGIN/../../paper_2603_26576_amd"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("collect_app build failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, APP_BIN)
    return APP_BIN


def build_all(verbose=False):
    out = [build(verbose), build_collect()]
    out.append(build_app())
    return out


if __name__ == "__main__":
    print(build_all(verbose="-v" in sys.argv))
