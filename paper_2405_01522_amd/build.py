"""Build libace.so (HIP, gfx950) in-tree.

Every source under csrc/ is compiled by hipcc for gfx950 into _build/ and linked into
paper_2405_01522_amd/libace.so.  Packed-FP32 instructions are disabled for all device code.

    python -m paper_2405_01522_amd.build [--jobs N]
"""

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libace.so")
SOURCES = ["poisson.hip", "poisson_queue.hip", "ace_kernels.hip", "tda.hip", "linalg.hip", "scf.hip",
           "convnet.hip", "batch.cpp",
           "abi.cpp", "scf_driver.cpp"]
ARCH = "gfx950"


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libace")
    return path


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I" + os.path.join(ROOT, "include")]


def compile_one(src, defines=(), build_dir=BUILD):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "-c"] + common_flags() + ["-D" + d for d in defines] + \
        ["-x", "hip", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), res.stderr[-6000:]))
    return obj


def build(jobs=4, verbose=False, defines=(), out=LIB):
    """Compile and link.  ``defines`` are extra -D macros (tuning knobs such as
    ACE_XY_THREADS); ``out`` is the library path (default: the in-tree libace.so)."""
    build_dir = BUILD if out == LIB else os.path.join(BUILD, os.path.basename(out) + ".d")
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: compile_one(s, defines, build_dir), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), res.stderr[-6000:]))
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("-D", dest="defines", action="append", default=[])
    ap.add_argument("--out", default=LIB)
    a = ap.parse_args(argv)
    build(a.jobs, verbose=True, defines=a.defines, out=os.path.abspath(a.out))


if __name__ == "__main__":
    sys.exit(main())
