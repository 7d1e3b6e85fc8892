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
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libace")
    return path


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I" + os.path.join(ROOT, "include")]


def compile_one(src, defines=(), build_dir=BUILD, flags=()):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "-c"] + common_flags() + ["-D" + d for d in defines] + list(flags) + \
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


# The C ABI layer (host code of these sources) under AddressSanitizer and UBSan; the kernels'
# objects are the ordinary ones.  The sanitizers apply to the host pass only.
HOST_SOURCES = ["abi.cpp", "batch.cpp", "scf_driver.cpp"]
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-g"]


def build_sanitized_driver(driver_src, out_dir, jobs=4):
    """Executable from driver_src (C++, calls the C ABI) linked against the library's objects
    with the host sources rebuilt under ASan + UBSan.  Returns its path."""
    os.makedirs(out_dir, exist_ok=True)
    # the kernels' objects of the last in-tree build when present, else compiled here
    plain = [s for s in SOURCES if s not in HOST_SOURCES]

    def kernel_obj(src):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        if os.path.exists(obj) and os.path.getmtime(obj) >= os.path.getmtime(os.path.join(CSRC, src)):
            return obj
        return compile_one(src, (), out_dir)

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: compile_one(s, (), out_dir, SANITIZE), HOST_SOURCES))
        objs += list(ex.map(kernel_obj, plain))
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    exe = os.path.join(out_dir, "abi_sanitize")
    cmd = [clang, "-std=c++17", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
           "-fsanitize=undefined", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "include"), driver_src] + objs + \
          ["-L" + os.path.join(ROCM, "lib"), "-Wl,-rpath," + os.path.join(ROCM, "lib"),
           "-lamdhip64", "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), res.stderr[-6000:]))
    return exe


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("-D", dest="defines", action="append", default=[])
    ap.add_argument("--out", default=LIB)
    a = ap.parse_args(argv)
    build(a.jobs, verbose=True, defines=a.defines, out=os.path.abspath(a.out))


if __name__ == "__main__":
    sys.exit(main())
