"""Build libkn.so (host C++ planner + gfx950 HIP engine) in-tree.

    python -m paper_1807_02119_amd.build            # libkn.so
    python -m paper_1807_02119_amd.build --sanitize # _build/san/libkn_san.so
    python -m paper_1807_02119_amd.build --checked  # libkn_checked.so

Host sources are compiled with g++, the HIP source with hipcc for gfx950
(packed-FP32 instruction selection disabled), and everything is linked by
hipcc into ``paper_1807_02119_amd/libkn.so``.  Always recompiles.

``--checked`` builds ``paper_1807_02119_amd/libkn_checked.so``: the engine with
device checks (KN_DEVICE_CHECKS: every task and its steps checked before they
run, a failing task skipped and reported, the guard zone after the arena
checked after each launch); load it with KN_LIBRARY=<path>.

``--sanitize`` builds a checking variant for the CPU tests: the host
sources with AddressSanitizer and UndefinedBehaviorSanitizer (g++), the
engine as usual, linked with g++ against the HIP runtime.  Load it with
KN_LIBRARY=<path> and the ASan runtime preloaded (see ``sanitizer_env``).
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libkn.so")

HOST_SOURCES = ["tait.cpp", "plan.cpp", "separator.cpp", "image.cpp", "jones.cpp", "runtime.cpp"]
HIP_SOURCES = ["engine.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")
ARCH = "gfx950"

HOST_FLAGS = ["-O3", "-march=x86-64-v2", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
              "-I" + os.path.join(ROOT, "include")]
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def _build_lib(out_dir, lib, hip_defines=(), verbose=False) -> str:
    os.makedirs(out_dir, exist_ok=True)
    jobs = []
    objs = []
    for s in HOST_SOURCES:
        o = os.path.join(out_dir, s.replace(".cpp", ".o"))
        jobs.append([CXX, *HOST_FLAGS, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in HIP_SOURCES:
        o = os.path.join(out_dir, s.replace(".hip", ".o"))
        jobs.append([HIPCC, *HIP_FLAGS, *hip_defines, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = lib + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, "-lpthread"])
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    return _build_lib(BUILD, LIB, verbose=verbose)


CHECKED_DIR = os.path.join(BUILD, "checked")
CHECKED_LIB = os.path.join(PKG, "libkn_checked.so")


def build_checked(verbose: bool = False) -> str:
    """libkn with the engine's device checks (KN_DEVICE_CHECKS)."""
    return _build_lib(CHECKED_DIR, CHECKED_LIB, hip_defines=("-DKN_DEVICE_CHECKS",),
                      verbose=verbose)


SAN_DIR = os.path.join(BUILD, "san")
SAN_LIB = os.path.join(SAN_DIR, "libkn_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def build_sanitized(verbose: bool = False) -> str:
    """libkn with the host code under ASan + UBSan (host-only instrumentation)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    host_flags = [f for f in HOST_FLAGS if f != "-O3"] + ["-O1", "-g"] + SAN_FLAGS
    jobs, objs = [], []
    for s in HOST_SOURCES:
        o = os.path.join(SAN_DIR, s.replace(".cpp", ".o"))
        jobs.append([CXX, *host_flags, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in HIP_SOURCES:
        o = os.path.join(SAN_DIR, s.replace(".hip", ".o"))
        jobs.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    _run([CXX, "-shared", "-fPIC", *SAN_FLAGS, *objs, "-o", SAN_LIB,
          "-L" + os.path.join(rocm, "lib"), "-Wl,-rpath," + os.path.join(rocm, "lib"),
          "-lamdhip64", "-lpthread"])
    return SAN_LIB


def sanitizer_env(env=None):
    """Environment for a process that loads the sanitized library: its path,
    the ASan runtime preloaded (the interpreter itself is not instrumented) and
    leak checking off (the interpreter and the HIP runtime keep memory to the
    end by design)."""
    env = dict(os.environ if env is None else env)
    asan = subprocess.run([CXX, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    env["KN_LIBRARY"] = SAN_LIB
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    elif "--checked" in sys.argv:
        print(build_checked(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
