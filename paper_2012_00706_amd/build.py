"""Compile libmpid.so (all HIP sources under csrc/) for gfx950 with hipcc.

Each source is compiled to an object in parallel, then the objects are linked
into one shared library (no relocatable device code: every translation unit
carries its own kernels)."""
from __future__ import annotations

import glob
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
REPO_DIR = os.path.dirname(PKG_DIR)
LIB_PATH = os.path.join(PKG_DIR, "libmpid.so")

HIPCC_FLAGS = [
    "-O3",
    "--offload-arch=gfx950",
    "-fPIC",
    "-std=c++17",
    # compiler-generated packed FP32 ops are kept off (v_pk_* fp32 forms)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG_DIR, "csrc", "*.hip")))


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res.stderr


def build_library(verbose: bool = False, jobs: int | None = None) -> str:
    """Always recompiles; writes to a temporary name and renames atomically."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(REPO_DIR, "include")]
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 1)))
    with tempfile.TemporaryDirectory(prefix="mpid_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in srcs]
        cmds = [[hipcc, *HIPCC_FLAGS, *inc, "-c", src, "-o", obj] for src, obj in zip(srcs, objs)]
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            logs = list(pool.map(_run, cmds))
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        logs.append(_run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]))
    if verbose:
        print("\n".join(x for x in logs if x))
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


# host code under AddressSanitizer and UndefinedBehaviorSanitizer (the device
# code is built as usual); "-Xarch_host" keeps each sanitizer off the GPU side
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
HOST_CHECK_SRC = os.path.join(REPO_DIR, "tests", "host_check", "host_check.cpp")


def build_host_check(outdir: str | None = None) -> str:
    """A sanitizer build of the library's host code (libmpid_host_check.so)
    and of the host-side ABI checker linked against it; returns the checker's
    path.  Runs without a GPU."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    outdir = outdir or os.path.join(REPO_DIR, "_build", "host_check")
    os.makedirs(outdir, exist_ok=True)
    inc = ["-I", os.path.join(REPO_DIR, "include")]
    srcs = sources()
    objs = [os.path.join(outdir, os.path.basename(src) + ".o") for src in srcs]
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + ["-O1"] + HOST_SANITIZE
    cmds = [[hipcc, *flags, *inc, "-c", src, "-o", obj] for src, obj in zip(srcs, objs)]
    with ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 1)) as pool:
        list(pool.map(_run, cmds))
    lib = os.path.join(outdir, "libmpid_host_check.so")
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs])
    exe = os.path.join(outdir, "host_check")
    _run([hipcc, "-O1", "--offload-arch=gfx950", *HOST_SANITIZE, *inc, HOST_CHECK_SRC, "-o", exe,
          "-L", outdir,
          "-lmpid_host_check", "-Wl,-rpath," + outdir])
    return exe


if __name__ == "__main__":
    print(build_library(verbose=False))
