"""Build libsg.so, the gfx950 HIP library behind ``include/sg.h``, in-tree.

    python -m paper_1706_04552_amd.build

compiles every source under ``csrc/`` with hipcc for gfx950 (it cross-compiles
without a GPU) and links them into ``paper_1706_04552_amd/libsg.so``.
"""
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsg.so")
ROOT = os.path.dirname(HERE)
BUILD_DIR = os.path.join(ROOT, "_build")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

# Packed-FP32 instructions are disabled for every HIP source.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


# Sources that define the temporally blocked life pass (the kernel, its
# device helpers, its launch bookkeeping and the compile flags in this file).
LIFE_TB_SOURCES = ("sg_life_tb.hip", "sg_device.h", "sg_launch.h")


def source_digest(names=None) -> str:
    """SHA-256 over library sources (all of them, or the csrc files named),
    plus the compile flags, used to tell whether a stored profile still
    describes the current kernels."""
    import hashlib
    h = hashlib.sha256()
    # the flags with the checkout's own path left out, so that a copy of the
    # tree elsewhere gives the same digest
    h.update(" ".join(f.replace(ROOT, ".") for f in HIP_FLAGS).encode())
    if names is None:
        files = sorted(glob.glob(os.path.join(CSRC, "*")) + [os.path.join(ROOT, "include", "sg.h")])
    else:
        files = [os.path.join(CSRC, n) for n in sorted(names)]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False, jobs: int = 8, extra_flags=(), lib: str = LIB,
          build_dir: str = BUILD_DIR) -> str:
    """Compile every HIP source and link libsg.so; returns the library path.
    extra_flags, lib and build_dir serve other builds of the same sources
    (the sanitized host-code build of the CPU tests)."""
    os.makedirs(build_dir, exist_ok=True)
    objs, procs = [], []
    for src in sources():
        obj = os.path.join(build_dir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *HIP_FLAGS, *extra_flags, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra_flags, "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    if out:
        sys.stdout.write(out)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}")


if __name__ == "__main__":
    print(build(verbose=True))
