"""Compile the CPU oracle (``sg_oracle.c``) into ``liboracle.so`` with gcc.

Test infrastructure only: the oracle is the checker of the HIP library, never
part of its compute path.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, cc: str = "gcc", extra_flags=(), lib: str = LIB) -> str:
    """Compile the oracle unconditionally and return the path of the library
    (cc, extra_flags and lib serve the sanitized build of the CPU tests)."""
    tmp = lib + ".tmp"
    cmd = [cc, "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", *extra_flags, "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
