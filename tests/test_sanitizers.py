"""CPU tests under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle and the host code of libsg (argument validation, pass planning,
the batch, pass-context and server objects, their C error paths) are built
again with -fsanitize=address,undefined for the host only (the gfx950 device
code is built as usual and never runs here), and the oracle pins, the C ABI
tests and the serving tests run against those builds with the sanitizer
runtime preloaded into the interpreter.  Any report fails the test: UBSan is
built not to recover, and the ASan log must be empty.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LLVM = "/opt/rocm/llvm"

# host-side sanitizer flags for hipcc: each -fsanitize= follows -Xarch_host,
# so only the host pass is instrumented
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address,undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
ORACLE_SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                   "-fno-omit-frame-pointer", "-g"]


def asan_runtime():
    found = sorted(glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux",
                                          "libclang_rt.asan-x86_64.so")))
    return found[-1] if found else None


@pytest.mark.slow
def test_oracle_abi_and_serving_tests_clean_under_asan_ubsan(tmp_path):
    rt = asan_runtime()
    clang = os.path.join(LLVM, "bin", "clang")
    if rt is None or not os.path.exists(clang):
        pytest.skip("the ROCm clang sanitizer runtime is not installed")
    sys.path.insert(0, ROOT)
    from oracle import build_oracle
    from paper_1706_04552_amd import build as sgbuild
    lib = sgbuild.build(extra_flags=HOST_SANITIZE, lib=str(tmp_path / "libsg_san.so"),
                        build_dir=str(tmp_path / "obj"))
    orc = build_oracle.build(cc=clang, extra_flags=ORACLE_SANITIZE,
                             lib=str(tmp_path / "liboracle_san.so"))
    log = tmp_path / "asan"
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        # the interpreter itself is not instrumented: its own allocations at
        # exit are not leaks of the code under test
        "ASAN_OPTIONS": f"detect_leaks=0:abort_on_error=0:halt_on_error=1:log_path={log}",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "SG_LIB_PATH": lib,
        "SG_ORACLE_LIB": orc,
        "OMP_NUM_THREADS": "4",
    })
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu and not slow",
           "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"),
           os.path.join(ROOT, "tests", "test_abi.py"),
           os.path.join(ROOT, "tests", "test_serving_cpu.py")]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    reports = sorted(glob.glob(str(log) + "*"))
    text = "".join(open(f).read() for f in reports)
    assert res.returncode == 0, res.stdout[-4000:] + res.stderr[-4000:] + text[-4000:]
    assert " passed" in res.stdout and " skipped" not in res.stdout, res.stdout[-2000:]
    assert "runtime error" not in res.stdout + res.stderr, res.stderr[-4000:]
    assert not reports, text[-4000:]
