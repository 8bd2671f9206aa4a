"""AddressSanitizer and UndefinedBehaviorSanitizer on the CPU.

* the oracle's C code (oracle/staggered.c), built with gcc and the sanitizers
  and driven by tests/sanitize/oracle_check.c over every exported routine;
* the host side of the C ABI: the library's host sources (api, driver,
  solver, rhmc) built with the sanitizers on the host pass only, linked with
  the device objects of the normal build, and driven by
  tests/sanitize/abi_host.c through the argument checks, bookkeeping and
  batch-driver paths that need no GPU.
A sanitizer report aborts the program (no recovery), so a clean run exits 0.
"""
import concurrent.futures as cf
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
# hipcc: every sanitizer flag on the host pass only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
HOST_SOURCES = ["api.cpp", "driver.cpp", "rhmc.cpp", "solver.cpp"]
CLANG = "/opt/rocm/llvm/bin/clang"


def _run(exe, tmp_path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env,
                       cwd=str(tmp_path))
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout[-3000:] + r.stderr[-6000:]


def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_check"
    subprocess.check_call(["gcc", "-std=c99", *SAN, os.path.join(ROOT, "oracle", "staggered.c"),
                           os.path.join(HERE, "sanitize", "oracle_check.c"), "-lm", "-o", str(exe)])
    _run(exe, tmp_path)


def test_abi_host_code_under_asan_ubsan(tmp_path):
    from paper_1808_01829_amd import build
    csrc = os.path.join(ROOT, "paper_1808_01829_amd", "csrc")
    dev = [os.path.join(build.OBJ, s + ".o") for s in build.sources() if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in dev):
        build.build()

    def compile_host(src):
        obj = str(tmp_path / (src + ".o"))
        cmd = (["hipcc"] + build.CFLAGS[:1] + ["-O1", "-g", "-std=c++17", "-fPIC"] + HOST_SAN +
               ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-I" + os.path.join(ROOT, "include"), "-x", "hip", "-c",
                os.path.join(csrc, src), "-o", obj])
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with cf.ThreadPoolExecutor(4) as ex:
        host = list(ex.map(compile_host, HOST_SOURCES))
    lib = tmp_path / "libbms_san.so"
    subprocess.check_call(["hipcc", build.CFLAGS[0], "-shared", "-fPIC", "-o", str(lib)] + dev +
                          host)
    exe = tmp_path / "abi_host"
    hip_lib = "/opt/rocm/lib"
    subprocess.check_call([CLANG, *SAN, "-I" + os.path.join(ROOT, "include"),
                           os.path.join(HERE, "sanitize", "abi_host.c"), "-L" + str(tmp_path),
                           "-lbms_san", "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath," + hip_lib,
                           "-o", str(exe)])
    _run(exe, tmp_path)
