"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle (C) and the library's host engine (C++, with stand-ins for the
device-side functions) are built with gcc / g++ -fsanitize=address,undefined
into a temporary folder; a child process that preloads the sanitizer
runtimes runs the oracle's pins and the library's host checks against those
builds (tests/sanitize/child.py).  Any sanitizer report ends the child with
a non-zero status and fails the test."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1410_1942_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g", "-O1"]


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                         text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.fixture(scope="module")
def builds():
    if not shutil.which("gcc") or not shutil.which("g++"):
        pytest.skip("gcc/g++ not available")
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes not installed")
    d = tempfile.mkdtemp(prefix="pcg_san_")
    try:
        oracle_so = os.path.join(d, "liboracle_san.so")
        subprocess.run(["gcc", "-std=c99", "-fopenmp", "-fPIC", "-shared", *SAN, "-o", oracle_so,
                        os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
        lib_so = os.path.join(d, "libpcgmi_san.so")
        subprocess.run(["g++", "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                        *SAN, "-o", lib_so, os.path.join(CSRC, "engine.cpp"),
                        os.path.join(HERE, "stub_launchers.cpp"),
                        "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64"],
                       check=True)
        yield oracle_so, lib_so, f"{asan}:{ubsan}"
    finally:
        shutil.rmtree(d, ignore_errors=True)


def test_host_code_under_sanitizers(builds):
    oracle_so, lib_so, preload = builds
    env = dict(os.environ, LD_PRELOAD=preload, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(HERE, "child.py"), oracle_so, lib_so],
                       env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "oracle: ok" in r.stdout and "library host code: ok" in r.stdout, tail
