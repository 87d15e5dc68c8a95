"""The host code under the sanitizers, on the CPU.

* libjpet's host side (argument validation, plan enumeration, workspace and batch layouts), built
  without device code (the launchers are stubs) with AddressSanitizer and
  UndefinedBehaviorSanitizer, driven through the C-ABI by a harness over many geometries;
* the oracle built with the same sanitizers, running its pins.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1502_07478_amd", "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, (" ".join(cmd), res.stdout[-4000:], res.stderr[-4000:])
    return res


def test_library_host_code_under_asan_ubsan(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    exe = str(tmp_path / "harness")
    _run([hipcc, "-x", "hip", "--cuda-host-only", "-std=c++17", "-O1", "-g", *SAN,
          "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          os.path.join(CSRC, "jpet_abi.hip"), os.path.join(HERE, "stubs.cpp"), os.path.join(HERE, "harness.cpp"),
          "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = _run([exe], env=env, timeout=600)
    assert "ok (0 failures)" in res.stdout, res.stdout[-2000:]


def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "libjpet_oracle_asan.so")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-o", lib, os.path.join(ROOT, "oracle", "jpet_oracle.c"), "-lm"])
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, JPET_ORACLE_LIB=lib, LD_PRELOAD=f"{asan} {ubsan}",
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         capture_output=True, text=True, env=env, cwd=ROOT, timeout=1200)
    assert res.returncode == 0, (res.stdout[-4000:], res.stderr[-4000:])
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
