"""Build libjpet.so (gfx950) and the rate microbenchmark in-tree with hipcc."""

from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libjpet.so")
MICROBENCH = os.path.join(HERE, "microbench")
ARCH = os.environ.get("JPET_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled: the compiler would otherwise pair ordinary float
# arithmetic into v_pk_* forms.
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", tmp, *sources()]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
        if out.strip():
            print(out)
    os.replace(tmp, LIB)
    build_microbench(hipcc)
    return LIB


def build_microbench(hipcc: str | None = None) -> str:
    """The instruction-rate probes (microbench.hip) as a stand-alone executable."""
    hipcc = hipcc or os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = MICROBENCH + f".tmp{os.getpid()}"
    flags = [f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    res = subprocess.run([hipcc, *flags, "-o", tmp, os.path.join(HERE, "microbench.hip")], capture_output=True,
                         text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed (microbench):\n" + res.stdout + res.stderr)
    os.replace(tmp, MICROBENCH)
    return MICROBENCH


if __name__ == "__main__":
    print(build(verbose=True))
