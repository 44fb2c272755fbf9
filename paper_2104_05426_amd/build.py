"""Compile libjefi.so for gfx950 in-tree (hipcc).

Flags: -O3; -ffp-contract=off so that only the FMAs written out in the
sources are emitted (the FP64 slice-index sequence must not be contracted);
packed FP32 instructions disabled for device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjefi.so")
SOURCES = [os.path.join(CSRC, "jefi_kernels.hip"), os.path.join(CSRC, "jefi_api.cpp"),
           os.path.join(CSRC, "jefi_server.cpp"), os.path.join(CSRC, "jefi_coupler.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def command(out: str):
    return [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", os.path.join(HERE, "..", "include"),
            "-o", out] + SOURCES


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libjefi.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
