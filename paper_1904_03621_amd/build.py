"""Build the gfx950 shared library (libsgpu.so) in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsgpu.so")
SOURCES = [os.path.join(CSRC, "sg_kernels.hip"), os.path.join(CSRC, "sg_logz.hip"),
           os.path.join(CSRC, "sg_dos.hip"), os.path.join(CSRC, "sg_qubo.hip"),
           os.path.join(CSRC, "sg_probe.hip"),
           os.path.join(CSRC, "sg_api.cpp")]
HEADERS = [os.path.join(CSRC, "sg_internal.h"),
           os.path.join(os.path.dirname(HERE), "include", "sg.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed fp32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every source into libsgpu.so (always recompiles unless force=False
    and the library is newer than all sources)."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in SOURCES + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, stderr=None if verbose else subprocess.PIPE)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
