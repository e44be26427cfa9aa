"""Build the HIP library (gfx950) in-tree.

``libsamplesort.so`` is compiled from ``csrc/samplesort.hip`` (which
includes the kernels) with hipcc for gfx950 only.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libsamplesort.so")
SOURCES = [os.path.join(CSRC, "samplesort.hip")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("ss_kernels.h", "ss_device.h", "ss_wide.h", "ss_pairs.h", "ss_sortfirst.h", "ss_tuned.h", "ss_strings.h")] + [
    os.path.join(os.path.dirname(HERE), "include", "samplesort.h")]


def hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def command(out):
    return [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            *SOURCES, "-o", out]


def build(verbose=False):
    tmp = SO + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    build(verbose=True)
    print(SO)
