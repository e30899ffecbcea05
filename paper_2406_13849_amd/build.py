"""Build libgt.so (HIP for gfx950) in-tree with hipcc.

Floating-point flags matter for correctness, not only speed: the tracker's
results must be the IEEE double results of the operation order written in
the sources, so contraction into fused multiply-add is off and no
fast-math option is used.  Packed FP32 instructions are disabled.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgt.so")
SOURCES = ["gt_geometry.cpp", "gt_tune.cpp", "gt_track.hip", "gt_track_axcz.hip", "gt_track_vert.hip", "gt_kinds.hip"]
ARCH = os.environ.get("GT_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def flags() -> list:
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel: the two kernel
    translation units take most of the time), then link libgt.so."""
    import tempfile
    with tempfile.TemporaryDirectory(prefix="gt_build_") as tmpdir:
        objs, procs = [], []
        for s in SOURCES:
            obj = os.path.join(tmpdir, s + ".o")
            cmd = [hipcc()] + flags() + ["-c", "-x", "hip", os.path.join(CSRC, s), "-o", obj]
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = []
        for s, pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                sys.stderr.write(out)
                failed.append(s)
        if failed:
            raise RuntimeError("hipcc failed on " + ", ".join(failed))
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libgt.so")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
