"""Build the CPU test library: the host preprocessor (gt_geometry.cpp,
gt_tune.cpp) with host-memory stand-ins for the HIP runtime, plus the
tracker's device functions (gt_device.h) compiled for the host.  Test
infrastructure only; `asan=True` adds AddressSanitizer (host code)."""

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2406_13849_amd", "csrc")


def compiler():
    for c in (os.environ.get("GT_HOST_CXX"), "/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


def build(asan: bool = False) -> str:
    out = os.path.join(HERE, "libgt_cpu%s.so" % ("_asan" if asan else ""))
    srcs = [os.path.join(CSRC, "gt_geometry.cpp"), os.path.join(CSRC, "gt_tune.cpp"),
            os.path.join(HERE, "host_stubs.cpp"), os.path.join(HERE, "cpu_track.cpp")]
    newest = max(os.path.getmtime(p) for p in srcs + [os.path.join(CSRC, f) for f in os.listdir(CSRC)]
                 + [os.path.join(HERE, "shim.h")])
    if os.path.exists(out) and os.path.getmtime(out) >= newest:
        return out
    cxx = compiler()
    if cxx is None:
        raise RuntimeError("no clang++ for the CPU test build")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
             "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + HERE, "-I" + CSRC, "-x", "c++"]
    if asan:
        flags += ["-fsanitize=address", "-fno-omit-frame-pointer"]
    tmp = out + ".tmp%d" % os.getpid()
    r = subprocess.run([cxx] + flags + srcs + ["-o", tmp], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("CPU test build failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, out)
    return out


def asan_runtime():
    cxx = compiler()
    if cxx is None:
        return None
    r = subprocess.run([cxx, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None
