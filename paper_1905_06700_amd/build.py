"""Build librt3d.so (gfx950) in-tree with hipcc.

Every HIP source of ``csrc/`` and the host runtime are compiled for gfx950
with -O3; packed FP32 instructions are disabled (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librt3d.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["rt3d_host.cpp", "k_compact.hip", "k_init.hip", "k_steps.hip", "k_apss.hip", "k_filter.hip",
           "k_cnn.hip", "k_events.hip", "k_loop.hip", "k_sr.hip"]
FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for s, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature flag; that warning is expected
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if lines and (verbose or p.returncode):
            print("\n".join(lines), file=sys.stderr)
        if p.returncode:
            failed.append(s)
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


def build_sanitized(outdir: str) -> str:
    """librt3d.so with AddressSanitizer and UndefinedBehavior Sanitizer in its
    host code (device code as usual), and csrc/host_selftest.c linked against
    it; returns the test executable's path (run it with
    ASAN_OPTIONS=detect_leaks=0: the HIP runtime keeps its allocations)."""
    os.makedirs(outdir, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"] + san
    procs, objs = [], []
    for s in SOURCES:
        obj = os.path.join(outdir, os.path.splitext(s)[0] + ".o")
        procs.append((s, subprocess.Popen([HIPCC] + flags + ["-x", "hip", "-c", os.path.join(CSRC, s), "-o", obj],
                                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = [s for s, p in procs if p.wait()]
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    lib = os.path.join(outdir, "librt3d.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-o", lib] + san + objs)
    exe = os.path.join(outdir, "host_selftest")
    subprocess.check_call([HIPCC, "-x", "c", os.path.join(CSRC, "host_selftest.c"), "-x", "none", "-o", exe, lib,
                           "-Wl,-rpath," + outdir, "-lm"] + san)
    return exe


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
