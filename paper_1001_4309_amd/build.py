"""Build the HIP library ``libsfd.so`` in-tree for gfx950 with hipcc.

Usage: ``python -m paper_1001_4309_amd.build`` (or ``__graft_entry__.build()``).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsfd.so")

SOURCES = ["sfd_api.cpp", "sfd_kernels.hip", "sfd_rows.hip", "sfd_cols.hip", "sfd_persist.hip", "sfd_noalloc.hip"]

# Packed FP32 instructions are disabled for every device compile: some of their
# forms have produced silently wrong results on this hardware.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HIP library cannot be built")


def build(verbose: bool = False, extra=None) -> str:
    """Compile every source (in parallel: the kernel translation units take
    the longest) and link libsfd.so."""
    tmp = os.path.join(PKG, "_build")
    os.makedirs(tmp, exist_ok=True)
    common = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC] + (extra or [])
    jobs = []
    for src in SOURCES:
        obj = os.path.join(tmp, src + ".o")
        cmd = common + DEVICE_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    objs, failed = [], []
    for src, obj, proc in jobs:
        out, _ = proc.communicate()
        if proc.returncode != 0:
            sys.stderr.write(out)
            failed.append(src)
        objs.append(obj)
    if failed:
        raise RuntimeError(f"hipcc failed on {', '.join(failed)}")
    tmp_lib = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libsfd.so failed")
    os.replace(tmp_lib, LIB)
    return LIB


SAN_LIB = os.path.join(PKG, "_build", "libsfd_san.so")


def build_sanitized(verbose: bool = False) -> str:
    """The library with its host code (sfd_api.cpp: planning, validation,
    descriptors) built with AddressSanitizer and UndefinedBehaviorSanitizer,
    linked with the kernel objects of the last build().  Loaded only by the
    CPU tests of the boundary, with the sanitizer runtime preloaded."""
    tmp = os.path.join(PKG, "_build")
    obj = os.path.join(tmp, "sfd_api_san.o")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    cmd = [hipcc(), "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC] + san + ["-c", os.path.join(CSRC, "sfd_api.cpp"), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("sanitized compile of sfd_api.cpp failed")
    objs = [obj] + [os.path.join(tmp, src + ".o") for src in SOURCES if src != "sfd_api.cpp"]
    r = subprocess.run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", SAN_LIB] + objs,
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of the sanitized library failed")
    return SAN_LIB


if __name__ == "__main__":
    print(build(verbose=True))
