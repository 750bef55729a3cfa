"""Build a copy of libssicov.so whose host code carries AddressSanitizer and
UndefinedBehaviorSanitizer (device code unchanged), for checking the host
side of the library on the CPU: parameter validation, layouts, footprints and
the error paths.  Load it with the sanitizer runtime preloaded and
SSI_LIBRARY pointing at it (tests/test_host_sanitizers.py does both)."""
from __future__ import annotations

import glob
import os
import subprocess

from . import build as B

OUT_DIR = os.path.join(B.BUILD, "sanitized")
LIB = os.path.join(OUT_DIR, "libssicov_sanitized.so")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def runtime() -> str:
    """The clang AddressSanitizer runtime of the ROCm toolchain."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("no libclang_rt.asan-x86_64.so under /opt/rocm/llvm")
    return hits[-1]


def build() -> str:
    """Compile every source with host sanitizers (skipped when the library is
    newer than all sources) and link; returns the library path."""
    srcs = sorted(glob.glob(os.path.join(B.CSRC, "*.hip")))
    deps = srcs + glob.glob(os.path.join(B.CSRC, "*.h")) + [os.path.join(B.ROOT, "include",
                                                                           "ssicov.h")]
    if os.path.exists(LIB) and os.path.getmtime(LIB) > max(os.path.getmtime(d) for d in deps):
        return LIB
    os.makedirs(OUT_DIR, exist_ok=True)
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g"] + HOST_SAN
    procs, objs = [], []
    for src in srcs:
        obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append((src, subprocess.Popen([B.HIPCC, *flags, "-c", src, "-o", obj],
                                            stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                            text=True)))
    for src, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{out}\n{err}")
    cmd = [B.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB, *objs,
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-shared-libsan"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    return LIB
