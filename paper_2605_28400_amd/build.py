"""Builds libtrioseq.so for gfx950 in-tree with hipcc (no JIT cache).

Each source is compiled to an object in parallel, then the objects are
linked into the shared library (written atomically next to this file).
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libtrioseq.so")
SOURCES = ["sweep.hip", "traceback.hip", "noalloc.hip", "api.cpp", "serve.cpp", "align.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are kept out of every code object we build.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    return res.returncode, res.stdout + res.stderr


def build(verbose: bool = False, extra: list | None = None, incremental: bool = False) -> str:
    """Compiles every source (incremental: only sources newer than their
    object in _build/, headers counting for all) and links the library."""
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    keep = os.path.join(PKG, "_build")
    with tempfile.TemporaryDirectory(prefix="trioseq_build_") as tmpd:
        odir = keep if incremental else tmpd
        os.makedirs(odir, exist_ok=True)
        objs = [os.path.join(odir, s + ".o") for s in srcs]
        headers = [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
        headers.append(os.path.join(PKG, "..", "include", "trioseq.h"))
        newest_h = max(os.path.getmtime(h) for h in headers)

        def stale(s, o):
            if not incremental or not os.path.exists(o):
                return True
            return os.path.getmtime(o) < max(newest_h, os.path.getmtime(os.path.join(CSRC, s)))

        cmds = [[HIPCC, *FLAGS, *(extra or []), "-c", "-o", o, os.path.join(CSRC, s)]
                for s, o in zip(srcs, objs) if stale(s, o)]
        with ThreadPoolExecutor(max_workers=max(1, min(len(cmds), os.cpu_count() or 1))) as ex:
            results = list(ex.map(_run, cmds))
        srcs = [c[-1].rsplit("/", 1)[-1] for c in cmds]
        for (rc, out), s in zip(results, srcs):
            if rc != 0:
                sys.stderr.write(out)
                raise RuntimeError(f"hipcc failed compiling {s}")
            if verbose and out:
                sys.stderr.write(out)
        tmp = LIB + ".tmp%d" % os.getpid()
        rc, out = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
        if rc != 0:
            sys.stderr.write(out)
            raise RuntimeError("hipcc failed linking libtrioseq.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
