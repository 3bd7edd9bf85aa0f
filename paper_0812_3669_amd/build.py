"""Builds the HIP library ``libmoff.so`` (C ABI in ``include/moff.h``) for gfx950 with hipcc.

Packed FP32 instructions are disabled for the device code (``-packed-fp32-ops``); hipcc's host pass warns that
it does not know that target feature, which is harmless.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmoff.so")
SOURCES = ["plan.cpp", "moff_api.cpp", "kernels.hip", "kernels_mfma.hip", "kernels_cal.hip", "kernels_probe.hip",
           "kernels_noalloc.hip", "kernels_rowgemm.hip"]
ARCH = os.environ.get("MOFF_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"),
            "-I" + CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("compile failed: " + " ".join(cmd) + "\n" + err)
    return err


def build(verbose: bool = False) -> str:
    """Compiles every source (in parallel) and links ``libmoff.so`` in the package directory; returns its path."""
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="moff_build_")
    try:
        objs = []
        cmds = []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            objs.append(obj)
            cmds.append([cc] + _flags() + ["-c", os.path.join(CSRC, src), "-o", obj])
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            outs = list(ex.map(_run, cmds))
        if verbose:
            for o in outs:
                if o.strip():
                    print(o, file=sys.stderr)
        out_tmp = LIB + ".tmp%d" % os.getpid()
        _run([cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", out_tmp] + objs)
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
