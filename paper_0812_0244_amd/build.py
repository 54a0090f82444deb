"""Compile libvdwnl.so (HIP, gfx950) in-tree with hipcc.

Each translation unit is compiled to an object in its own hipcc process (in
parallel), then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libvdwnl.so")
SOURCES = ("api.hip", "kernels_f32_z.hip", "kernels_f32_x.hip", "kernels_f32_y.hip", "kernels_f64_z.hip",
           "kernels_f64_x.hip", "kernels_f64_y.hip", "kernels_dispatch.hip", "table_gen.hip")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed-FP32 instructions off: plain scalar/vector FP32 only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libvdwnl.so (always recompiles)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tag = ".%d" % os.getpid()
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + tag + ".o")
        cmd = [hipcc] + HIPCC_FLAGS + ["-c", "-o", obj, os.path.join(CSRC, src)]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        objs.append(obj)
    failed = False
    for src, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out + err)
            failed = True
        elif verbose:
            sys.stdout.write(err)
    try:
        if failed:
            raise RuntimeError("hipcc failed building libvdwnl.so")
        tmp = LIB + ".tmp%d" % os.getpid()
        res = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
                             capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libvdwnl.so")
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build())
