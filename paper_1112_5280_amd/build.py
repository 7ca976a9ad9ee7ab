"""Build ``libwilson.so`` (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_1112_5280_amd.build`` (or ``build()`` from Python).
Every source is compiled each call; objects go to ``_build/`` at the repo root.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libwilson.so")

SOURCES = ["wl_api.hip", "wl_dslash.hip", "wl_hop_f64.hip", "wl_hop_f32.hip", "wl_hop_f16.hip",
           "wl_blas.hip", "wl_solver.hip", "wl_server.hip", "wl_meson.hip",
           "wl_gauge.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in any kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-pthread",
    "-I", INCLUDE, "-I", CSRC,
]


def _compile(src: str, defines=(), build_dir=BUILD) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, *["-D" + d for d in defines], "-c", os.path.join(CSRC, src),
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose: bool = False, defines=(), out: str = LIB) -> str:
    """Compile every source and link ``out`` (default: the in-tree library).

    ``defines`` are extra ``NAME=VALUE`` preprocessor definitions (launch-shape
    knobs of the kernels); objects of such builds go to their own folder.
    """
    build_dir = BUILD if not defines else os.path.join(
        BUILD, "v_" + "_".join(d.replace("=", "") for d in defines))
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, defines, build_dir), SOURCES))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
