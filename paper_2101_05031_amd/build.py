"""Builds liblsl.so (the HIP kernels and the C ABI) for gfx950 in-tree."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblsl.so")
TOOL = os.path.join(HERE, "lsl_slice")
SOURCES = ["primitives.hip", "prep.hip", "bin.hip", "field.hip", "contours.hip",
           "backward.hip", "batch.hip", "probe.hip", "support.hip", "density.hip",
           "api.cpp", "autotune.cpp"]
ARCH = os.environ.get("LSL_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags() -> list[str]:
    # -ffp-contract=off: every fused multiply-add is written out explicitly,
    # and the binning formulas round exactly as written.  Packed FP32 VALU
    # instructions are disabled.
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def _compile(src: str, out_dir: str) -> str:
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [hipcc()] + flags() + lang + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    return obj


KERNEL_SOURCES = {
    "field": ["field_q32.hpp", "field_block.hpp", "batch.hip", "common.hpp", "kernels.hpp"],
    "backward": ["backward.hip", "field_q32.hpp", "common.hpp", "kernels.hpp"],
    "binning": ["prep.hip", "bin.hip", "primitives.hip", "common.hpp", "kernels.hpp"],
    "contours": ["contours.hip", "common.hpp", "kernels.hpp"],
}


def kernel_hash(name: str) -> str:
    """Hash of the code a kernel is built from, comments and whitespace left
    out (to tell whether a stored profile still describes the current
    kernel)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[name]:
        with open(os.path.join(CSRC, f), "r", encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def build(verbose: bool = True) -> str:
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, out_dir), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    # lsl_slice: a command-line slicer on the C ABI alone
    tool = os.path.join(HERE, "lsl_slice")
    cmd = [hipcc(), "-O2", "-std=c++17", f"--offload-arch={ARCH}",
           "-Wno-unused-command-line-argument", "-I", INCLUDE,
           os.path.join(HERE, "tools", "lsl_slice.cpp"), "-L", HERE, "-llsl",
           "-Wl,-rpath,$ORIGIN", "-o", tool + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"tool build failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tool + ".tmp", tool)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
