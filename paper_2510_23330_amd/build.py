"""Build libgx.so (HIP for gfx950) in-tree with hipcc.

Each translation unit is compiled separately (in parallel) and linked into
one shared library next to this file.  The tree and walk units are compiled
with FP contraction off: their key and opening-criterion arithmetic must be
the exact IEEE sequence the tree definition states.  Packed FP32 instructions
are disabled for every unit.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libgx.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = {
    "gx_prims.hip": [],
    "gx_tree.hip": ["-ffp-contract=off"],
    "gx_walk.hip": ["-ffp-contract=off"],
    "gx_gravity.hip": [],
    "gx_integrate.hip": [],
    "gx_sph.hip": [],
    "gx_sn.hip": [],
    "gx_nn.hip": [],
    "gx_unet.hip": [],
}
ARCH = os.environ.get("GX_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INC, "-I", CSRC,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def _compile(src: str, extra: list[str]) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = ["hipcc", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every unit and link libgx.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, SOURCES[s]), srcs))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
