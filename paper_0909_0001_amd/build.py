"""Build libomniscope.so for gfx950 with hipcc (in-tree, no JIT cache).

    python paper_0909_0001_amd/build.py [--incremental]   # or __graft_entry__.build()

Every source under csrc/ is compiled to an object in _build/ (in parallel),
then linked into paper_0909_0001_amd/libomniscope.so.  All device code is
built with packed-FP32 instructions disabled.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libomniscope.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


COMMON = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    "-Xclang",
    "-target-feature",
    "-Xclang",
    "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I",
    os.path.join(ROOT, "include"),
    "-I",
    CSRC,
]


# Per-source extra flags.  fengine.hip: keep matrix-core results in ordinary VGPRs (its int32 accumulators are
# read by vector code right after each block; in accumulation registers every value costs one extra move).
EXTRA = {"fengine.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _local_includes(path: str, seen: set) -> set:
    """The project headers `path` includes, directly or through other project headers."""
    for line in open(path):
        line = line.strip()
        if line.startswith("#include") and '"' in line:
            name = line.split('"')[1]
            for d in (CSRC, os.path.join(ROOT, "include")):
                h = os.path.join(d, name)
                if os.path.exists(h) and h not in seen:
                    seen.add(h)
                    _local_includes(h, seen)
    return seen


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        deps = [src, *_local_includes(src, set())]
        if all(os.path.getmtime(obj) >= os.path.getmtime(d) for d in deps):
            return obj
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [hipcc(), *COMMON, *EXTRA.get(os.path.basename(src), []), *lang, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(
        os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp"))
    )
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, incremental), srcs))
    tmp = LIB + ".tmp"
    # roctx ranges around the entry points (rocprofv3 --marker-trace shows them)
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-L/opt/rocm/lib",
           "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
