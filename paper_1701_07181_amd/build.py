"""Build libirk.so for gfx950 in-tree with hipcc.

Every translation unit is compiled with -O3 for gfx950 and with packed FP32
instructions disabled (some of their forms have produced wrong results on
the target machines); the objects are linked into one shared library next
to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libirk.so")
SOURCES = ["irk_api.hip", "k_matvec.hip", "k_sweep.hip", "k_sweep_flow.hip", "k_factor.hip", "k_krylov.hip",
           "k_untransformed.hip", "k_step.hip"]
ARCH = os.environ.get("IRK_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # matrix-core accumulators in ordinary VGPRs (no copies through AGPRs
         # around the FP64 MFMA loops)
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC,
         "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def _includes(path: str, seen: set) -> set:
    """Local headers a source includes, transitively (quoted includes found
    in csrc/ or include/)."""
    import re
    for name in re.findall(r'^\s*#\s*include\s+"([^"]+)"', open(path).read(), re.M):
        for d in (CSRC, os.path.join(ROOT, "include")):
            f = os.path.join(d, name)
            if os.path.exists(f) and f not in seen:
                seen.add(f)
                _includes(f, seen)
    return seen


def _up_to_date(obj: str, src: str) -> bool:
    if not os.path.exists(obj):
        return False
    path = os.path.join(CSRC, src)
    deps = [path] + sorted(_includes(path, set()))
    return os.path.getmtime(obj) > max(os.path.getmtime(d) for d in deps)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if incremental and _up_to_date(obj, src):
        return obj
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    if out.strip():
        print(out, file=sys.stderr)
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental=True skips objects newer than their
    source and every header) and link libirk.so."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda f: _compile(f, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
