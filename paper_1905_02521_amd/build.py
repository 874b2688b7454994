"""Build libqtb.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1905_02521_amd.build [--jobs N]

Each source compiles to an object of its own (in parallel), then one shared
library is linked next to this file.  Flags: -O3, gfx950 only, packed FP32
instructions disabled, and no FMA contraction in the noise generator (its
Gaussian transform is specified operation by operation).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libqtb.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["noise.hip", "fir.hip", "update.hip", "nlist.hip", "forces.hip", "ml.hip", "vdos.hip",
           "filter_design.cpp", "qtb_api.cpp"]
ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
PER_FILE = {"noise.hip": ["-ffp-contract=off"]}


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


# Host-code sanitizers (AddressSanitizer, UndefinedBehaviorSanitizer) for a
# checking build of the same sources: every flag applies to the host pass only
# (-Xarch_host), the GPU code is compiled as usual.
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [hipcc(), *COMMON, *PER_FILE.get(src, []), *extra, "-c", os.path.join(CSRC, src),
           "-o", obj]
    if src.endswith(".cpp"):
        cmd = [hipcc(), *[c for c in COMMON if not c.startswith("--offload-arch")], *extra,
               "-D__HIP_PLATFORM_AMD__", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 8, verbose: bool = False, sanitize: bool = False) -> str:
    """Compile and link libqtb.so next to this file; sanitize=True instead
    writes _build/san/libqtb_san.so with the host-code sanitizers (for the
    CPU tests that load it in a process preloading clang's ASan runtime)."""
    bdir = os.path.join(BUILD, "san") if sanitize else BUILD
    out = os.path.join(bdir, "libqtb_san.so") if sanitize else OUT
    extra = SAN if sanitize else []
    os.makedirs(bdir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda f: _compile(f, bdir, extra), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *extra,
           *(["-shared-libsan"] if sanitize else []), "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    a = ap.parse_args()
    build(a.jobs, verbose=True)
    sys.exit(0)
