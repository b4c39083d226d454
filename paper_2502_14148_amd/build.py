"""Build liboc.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2502_14148_amd.build  [--jobs N]

Every HIP translation unit under csrc/ is compiled for gfx950 with packed
FP32 instructions disabled, then linked into paper_2502_14148_amd/liboc.so.
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "liboc.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-munsafe-fp-atomics",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]

SOURCES = ["tendency_r5.hip", "tendency_r4.hip", "tendency.hip",
           "api.hip", "stencil.hip", "poisson.hip", "barotropic.hip", "mlp.hip",
           "closure_api.hip", "hydrostatic.hip",
           "ensemble_api.hip", "coarse.hip", "vertical.hip", "les.hip", "immersed.hip"]


def _compile(src, defines=(), build_dir=None):
    obj = os.path.join(build_dir or BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *[f"-D{x}" for x in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int = 4, verbose: bool = False, defines=(), out=None) -> str:
    """Compile and link; `defines` (NAME=VALUE strings) and `out` build a
    variant library elsewhere (for tuning experiments)."""
    lib = out or LIB
    build_dir = BUILD if out is None else os.path.join(BUILD, os.path.basename(out) + ".d")
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s_: _compile(s_, defines, build_dir), SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    try:
        build(a.jobs, verbose=True)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
