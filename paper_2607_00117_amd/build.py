"""Compiles libschw.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

Every device translation unit is built with the packed-FP32 target feature
disabled.  The double-precision integrator is additionally built with
-ffp-contract=off so its arithmetic is evaluated exactly as written.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libschw.so")
ARCH = os.environ.get("SCHW_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]
SOURCES = {
    "host.cpp": [],
    "integrate.hip": [],
    "integrate_f32.hip": [],
    "integrate_f64.hip": ["-ffp-contract=off"],
    "solve.hip": [],
    "gemm.hip": [],
    "mlp.hip": [],
    "gh.hip": [],
    "bootstrap.hip": [],
    "cellmass.hip": [],
    "jeans.hip": [],
    "bs23.hip": ["-ffp-contract=off"],
}


def _compile(src, extra):
    obj = os.path.join(BUILD, src + ".o")
    cmd = ["hipcc", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + extra
    if src.endswith(".cpp"):
        cmd = ["hipcc", "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + extra
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, SOURCES[s]), srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libschw.so failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
