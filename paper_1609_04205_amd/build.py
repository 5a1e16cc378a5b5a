"""Build the HIP library libafc.so (gfx950) in-tree with hipcc.

Every HIP source is compiled with packed-FP32 instruction selection turned
off; objects are compiled in parallel and linked into one shared library.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libafc.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["ppf.hip", "ppf_fine.hip", "xengine.hip", "validity.hip", "flag.hip", "imaging.hip", "calib.hip", "checked.hip",
           "afc_api.cpp"]
# calib.hip relies on error-free product/sum transformations: no contraction
EXTRA = {"calib.hip": ["-ffp-contract=off"]}
ARCH = os.environ.get("AFC_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fvisibility=hidden", "-Wall", "-Wno-unused-function"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", *COMMON, *EXTRA.get(src, []), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    os.makedirs(BUILD, exist_ok=True)
    global COMMON
    saved = COMMON
    COMMON = COMMON + [f"-D{d}" for d in defines]
    try:
        with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
            objs = list(ex.map(_compile, SOURCES))
    finally:
        COMMON = saved
    tmp = out + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
