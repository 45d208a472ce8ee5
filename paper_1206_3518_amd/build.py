"""Compiles the HIP sources under csrc/ for gfx950 into libbse.so (in-tree)."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libbse.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["pair_density.hip", "gemm_f64.hip", "gemm_mixed.hip", "spectrum.hip", "backward.hip", "validate.hip",
           "time_reversal.hip", "noalloc.hip", "haydock.hip", "screening.hip", "bse_api.cpp"]

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", "-c", *FLAGS, "-o", obj, os.path.join(SRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines() if "unknown target feature" not in l
                    and "warning generated" not in l and "warnings generated" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    return obj, err


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(SRC, s))]
    with cf.ThreadPoolExecutor(max_workers=jobs or min(8, len(srcs))) as ex:
        res = list(ex.map(_compile, srcs))
    if verbose:
        for _, e in res:
            if e.strip():
                print(e, file=sys.stderr)
    tmp = OUT + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + [o for o, _ in res]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    print(OUT)
