"""Build the HIP library libnlfeast.so in-tree for gfx950.

    python -m paper_1801_09794_amd.build [-j JOBS]

Every .hip and .cpp file under csrc/ is compiled with hipcc (-O3, --offload-arch=gfx950,
packed-FP32 instructions disabled) into an object under csrc/_build/, then linked into
paper_1801_09794_amd/libnlfeast.so.  Always recompiles.
"""
import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(CSRC, "_build")
LIB = os.path.join(HERE, "libnlfeast.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I", INCLUDE,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# device code: MFMA accumulators in ordinary VGPRs (the loop-carried accumulators of the GEMM
# tile otherwise bounce between VGPRs and AccVGPRs on every K step)
DEVICE_FLAGS = ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]
# host-only numerics (the reduced eigenproblem): AVX2/FMA and Fortran complex arithmetic rules
# (no C99 NaN recovery in complex multiply; Smith's division)
HOST_FLAGS = ["-march=x86-64-v3", "-fcx-fortran-rules"]
HOST_ONLY_SOURCES = {"host_dense.cpp"}


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + DEVICE_FLAGS + ["-c", src, "-o", obj]
    if os.path.basename(src) in HOST_ONLY_SOURCES:
        cmd = [HIPCC] + COMMON + HOST_FLAGS + ["-x", "c++", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), errs))
    return obj


def build(jobs=None, verbose=False):
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found at %s" % HIPCC)
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))
    jobs = jobs or min(8, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args()
    build(a.j, verbose=True)
