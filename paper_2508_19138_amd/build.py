"""Build the HIP library libqtx_rgf.so in-tree for gfx950.

    python -m paper_2508_19138_amd.build

Every source under csrc/ is compiled by hipcc into an object (in parallel)
and linked into paper_2508_19138_amd/libqtx_rgf.so.  Always rebuilds.
"""

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libqtx_rgf.so")

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core accumulators in ordinary VGPRs: avoids AGPR<->VGPR copies
    # of every accumulator around the k-loop
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-result",
]


# Per-source options.  zinv.hip: the panel kernel keeps R rows of the panel
# in registers, which needs every loop over them fully unrolled (the
# largest instance exceeds the default size limit of a requested unroll)
# and no indexed access to them: the candidate row is copied out of one of
# the R rows chosen at run time, written as one branch per row, and sinking
# the branches' common stores into one block would turn that into an
# indexed access and move the whole row array to scratch memory.
PER_FILE = {
    "zinv.hip": ["-mllvm", "-simplifycfg-sink-common=false",
                 "-mllvm", "-pragma-unroll-threshold=200000"],
}


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    extra = PER_FILE.get(os.path.basename(src), [])
    cmd = [HIPCC] + COMMON + extra + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) +
                  glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
