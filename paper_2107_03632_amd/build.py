"""Build librbffd.so (gfx950) from csrc/*.hip with hipcc, in-tree."""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librbffd.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no fused multiply-add unless written as fma(): the kernels reproduce the
    # reference's exact sequence of roundings
    "-ffp-contract=off",
    # keep packed FP32 instructions out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-pragma-unroll-threshold=2000000",
    "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


# per-source additions: the mixed-precision kernels keep their FP32 matrix-core
# accumulators in ordinary VGPRs (with accumulation registers the compiler
# copies the tiles back and forth and needs twice the registers)
EXTRA_FLAGS = {
    "weights_mx_k45.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "weights_mx_k84.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "weights_mx_op_k45.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "weights_mx_op_k84.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _deps(src: str) -> list[str]:
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    return [src, os.path.join(INCLUDE, "rbffd.h"), *hdrs, os.path.abspath(__file__)]


def _compile(src: str, force: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    if not force and os.path.exists(obj) and \
            os.path.getmtime(obj) >= max(os.path.getmtime(d) for d in _deps(src)):
        return obj
    tmp = obj + ".tmp"
    extra = EXTRA_FLAGS.get(os.path.basename(src), [])
    subprocess.run([HIPCC, *FLAGS, *extra, "-c", src, "-o", tmp], check=True)
    os.replace(tmp, obj)
    return obj


CALIB_SRC = os.path.join(HERE, "calib", "fma_peak.hip")
CALIB_LIB = os.path.join(HERE, "libcalib.so")


def build_calib() -> str:
    """The benchmark's FMA-rate calibration kernels (not part of librbffd)."""
    tmp = CALIB_LIB + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC, *FLAGS, "-shared", CALIB_SRC, "-o", tmp], check=True)
    os.replace(tmp, CALIB_LIB)
    return CALIB_LIB


def build(jobs: int = 16, force: bool = True) -> str:
    """Compile every source (force) or only the out-of-date ones, then link."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    # the slowest translation units first
    srcs.sort(key=lambda p: -os.path.getsize(p) if "weights_" not in p else -1e9)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    if force or not os.path.exists(CALIB_LIB) or \
            os.path.getmtime(CALIB_LIB) < os.path.getmtime(CALIB_SRC):
        build_calib()
    return LIB


if __name__ == "__main__":
    import sys
    print(build(force="--force" in sys.argv))
