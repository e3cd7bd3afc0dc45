"""Build libtc.so (the HIP kernels and the C-ABI runtime) for gfx950.

    python -m paper_2608_17390_amd.build

Compiles every source under csrc/ with hipcc into _build/ and links
paper_2608_17390_amd/libtc.so in-tree.  Packed FP32 instructions are
disabled for all device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtc.so")
INCLUDE = os.path.join(ROOT, "include")
SOURCES = ["tc_map.hip", "tc_render.hip", "tc_march.hip", "tc_shade.hip", "tc_api.cpp",
           "tc_plan.cpp", "tc_frame.cpp", "tc_server.cpp", "tc_noalloc.hip",
           "tc_voxel.hip"]
# per-source flags: the sampled march and the shading pass are defined one
# IEEE single operation at a time, so nothing may be fused into a multiply-add
EXTRA = {"tc_march.hip": ["-ffp-contract=off"], "tc_shade.hip": ["-ffp-contract=off"]}
ARCH = os.environ.get("TC_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I" + INCLUDE, "-I" + CSRC]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + EXTRA.get(src, []) + [
            "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    rc = [p.wait() for p in procs]
    if any(rc):
        raise RuntimeError("hipcc failed for %s" % [s for s, r in zip(SOURCES, rc) if r])
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs,
         verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
