"""Build librd.so (HIP, gfx950) in the package directory.

Every translation unit is compiled with hipcc for gfx950 only, without the
compiler's packed-FP32 instruction selection, and with floating-point
contraction limited to single expressions (so a given source expression is
rounded identically wherever it is inlined).  Run: python -m
paper_1506_04651_amd.build
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "librd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["rd_api.cpp", "rd_serving.cpp", "rd_kernels_small.hip", "rd_kernels_group.hip",
           "rd_kernels_fd.hip", "rd_order.hip", "rd_diffusion.hip", "rd_strang.cpp", "rd_mra.hip",
           "rd_noalloc.hip", "rd_kernels_group_fd.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC]


# the 16-lane group kernels unroll 16-step LU loops completely; the default
# pragma threshold would stop short and leave the cell state in scratch
EXTRA = {"rd_kernels_group.hip": ["-mllvm", "-pragma-unroll-threshold=200000"],
         "rd_kernels_group_fd.hip": ["-mllvm", "-pragma-unroll-threshold=200000"],
         # the multiresolution thresholds compare floating-point details: every
         # formula is evaluated operation by operation, without contraction
         "rd_mra.hip": ["-ffp-contract=off"]}


PHASE_BUILD = os.path.join(os.path.dirname(HERE), "_build_phase")
PHASE_LIB = os.path.join(HERE, "librd_phase.so")


def _compile(src, verbose, build_dir=BUILD, defines=()):
    path = os.path.join(CSRC, src)
    obj = os.path.join(build_dir, src + ".o")
    cmd = [HIPCC] + FLAGS + list(defines) + EXTRA.get(src, []) + ["-x", "hip", "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def _build(lib, build_dir, defines, verbose, jobs):
    os.makedirs(build_dir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, build_dir, defines), srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False, jobs: int = 8) -> str:
    return _build(LIB, BUILD, (), verbose, jobs)


def build_phase_profile(verbose: bool = False, jobs: int = 8) -> str:
    """A diagnostic copy of the library whose persistent kernels count the
    cycles of their phases (RD_PHASE_PROFILE, rd_phase.h), for
    phase_profile.py; the product library is not touched."""
    return _build(PHASE_LIB, PHASE_BUILD, ("-DRD_PHASE_PROFILE",), verbose, jobs)


if __name__ == "__main__":
    if "--phase-profile" in sys.argv:
        print(build_phase_profile(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
