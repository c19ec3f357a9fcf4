"""Compile tests/c/capi_check.c (a plain C program that drives librd.so through
include/rd.h) into tests/c/capi_check.  Called by the repository's build step
after the library is built."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> str:
    exe = os.path.join(HERE, "capi_check")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "capi_check.c"), "-o", exe,
           "-L", os.path.join(ROOT, "paper_1506_04651_amd"), "-lrd",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/../../paper_1506_04651_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("capi_check build failed:\n" + r.stderr[-4000:])
    return exe


if __name__ == "__main__":
    print(build())
