"""Measure the device's vector FMA throughput (FP64 and FP32 without packed
instructions), the peaks the roofline fractions are quoted against.  Builds
peak_probe.hip with the library's code-generation flags into _build/ and runs
it; prints one JSON line.  Run: python -m paper_1506_04651_amd.peak_probe"""
import os
import subprocess
import sys

from .build import BUILD, HIPCC

HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "peak_probe")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature",
                    "-Xclang", "-packed-fp32-ops", os.path.join(HERE, "peak_probe.hip"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def main():
    return subprocess.run([build()]).returncode


if __name__ == "__main__":
    sys.exit(main())
