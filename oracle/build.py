"""Build the CPU oracle shared library (test infrastructure only).

Plain C++17, FP64, -O2, contraction of multiply-add into FMA switched off so
that every product is rounded as written.  Run as ``python -m oracle.build``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "radau5_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def compile_oracle(src: str, out: str, verbose: bool = False) -> str:
    """Compile an oracle source file into the shared library `out`."""
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
           "-I", HERE, "-o", out + ".tmp", src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build_oracle(verbose: bool = False) -> str:
    return compile_oracle(SRC, LIB, verbose)


if __name__ == "__main__":
    print(build_oracle(verbose="-v" in sys.argv))
