"""The C ABI from a plain C program: tests/c/capi_check.c allocates device
memory with the HIP runtime, calls rd_reaction_step / rd_reaction_step_ex
through include/rd.h and checks the states against the exact solution of a
diagonal linear model, the counters, the one-launch schedule against the
persistent one, and the error returns of invalid calls (no Python or torch on
that path)."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu


def test_c_program_through_the_abi():
    exe = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "capi_check")
    if not os.path.exists(exe):
        pytest.fail("tests/c/capi_check is not built (run the build step)")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
