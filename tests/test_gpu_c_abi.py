"""The library driven from plain C through include/hfgpe.h (tests/c_abi_driver.c):
no Python binding and no torch in the process.  The driver checks closed forms
of the linear harmonic oscillator (coherent state, 2-D ground state), norm
conservation of a ragged nonlinear c64 batch, and the error paths."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1007_3470_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_c_driver(tmp_path):
    assert os.path.exists(os.path.join(LIBDIR, "libhfgpe.so")), "libhfgpe.so is not built"
    exe = str(tmp_path / "c_abi_driver")
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROCM, "include"), "-D__HIP_PLATFORM_AMD__",
                           os.path.join(ROOT, "tests", "c_abi_driver.c"), "-o", exe, "-L", LIBDIR, "-lhfgpe",
                           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm", "-Wl,-rpath," + LIBDIR,
                           "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    print("running the C driver", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK: 0 failed" in r.stdout
