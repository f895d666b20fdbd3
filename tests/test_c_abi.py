"""The C ABI from C: include/fnlsim.h compiled as C11 (gcc, no C++), linked
against libfnlsim.so, and the validation paths called (they run before any
HIP call, so no GPU is needed).  Runs tests/c/abi_check.c."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_0909_0009_amd")


@pytest.fixture(scope="module")
def libdir():
    from paper_0909_0009_amd import build
    if build.stale():
        build.build()
    return PKG


def test_header_compiles_as_c_and_validation_holds(libdir, tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not available")
    exe = str(tmp_path / "abi_check")
    cmd = [gcc, "-std=c11", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "abi_check.c"), "-L", libdir, "-lfnlsim",
           f"-Wl,-rpath,{libdir}", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "C ABI checks passed" in out.stdout
