"""The library called from plain C (tests/c_abi_check.c, compiled with gcc
against include/ttn.h and the HIP runtime's C API): argument errors on the
CPU, and on the GPU the same energies as the Python binding gives for the
same configuration."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1905_01331_amd import binding
from paper_1905_01331_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.fixture(scope="module")
def c_prog(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        pytest.skip("gcc or the HIP headers are not installed")
    if not os.path.exists(binding.LIB_PATH):
        from paper_1905_01331_amd import build
        build.build()
    libdir = os.path.dirname(binding.LIB_PATH)
    out = str(tmp_path_factory.mktemp("c_abi") / "c_abi_check")
    cmd = [gcc, "-O2", "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c_abi_check.c"), "-o", out,
           "-L", libdir, "-lttn", "-Wl,-rpath," + libdir,
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return out


def test_c_caller_argument_checks(c_prog):
    r = subprocess.run([c_prog, "cpu"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "cpu checks passed" in r.stdout


@pytest.mark.gpu
def test_c_caller_matches_the_binding(c_prog):
    r = subprocess.run([c_prog, "gpu"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    e_c = [float(x) for x in r.stdout.split()]
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    binding.load_library()
    t = binding.TTN(binding.ChainInput(I.tfim_chain(1.0), 32, 6, "fp64", seed=7))
    e0 = t.energy()[0]
    t.sweep(2)
    e1 = t.energy()[0]
    t.sweep_grouped(1, 2)
    e2 = t.energy()[0]
    site, bond, _ = t.local_energies()
    total = float(site.sum() + bond.sum())
    t.close()
    print(f"  C {e_c}, binding {[e0, e1, e2, total]}")
    assert e_c[:3] == [e0, e1, e2]
    assert e2 <= e1 <= e0
    # the same minimum-size work buffer on both sides: the same launches
    assert abs(e_c[3] - total) <= 1e-13 * 32
    assert abs(total / 32 - e2) <= 1e-12
