"""The C ABI from a plain C program (tests/c_abi_client.c): it compiles against
include/fse.h and links libfse.so on the CPU; on the GPU it runs the
closed-form constant-image case for the whole image and the tile framework."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2207_00238_amd")


def _compile(out_path):
    cmd = ["gcc", "-std=c11", "-O1", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c_abi_client.c"), "-o", out_path,
           "-L" + PKG, "-lfse", "-Wl,-rpath," + PKG, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
           "-lm"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout


def test_c_client_compiles_and_links(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libfse.so")):
        pytest.skip("libfse.so is not built")
    _compile(str(tmp_path / "c_abi_client"))


@pytest.mark.gpu
def test_c_client_runs(tmp_path):
    exe = str(tmp_path / "c_abi_client")
    _compile(exe)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "whole:" in r.stdout and "tiled:" in r.stdout
