"""Host build of the FFT building blocks and the real-to-complex pair-stage
bodies (the device code of fft.h and pair_phases.h, compiled by g++ against a
host stand-in for the HIP runtime header and run with one thread), checked
against naive DFTs written from the definitions: every radix plan of the pair
stage's grid sizes in both signs and plan orders, the forward in-plane
transform of a pair density, the inverse round trip, and the z pass with v(G)
including ragged last tiles (table-driven and per-element v(G) bitwise
equal)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_fft_and_plane_bodies_on_host(tmp_path):
    exe = str(tmp_path / "fft_check")
    src = os.path.join(HERE, "cpu_fft", "fft_check.cpp")
    build = subprocess.run(["g++", "-std=c++17", "-O2", "-I", os.path.join(HERE, "cpu_fft"), "-o", exe, src],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-4000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, run.stdout[-4000:]
    assert "FAIL" not in run.stdout
