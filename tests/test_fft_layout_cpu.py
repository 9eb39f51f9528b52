"""Host emulation of the GPU FFT building blocks (no GPU needed).

tests/cpu/fft_layout_emu.cpp includes the device header fft.hpp, runs each
transform with one host thread per GPU thread, and checks the digit-reversed
storage order against the plain DFT for every supported length.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
def test_block_fft_index_math(tmp_path):
    exe = tmp_path / "fft_layout_emu"
    cmd = ["g++", "-std=c++20", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "paper_1706_02261_amd", "csrc"),
           os.path.join(HERE, "cpu", "fft_layout_emu.cpp"), "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0 and "ALL OK" in r.stdout
