"""The FFT's in-register butterflies on the host (no GPU): fft_lds.h's
twiddled and plain DFTs of lengths 2-16, both signs, FP32 and FP64, built
host-only and checked against the DFT's definition in long double
(tests/host_fft/dft_check.cpp).  A wrong twiddle, sign or output index in
the even/odd split shows up as an O(1) error."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_01342_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_register_dfts_match_the_definition(tmp_path):
    src = os.path.join(ROOT, "tests", "host_fft", "dft_check.cpp")
    exe = str(tmp_path / "dft_check")
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "--cuda-host-only",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}", "-x", "hip", src,
                        "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stdout[-4000:]
    assert run.stdout.strip().endswith("ok")
