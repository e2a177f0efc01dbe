"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the library's sources are compiled host-only with both sanitizers and linked
into tests/host_sanitize/footprint_main.cpp, which runs plan construction's
host layout over many geometries (see that file)."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_01342_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_plan_layout_under_asan_and_ubsan(tmp_path):
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-DPC_BUILD",
             f"-I{os.path.join(ROOT, 'include')}"] + SAN

    def compile_one(f):
        out = str(tmp_path / (f + ".o"))
        lang = ["-x", "hip"] if f.endswith(".hip") else []
        r = subprocess.run([HIPCC] + flags + lang + ["-c", os.path.join(CSRC, f), "-o", out],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return out

    main = os.path.join(ROOT, "tests", "host_sanitize", "footprint_main.cpp")
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    main_o = str(tmp_path / "footprint_main.o")
    r = subprocess.run([HIPCC] + flags + ["-c", main, "-o", main_o], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    exe = str(tmp_path / "footprint_main")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-fsanitize=address,undefined", main_o]
                       + objs + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-6000:])
    assert run.stdout.strip().endswith("ok")
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
