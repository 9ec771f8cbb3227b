"""The serving loop's host code under ThreadSanitizer (CPU only).

Builds the library's sources with the host half instrumented (-Xarch_host, device code
unchanged) and runs tests/tsan/server_race.cpp: concurrent submitters, waiters and a
completion drain against a simulated device.  No race report and no failed request
are allowed.  Skipped where hipcc or clang++ is missing.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/lib/llvm/bin/clang++"


@pytest.mark.slow
def test_server_under_tsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc / clang++ not available")
    from paper_1612_05778_amd.build import SOURCES, CSRC
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=thread", "-x", "hip", "-c", os.path.join(CSRC, src),
               "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "drv.o")
    r = subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=thread",
                        "-I", os.path.join(ROOT, "include"), "-c",
                        os.path.join(HERE, "tsan", "server_race.cpp"), "-o", drv],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "server_race")
    r = subprocess.run([CLANG, "-fsanitize=thread", drv, *objs, "-o", exe,
                        "-L/opt/rocm/lib", "-lamdhip64", "-lpthread",
                        "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout + r.stderr)[-2000:]
