"""The C ABI's host paths under AddressSanitizer + LeakSanitizer (no GPU).

asan_host_paths.cpp drives etm_plan_create (valid plans and each class of
rejected input), etm_plan_footprint / _dt / _dofs / _destroy and
etm_batch_create with well-formed and malformed tuning JSON.  The library
sources are compiled here with the host side instrumented (device code is
compiled as usual and never launched) and linked into one executable, which
must finish with no sanitizer report and no leak.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2603_07038_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["em.hip", "mech.hip", "mg.hip", "batch.hip", "plan.cpp"]
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
         "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_paths_clean_under_asan(tmp_path):
    def compile_one(src):
        path = os.path.join(HERE, src) if src.endswith("asan_host_paths.cpp") else os.path.join(CSRC, src)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([HIPCC] + FLAGS + lang + ["-c", path, "-o", obj], capture_output=True, text=True,
                           timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES) + 1) as ex:
        objs = list(ex.map(compile_one, SOURCES + ["asan_host_paths.cpp"]))
    exe = str(tmp_path / "asan_host_paths")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-o", exe] + objs
                       + ["-lrocprofiler-sdk-roctx"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:exitcode=99")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "ALL OK" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-6000:])
    assert "AddressSanitizer" not in r.stderr and "LeakSanitizer" not in r.stderr, r.stderr[-6000:]
