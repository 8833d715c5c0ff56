"""The host runtime's device-free paths under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only): tests/host_plan_driver.cpp,
built with the sanitizers on the host side of the compile, plans 300
random descriptors (uneven meshes, per-cell networks, both lattices, both
signalling kinds, with and without S), every chi launch plan of each
(modes 0..4, regroup off/on/automatic, small and full devices), batch
layouts with repeated members, and 22 descriptors broken one field at a
time; any report aborts it, and it checks that every cell lands in exactly
one work item of every plan."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1806_10889_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(os.path.join(PKG, "libtissue.so"))),
                    reason="needs hipcc and the built library")
def test_host_plans_clean_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "driver")
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
               "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-x", "hip", os.path.join(ROOT, "tests", "host_plan_driver.cpp"),
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all",
               "-I", os.path.join(ROOT, "include"), "-L", PKG, "-ltissue", "-lhiprtc",
               f"-Wl,-rpath,{PKG}", "-o", exe]
        b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert b.returncode == 0, b.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env, cwd=d)
        assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
        print(r.stdout)
        assert "failures 0" in r.stdout and "broken descriptors rejected: 22" in r.stdout
