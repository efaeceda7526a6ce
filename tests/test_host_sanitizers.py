"""The library's host code (validation, workspace planning, table building and
carving) built with AddressSanitizer and UndefinedBehaviorSanitizer and
driven over many synthetic trees by tests/host_checks/planning_driver.cpp.

Only the host pass is instrumented (-Xarch_host before each -fsanitize=); the
kernels are the library's own objects.  No device is touched: the driver
stops every factorization at its device check, after validation, planning
and carving.
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1602_01376_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "host_checks", "planning_driver.cpp")
HIPCC = "/opt/rocm/bin/hipcc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all"]
COMMON = ["-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC",
          "-Wno-unused-command-line-argument", "-Wno-unused-value",
          "-I", os.path.join(ROOT, "include")]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_planning_under_address_and_ub_sanitizers(tmp_path):
    kernels = sorted(glob.glob(os.path.join(ROOT, "_build", "kernels_*.o")))
    if len(kernels) < 5:
        from paper_1602_01376_amd import build
        build.build()
        kernels = sorted(glob.glob(os.path.join(ROOT, "_build", "kernels_*.o")))
    # the kernels' objects carry their own code objects; a copy keeps a
    # concurrent rebuild from changing them under the link
    local = []
    for k in kernels:
        dst = tmp_path / os.path.basename(k)
        shutil.copyfile(k, dst)
        local.append(str(dst))
    lib_o = str(tmp_path / "invaskit_san.o")
    drv_o = str(tmp_path / "driver.o")
    exe = str(tmp_path / "planning_driver")
    _run([HIPCC, "-x", "hip", "--offload-arch=gfx950", *COMMON, *SAN, "-c",
          os.path.join(CSRC, "invaskit.cpp"), "-o", lib_o])
    _run([HIPCC, "-x", "hip", "--offload-host-only", *COMMON, *SAN, "-c", DRIVER,
          "-o", drv_o])
    _run([HIPCC, *SAN, "-Wno-unused-command-line-argument", drv_o, lib_o, *local, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, f"rc={r.returncode}\n{r.stdout[-4000:]}\n{r.stderr[-6000:]}"
    assert "0 failure(s)" in r.stdout
