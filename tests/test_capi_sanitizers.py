"""The C ABI's host code under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer (CPU, no device).

tests/capi_sanitize_driver.cpp calls the host side of every entry point that
can run without a device: status strings, workspace sizing over a grid of
valid and invalid parameters (enum fields out of range included), NULL
handles and bad arguments, and chain, engine and allocation-free calls that
pass validation and then fail at their first device call.  The library's
sources are built here with the sanitizers on the host pass only (the device
code is compiled as usual and never runs); the driver must run clean, and its
output must equal that of the same driver linked against the product
library (the sanitizers change no result).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1303_6016_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "capi_sanitize_driver.cpp")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["gfmc_kernels.hip", "gfmc_capi.hip", "gfmc_engine.hip", "gfmc_probe.hip"]
BASE = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# host pass only: the device code is never run here
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _no_device_env():
    env = dict(os.environ)
    env["HIP_VISIBLE_DEVICES"] = "-1"
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=24"
    return env


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc missing")
def test_capi_host_code_runs_clean_under_sanitizers(tmp_path):
    tmp = str(tmp_path)
    jobs = []
    objs = []
    for s in SOURCES:
        o = os.path.join(tmp, s.replace(".hip", ".o"))
        objs.append(o)
        jobs.append(subprocess.Popen([HIPCC, *BASE, *SAN, "-c", os.path.join(CSRC, s), "-o", o],
                                     stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    drv_o = os.path.join(tmp, "driver.o")
    jobs.append(subprocess.Popen([HIPCC, *BASE, *SAN, "--cuda-host-only", "-x", "hip", "-c", DRIVER,
                                  "-o", drv_o], stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for j in jobs:
        out, _ = j.communicate(timeout=600)
        assert j.returncode == 0, out.decode(errors="replace")[-2000:]
    san_exe = os.path.join(tmp, "driver_san")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", *SAN[:4], "-o", san_exe, drv_o, *objs])

    # the same driver against the product library (plain build)
    lib_dir = os.path.join(ROOT, "paper_1303_6016_amd")
    if not os.path.exists(os.path.join(lib_dir, "libgfmc.so")):
        pytest.skip("libgfmc.so not built")
    plain_o = os.path.join(tmp, "driver_plain.o")
    plain_exe = os.path.join(tmp, "driver_plain")
    subprocess.check_call([HIPCC, *BASE, "--cuda-host-only", "-x", "hip", "-c", DRIVER,
                           "-o", plain_o])
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-o", plain_exe, plain_o,
                           "-L", lib_dir, "-lgfmc", "-Wl,-rpath," + lib_dir])

    env = _no_device_env()
    san = subprocess.run([san_exe], capture_output=True, text=True, timeout=300, env=env)
    if san.returncode == 3:
        pytest.skip("a device is visible")
    print(san.stdout)
    assert san.returncode == 0, san.stdout[-3000:] + san.stderr[-3000:]
    assert "driver: clean" in san.stdout
    assert "runtime error" not in san.stderr and "ERROR: AddressSanitizer" not in san.stderr
    plain = subprocess.run([plain_exe], capture_output=True, text=True, timeout=300, env=env)
    assert plain.returncode == 0, plain.stdout[-3000:] + plain.stderr[-3000:]
    assert plain.stdout == san.stdout
