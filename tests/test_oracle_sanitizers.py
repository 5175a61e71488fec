"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

oracle/sanitize_driver.c calls every oracle entry point on small lattices and
edge cases (L = 2, odd L, M = 2, K > M, both kernels, cap proposals, mixed
start vectors, every initialisation); built here with -fsanitize=address and
-fsanitize=undefined (no recovery), it must run clean, and its results must
equal those of the plain build bit for bit (the sanitizers change no
arithmetic).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle")


def _build(tmp, name, flags):
    exe = os.path.join(tmp, name)
    subprocess.check_call(["gcc", "-std=gnu11", "-g", *flags, "-I", ORC, "-o", exe,
                           os.path.join(ORC, "sanitize_driver.c"),
                           os.path.join(ORC, "gfmc_oracle.c"), "-lm"])
    return exe


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    plain = _build(str(tmp_path), "plain", ["-O1"])
    san = _build(str(tmp_path), "san", ["-O1", "-fsanitize=address,undefined",
                                        "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([san], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    p = subprocess.run([plain], capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stdout
    assert r.stdout == p.stdout
    assert "checksum" in r.stdout
