"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer: every
entry point on small random inputs with buffers of exactly the documented
sizes (tests/oracle_asan_check.c)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_asan_check")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "vref.c"),
           os.path.join(ROOT, "tests", "oracle_asan_check.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert r.stdout.strip().endswith("OK")
