"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
tests/oracle_sanitize_check.c links oracle/sw_oracle.c and drives every entry point; any
out-of-bounds access, undefined operation or leak ends it with an error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_check")
    flags = ["-O1", "-g", "-std=c99", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]
    subprocess.run(["gcc", *flags, "-o", exe, os.path.join(ROOT, "tests", "oracle_sanitize_check.c"),
                    os.path.join(ORACLE, "sw_oracle.c")], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.startswith("ok: 18000 pair checks")
