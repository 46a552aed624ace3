"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
host driver (tests/oracle_sanitize_main.c) runs the tracer, the projections of
every system-model option, the penalty, the objective and all five
preconditioner modes on small 2D and 3D geometries; any sanitizer report or
non-finite result fails."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-D_GNU_SOURCE", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
           os.path.join(HERE, "oracle_sanitize_main.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "oracle sanitize: ok" in res.stdout
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr
