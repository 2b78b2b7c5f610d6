"""The oracle under gcc's address and undefined-behaviour sanitizers: a
driver (oracle/sanitize_main.c) calls every oracle entry point on tiny
problems -- both solvers with and without a preconditioner, every fault-plan
shape, truncated logs and histories, invalid arguments, the octahedral mesh
-- and any out-of-bounds access, leak or undefined operation in the oracle
fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not on PATH")
def test_oracle_runs_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    src = [os.path.join(ROOT, "oracle", "sanitize_main.c"), os.path.join(ROOT, "oracle", "ftgcr_oracle.c")]
    flags = ["-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-Wall", "-Wextra", "-Werror"]
    subprocess.run(["gcc", *flags, "-o", str(exe), *src, "-lm"], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    assert "all entry points ran clean" in r.stdout
