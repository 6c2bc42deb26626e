"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
oracle_sanitize_driver.c calls every oracle entry point on small seeded
graphs (including a one-vertex graph, a rejected batch and an empty batch),
built with gcc and both sanitizers, any report fatal.  The OpenMP pragmas
are left out of this build, so the loops run on one thread."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_runs_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-Wno-unknown-pragmas",
                    "-Werror", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", ORACLE,
                    os.path.join(HERE, "oracle_sanitize_driver.c"),
                    os.path.join(ORACLE, "dfpr_oracle.c"), "-lm", "-o", exe],
                   check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip() == "ok"
