"""The serving loop's admission rule on the CPU: serve_policy_driver.cpp
drives next_admission (paper_2401_03256_amd/csrc/serve_policy.h, the
function the server calls) with a fake clock and a mock budget, built with
g++ and AddressSanitizer/UndefinedBehaviorSanitizer."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2401_03256_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_admission_rule(tmp_path):
    exe = str(tmp_path / "serve_policy")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-Wall", "-Wextra", "-Werror",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", CSRC,
                    os.path.join(HERE, "serve_policy_driver.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip() == "ok"
