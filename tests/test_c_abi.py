"""The boundary from plain C: tests/abi_c_driver.c, a C99 program with no
Python or torch in its process, includes include/dfpr.h, links the built
library and runs load, Static, apply, Dynamic Frontier and Naive-dynamic
plus the error returns.  On the CPU it must compile and link; on the GPU
its ranks must match the oracle's within 1e-9 and its counts exactly."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2401_03256_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2401_03256_amd")
LIB = os.path.join(PKG, "libdfpr.so")
DRIVER = os.path.join(ROOT, "tests", "abi_c_driver.c")
TOL_RANK = 1e-9


def _build(out):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    if not os.path.exists(LIB):
        pytest.skip("libdfpr.so not built (run __graft_entry__.build())")
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    cmd = [gcc, "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
           DRIVER, "-L", PKG, "-ldfpr", f"-Wl,-rpath,{PKG}", f"-Wl,-rpath-link,{rocm_lib}",
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]


def test_c_caller_compiles_and_links(tmp_path):
    _build(str(tmp_path / "drv"))


def _write_pairs(f, a, b):
    for u, v in zip(a.tolist(), b.tolist()):
        f.write(f"{u} {v}\n")


@pytest.mark.gpu
def test_c_caller_matches_oracle(tmp_path):
    drv = str(tmp_path / "drv")
    _build(drv)
    n, src, dst = synth.rmat(12, 16, seed=31)
    b = synth.random_batch(src, dst, n, 30, 120, seed=32)
    with open(tmp_path / "edges.txt", "w") as f:
        f.write(f"{n} {src.size}\n")
        _write_pairs(f, src, dst)
    with open(tmp_path / "batch.txt", "w") as f:
        f.write(f"{b.del_src.size} {b.ins_src.size}\n")
        _write_pairs(f, b.del_src, b.del_dst)
        _write_pairs(f, b.ins_src, b.ins_dst)
    prefix = str(tmp_path / "out")
    sys.stdout.write(f"\n[case] C driver on R-MAT scale 12, batch of {b.size}\n")
    sys.stdout.flush()
    r = subprocess.run([drv, str(tmp_path / "edges.txt"), str(tmp_path / "batch.txt"), prefix],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    f = r.stdout.split()
    got = {f[i]: f[i + 1:i + 3] if f[i] == "applied" else f[i + 1] for i in range(0, len(f))
           if f[i] in ("n", "m", "applied", "m_after", "df_affected")}
    o = oracle.OracleGraph(n, src, dst)
    assert int(got["m"]) == o.m
    Ro, _ = o.static()
    applied = o.apply_batch(b)
    assert (int(got["applied"][0]), int(got["applied"][1])) == tuple(applied)
    assert int(got["m_after"]) == o.m
    Rd, _ = o.dynamic_frontier(b, Ro)
    Rn, _ = o.naive_dynamic(Ro)
    for tag, ref in (("static", Ro), ("df", Rd), ("naive", Rn)):
        R = np.loadtxt(f"{prefix}.{tag}")
        assert R.shape == (n,)
        assert np.max(np.abs(R - ref)) < TOL_RANK, tag
