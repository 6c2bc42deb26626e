"""The C-ABI library loads and exports every entry point that include/dfpr.h
declares (no GPU needed: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dfpr.h")
LIB = os.path.join(ROOT, "paper_2401_03256_amd", "libdfpr.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dfpr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_method_calls():
    syms = declared_symbols()
    for name in ("dfpr_load_graph", "dfpr_apply_batch", "dfpr_pagerank_static",
                 "dfpr_pagerank_naive_dynamic", "dfpr_pagerank_dynamic_frontier"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdfpr.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdfpr.so not built")
def test_binding_lists_every_declared_symbol():
    from paper_2401_03256_amd import dfpr
    assert sorted(dfpr.EXPORTED) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdfpr.so not built")
def test_params_defaults_match_the_paper():
    from paper_2401_03256_amd import dfpr
    p = dfpr.params()
    assert p.alpha == 0.85 and p.tol == 1e-10 and p.max_iters == 500
    assert p.frontier_tol == pytest.approx(1e-15)
    assert p.precision == dfpr.FP64


def test_library_is_built_for_gfx950():
    if not os.path.exists(LIB):
        pytest.skip("libdfpr.so not built")
    data = open(LIB, "rb").read()
    assert b"gfx950" in data


def test_bench_refuses_more_than_one_gpu():
    # the benchmark measures one GPU; asking for more ends at argument
    # checking, before any device is touched
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_binding_rejects_ragged_batches():
    # the library reads n_del (n_ins) entries from both arrays of a side, so
    # the binding refuses arrays of different lengths before any call
    import numpy as np
    from paper_2401_03256_amd import dfpr, synth
    z = np.zeros(0, np.int32)
    ok = synth.Batch(np.array([1, 2], np.int32), np.array([3, 4], np.int32), z, z)
    assert [a.size for a in dfpr._batch_arrays(ok)] == [2, 2, 0, 0]
    for bad in (synth.Batch(np.array([1, 2], np.int32), np.array([3], np.int32), z, z),
                synth.Batch(z, z, np.array([5], np.int32), z),
                synth.Batch(z, z, np.zeros((1, 1), np.int32), np.zeros((1, 1), np.int32))):
        with pytest.raises(ValueError):
            dfpr._batch_arrays(bad)
