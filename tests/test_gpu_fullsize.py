"""Parity at full size, in the launch configuration the bench times.

R-MAT scale 22 (4,194,304 vertices, about 6.9e7 edges with self-loops)
and the 4096 x 4096 grid with 5% diagonal shortcuts (16,777,216 vertices):
the HIP library against the oracle on the same seeded inputs.  CSRs and
initial markings bit-exact; ranks within 1e-9 L-inf, each side starting
from its own previous ranks.  The oracle runs on the host cores, so these
cases take tens of seconds each.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2401_03256_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TOL_RANK = 1e-9
FTOL = 1e-13


@pytest.fixture(scope="module")
def dfpr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2401_03256_amd import dfpr as mod
    mod.lib()
    return mod


def _say(msg):
    sys.stdout.write(f"\n[case] {msg}\n")
    sys.stdout.flush()


def _same_csr(g, o):
    for out in (True, False):
        a_off, a_idx = g.csr(out)
        b_off, b_idx = o.csr(out)
        assert np.array_equal(a_off, b_off), f"offsets differ (out={out})"
        assert np.array_equal(a_idx, b_idx), f"indices differ (out={out})"


def _run_sequence(dfpr, g, o, batches, tag):
    p = dfpr.params(frontier_tol=FTOL)
    R0, st = g.static(p)
    Ro, sto = o.static()
    _say(f"{tag}: static {st.iterations} it (oracle {sto.iterations})")
    assert np.max(np.abs(R0 - Ro)) < TOL_RANK
    for i, b in enumerate(batches):
        _say(f"{tag}: batch {i}, {b.size} edges")
        assert g.apply_batch(b) == o.apply_batch(b)
        assert np.array_equal(g.mark_affected(b), o.mark_initial(b))
        R, st = g.dynamic_frontier(b, p=p)
        Ro, sto = o.dynamic_frontier(b, Ro, frontier_tol=FTOL)
        assert st.converged and sto.converged
        assert abs(st.iterations - sto.iterations) <= 1
        assert np.max(np.abs(R - Ro)) < TOL_RANK, f"batch {i}"
        assert abs(st.affected_initial - sto.affected_initial) == 0
    _same_csr(g, o)
    return Ro


def test_rmat22_static_and_dynamic_frontier(dfpr):
    n, src, dst = synth.rmat(22, 16, seed=1)
    g = dfpr.Graph(n, src, dst)
    o = oracle.OracleGraph(n, src, dst)
    _same_csr(g, o)
    m = o.m
    counts = [synth.batch_counts(f, m) for f in (1e-7, 1e-5, 1e-3)]
    batches = synth.batch_sequence(src, dst, n, counts, seed=2)
    Ro = _run_sequence(dfpr, g, o, batches, "rmat22")
    # Dynamic Traversal on one more batch, each side from its own ranks
    b = synth.random_batch(src, dst, n, *counts[1], seed=3)
    _say("rmat22: dynamic traversal")
    assert g.apply_batch(b) == o.apply_batch(b)
    assert np.array_equal(g.mark_reachable(b), o.mark_reachable(b))
    R, st = g.dynamic_traversal(b, p=dfpr.params(frontier_tol=FTOL))
    Rt, sto = o.dynamic_traversal(b, Ro)
    assert st.converged and st.affected_final == sto.affected_final
    assert np.max(np.abs(R - Rt)) < TOL_RANK


def test_grid4096_uniform_and_localised(dfpr):
    side = 4096
    n, src, dst = synth.grid2d(side, 0.05, seed=1)
    g = dfpr.Graph(n, src, dst)
    o = oracle.OracleGraph(n, src, dst)
    nd, ni = synth.batch_counts(1e-5, o.m)
    uni = synth.batch_sequence(src, dst, n, [(nd, ni)], seed=2)
    loc = [synth.localized_batch(src, dst, side, nd, ni, seed=10)]
    _run_sequence(dfpr, g, o, uni + loc, "grid4096")
