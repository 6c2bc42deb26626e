"""Parity at full size, in the launch configuration the bench times.

R-MAT scale 22 (4,194,304 vertices, about 6.9e7 edges with self-loops),
R-MAT scale 24 (16,777,216 vertices, about 2.8e8 edges, the precision
form's workload), the 4096 x 4096 grid with 5% diagonal shortcuts
(16,777,216 vertices) and the serving form's twelve resident R-MAT graphs
(scales 16 to 22): the HIP library against the oracle on the same seeded
inputs.  CSRs and initial markings bit-exact; FP64 ranks within
1e-9 L-inf, each side starting from its own previous ranks.  The oracle
runs on the host cores, so these cases take tens of seconds to a few
minutes each.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2401_03256_amd import synth
from markcheck import check_final_marks

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
        Ro, sto, _, f1, ch = o.dynamic_frontier(b, Ro, frontier_tol=FTOL, return_flags=True,
                                                return_changes=True)
        assert st.converged and sto.converged
        assert abs(st.iterations - sto.iterations) <= 1
        assert np.max(np.abs(R - Ro)) < TOL_RANK, f"batch {i}"
        assert abs(st.affected_initial - sto.affected_initial) == 0
        check_final_marks(g.affected(), f1, ch, *o.csr(out=False), FTOL, f"{tag} batch {i}",
                          st.iterations == sto.iterations)
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


# FP32 phase of the precision form against as many FP64 iterations of the
# oracle.  A stored FP32 contribution carries a relative rounding error of
# at most u = 2^-24 and the Kahan row sum adds at most 2u (Kahan 1965;
# Higham, Accuracy and Stability of Numerical Algorithms, 4.3), all terms
# being positive.  One iteration thus moves a rank by at most 3u of itself
# on top of the relative error of its inputs, and k iterations (plus the
# initial rounding of the contributions) by at most (3k + 1) u of the rank.
# In L1 the iteration contracts by alpha, so the L1 error stays below
# (3 + 1) u / (1 - alpha).  A vertex may also be processed on one side only
# when a rank change lies within rounding of the frontier tolerance; the
# change such a vertex misses is of the order of that tolerance, allowed for
# by an absolute term of 10 tau_f per vertex.
U32 = 2.0 ** -24


def _fp32_phase_bounds(k, alpha=0.85):
    return (3 * k + 1) * U32, 4 * U32 / (1 - alpha)


def test_rmat24_fp64_and_fp32_form(dfpr):
    # batches of 1e-6 and 1e-4 |E|, each side from its own previous ranks:
    # FP64 Dynamic Frontier and the FP32 storage form (FP32 phase + FP64
    # refinement) from the same previous ranks, both within 1e-9 of the
    # oracle; the FP32 phase alone against as many FP64 iterations of the
    # oracle, within the rounding bounds above and the 1e-6 gate
    n, src, dst = synth.rmat(24, 16, seed=1)
    _say(f"rmat24: generated, {src.size} edges")
    g = dfpr.Graph(n, src, dst)
    o = oracle.OracleGraph(n, src, dst)
    m = o.m
    batches = synth.batch_sequence(src, dst, n, [synth.batch_counts(f, m) for f in (1e-6, 1e-4)],
                                   seed=2)
    del src, dst
    p64 = dfpr.params(frontier_tol=FTOL)
    p32 = dfpr.params(frontier_tol=FTOL, precision=dfpr.FP32_KAHAN)
    R0, st = g.static(p64)
    Ro, sto = o.static()
    _say(f"rmat24: static {st.iterations} it (oracle {sto.iterations})")
    assert np.max(np.abs(R0 - Ro)) < TOL_RANK
    for b in batches:
        _say(f"rmat24: batch of {b.size} edges")
        assert g.apply_batch(b) == o.apply_batch(b)
        assert np.array_equal(g.mark_affected(b), o.mark_initial(b))
        R32, s32 = g.dynamic_frontier(b, p=p32)
        k32 = s32.iterations - s32.refine_sweeps
        g.set_ranks(R0)
        R32p, s32p = g.dynamic_frontier(
            b, p=dfpr.params(frontier_tol=FTOL, precision=dfpr.FP32_KAHAN, max_iters=k32))
        g.set_ranks(R0)
        R64, s64 = g.dynamic_frontier(b, p=p64)
        _say(f"rmat24: FP64 {s64.iterations} it, FP32 form {s32.iterations} it "
             f"({s32.refine_sweeps} refinement sweeps); oracle")
        Rd, sd = o.dynamic_frontier(b, Ro, frontier_tol=FTOL)
        Rk, _ = o.dynamic_frontier(b, Ro, frontier_tol=FTOL, max_iters=k32)
        assert s64.converged and s32.converged and sd.converged
        assert abs(s64.iterations - sd.iterations) <= 1
        assert s64.affected_initial == sd.affected_initial
        err = {"fp64": R64 - Rd, "fp32 form": R32 - Rd, "fp32 phase": R32p - Rk}
        for k_, e in err.items():
            _say(f"rmat24 {b.size}: {k_} vs oracle: Linf {np.max(np.abs(e)):.3e}, "
                 f"L1 {np.sum(np.abs(e)):.3e}")
        assert np.max(np.abs(R64 - Rd)) < TOL_RANK
        assert np.max(np.abs(R32 - Rd)) < TOL_RANK
        assert s32p.iterations == k32 and s32p.refine_sweeps == 0
        rel_bound, l1_bound = _fp32_phase_bounds(k32)
        e = np.abs(R32p - Rk)
        rel = e / Rk
        _say(f"rmat24 {b.size}: fp32 phase ({k32} it) max rel {np.max(rel):.3e} "
             f"(bound {rel_bound:.3e}), L1 {np.sum(e):.3e} (bound {l1_bound:.3e})")
        assert np.max(e) < 1e-6
        assert np.all(e <= rel_bound * Rk + 10 * FTOL)
        assert np.sum(e) <= l1_bound
        R0, Ro = R64, Rd
    _say("rmat24: CSRs")
    _same_csr(g, o)


def test_grid4096_uniform_and_localised(dfpr):
    side = 4096
    n, src, dst = synth.grid2d(side, 0.05, seed=1)
    g = dfpr.Graph(n, src, dst)
    o = oracle.OracleGraph(n, src, dst)
    nd, ni = synth.batch_counts(1e-5, o.m)
    uni = synth.batch_sequence(src, dst, n, [(nd, ni)], seed=2)
    loc = [synth.localized_batch(src, dst, side, nd, ni, seed=10)]
    _run_sequence(dfpr, g, o, uni + loc, "grid4096")


def test_serving_twelve_graphs_alone_and_in_the_mix(dfpr):
    # the serving workload's graphs (R-MAT scales 16, 18, 20, 22, three
    # seeds each, FP32 storage on the second seed of every scale) and 24
    # requests of log-uniform size in [1e-7, 1e-3] |E| for uniformly chosen
    # graphs, all arriving at once: every served result equals the plain
    # calls one at a time, bitwise (FP64 and FP32 graphs); the graphs of
    # scales 16 and 18 are replayed by the oracle, within 1e-9
    rng = synth.rng_for(71)
    work = []
    for sc in (16, 18, 20, 22):
        for k in range(3):
            n, s_, d_ = synth.rmat(sc, 16, seed=100 + 10 * sc + k)
            work.append([sc, n, s_, d_, dfpr.FP32_KAHAN if k == 1 else dfpr.FP64, []])
    nreq = 24
    gids = rng.integers(0, len(work), size=nreq)
    fracs = np.exp(np.log(1e-7) + rng.random(nreq) * (np.log(1e-3) - np.log(1e-7)))
    for gi, w in enumerate(work):
        _, n, s_, d_, _, bl = w
        ks = [k for k in range(nreq) if gids[k] == gi]
        counts = [synth.batch_counts(fracs[k], s_.size + n) for k in ks]
        bl.extend(zip(ks, synth.batch_sequence(s_, d_, n, counts, seed=300 + gi)))
    _say(f"serving: 12 graphs generated, requests per graph {np.bincount(gids, minlength=12).tolist()}")
    p0 = dfpr.params(frontier_tol=FTOL)
    pg = [dfpr.params(frontier_tol=FTOL, precision=w[4]) for w in work]
    # one at a time through the plain calls
    alone_R, alone_it = [], {}
    for w, p in zip(work, pg):
        g = dfpr.Graph(w[1], w[2], w[3])
        g.static(p0, out=False)
        for k, b in w[5]:
            g.apply_batch(b)
            _, st = g.dynamic_frontier(b, p=p, out=False)
            alone_it[k] = st.iterations
        alone_R.append(g.ranks())
        g.close()
    _say("serving: one at a time done")
    # the same requests through the server
    srv = dfpr.Server(max_slots=8, hbm_budget_bytes=200 << 30)
    graphs = []
    for w, p in zip(work, pg):
        g = dfpr.Graph(w[1], w[2], w[3])
        g.static(p0, out=False)
        graphs.append((g, srv.add_graph(g, p)))
    rid = {}
    for k in range(nreq):
        gi = int(gids[k])
        b = dict(work[gi][5])[k]
        rid[k] = srv.submit(graphs[gi][1], 0.0, b)
    st = srv.run()
    _say(f"serving: served, max active {st['max_active']}, steps {st['steps']}")
    assert st["completed"] == nreq and st["failed"] == 0 and st["max_active"] > 1
    for k in range(nreq):
        r = srv.result(rid[k])
        assert r["status"] == 0 and r["converged"] and r["iterations"] == alone_it[k]
    for gi, (g, _) in enumerate(graphs):
        assert np.array_equal(g.ranks(), alone_R[gi]), work[gi][0]
    # the oracle replays the small graphs
    for gi, w in enumerate(work):
        if w[0] > 18:
            continue
        o = oracle.OracleGraph(w[1], w[2], w[3])
        Ro, _ = o.static()
        for k, b in w[5]:
            o.apply_batch(b)
            Ro, sto = o.dynamic_frontier(b, Ro, frontier_tol=FTOL)
            assert sto.converged
        assert np.max(np.abs(alone_R[gi] - Ro)) < TOL_RANK, f"graph {gi}"
    srv.close()
    for g, _ in graphs:
        g.close()
