"""GPU parity: the HIP library against the CPU oracle on the same seeded
inputs.  Integer results (CSRs, applied counts, initial marks) must be
bit-exact; FP64 ranks must agree within 1e-9 in L-inf."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2401_03256_amd import synth
from markcheck import check_final_marks

pytestmark = pytest.mark.gpu

TOL_RANK = 1e-9       # FP64 ranks, L-inf


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


def _pair(dfpr, n, src, dst):
    return dfpr.Graph(n, src, dst), oracle.OracleGraph(n, src, dst)


def _same_csr(g, o):
    for out in (True, False):
        a_off, a_idx = g.csr(out)
        b_off, b_idx = o.csr(out)
        assert np.array_equal(a_off, b_off), f"offsets differ (out={out})"
        assert np.array_equal(a_idx, b_idx), f"indices differ (out={out})"


def _arr(pairs):
    if not pairs:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    a = np.array(pairs, dtype=np.int32)
    return a[:, 0].copy(), a[:, 1].copy()


def _batch(dels, ins):
    return synth.Batch(*_arr(dels), *_arr(ins))


# ---------------------------------------------------------------------------
# graph store and batch applier (bit-exact)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["gnm", "rmat12", "grid", "single"])
def test_load_matches_oracle(dfpr, case):
    _say(f"load {case}")
    if case == "gnm":
        n = 3000
        src, dst = synth.gnm(n, 20000, seed=1)
    elif case == "rmat12":
        n, src, dst = synth.rmat(12, 16, seed=2)
        # repeated edges and ids in any order are accepted
        src = np.concatenate([src, src[:500]])[::-1].copy()
        dst = np.concatenate([dst, dst[:500]])[::-1].copy()
    elif case == "grid":
        n, src, dst = synth.grid2d(40, 0.05, seed=3)
    else:
        n, src, dst = 1, np.zeros(0, np.int32), np.zeros(0, np.int32)
    g, o = _pair(dfpr, n, src, dst)
    assert g.m == o.m
    _same_csr(g, o)


def test_apply_messy_batches_match_oracle(dfpr):
    rng = np.random.default_rng(7)
    n = 500
    src, dst = synth.gnm(n, 4000, seed=5)
    g, o = _pair(dfpr, n, src, dst)
    for step in range(12):
        _say(f"messy batch {step}")
        k = int(rng.integers(0, 300))
        # deletions: mostly existing edges, some absent, some self-loops, repeats
        off, idx = o.csr(True)
        rows = np.repeat(np.arange(n), np.diff(off))
        pick = rng.integers(0, idx.size, k)
        ds, dd = rows[pick], idx[pick]
        ds = np.concatenate([ds, rng.integers(0, n, 20), np.arange(5)])
        dd = np.concatenate([dd, rng.integers(0, n, 20), np.arange(5)])
        is_ = rng.integers(0, n, k + 30)
        id_ = rng.integers(0, n, k + 30)
        is_ = np.concatenate([is_, is_[:10], ds[:5]])   # repeats, present edges, re-inserts
        id_ = np.concatenate([id_, id_[:10], dd[:5]])
        b = synth.Batch(ds.astype(np.int32), dd.astype(np.int32), is_.astype(np.int32),
                        id_.astype(np.int32))
        assert g.apply_batch(b) == o.apply_batch(b)
        assert g.m == o.m
        _same_csr(g, o)


def test_apply_forces_overflow_and_big_rows(dfpr):
    # a hub with a long in-row and out-row (beyond the LDS copy), then batches
    # far larger than the slack of the touched rows
    n = 12000
    leaves = np.arange(1, 9001, dtype=np.int32)
    src = np.concatenate([leaves, np.zeros(9000, np.int32), np.arange(9001, n - 1)])
    dst = np.concatenate([np.zeros(9000, np.int32), leaves, np.arange(9002, n)])
    g, o = _pair(dfpr, n, src, dst)
    _same_csr(g, o)
    rng = np.random.default_rng(3)
    for step in range(4):
        _say(f"overflow batch {step}")
        hub_del = rng.choice(leaves, 700, replace=False)
        new = rng.integers(9001, n, 3000).astype(np.int32)
        b = synth.Batch(
            np.concatenate([hub_del, np.zeros(300, np.int32)]).astype(np.int32),
            np.concatenate([np.zeros(700, np.int32), rng.choice(leaves, 300)]).astype(np.int32),
            np.concatenate([new, np.full(2500, 9005, np.int32)]),
            np.concatenate([np.zeros(3000, np.int32), rng.integers(0, n, 2500).astype(np.int32)]))
        assert g.apply_batch(b) == o.apply_batch(b)
        _same_csr(g, o)


def test_apply_row_growing_past_the_lds_copy(dfpr):
    # out-row of vertex 1 and in-row of vertex 2 start below the 4096 entries
    # a workgroup copies to LDS and take 3000 insertions in one batch: the
    # merge runs in rounds of 1024 entries and the rows outgrow the LDS copy
    # between rounds; deletions early in the rows, and rows with few changes,
    # ride along
    n = 9000
    a = np.arange(3, 3103, dtype=np.int32)
    src = np.concatenate([np.ones(3100, np.int32), a, np.arange(5000, 8999, dtype=np.int32)])
    dst = np.concatenate([a, np.full(3100, 2, np.int32), np.arange(5001, 9000, dtype=np.int32)])
    g, o = _pair(dfpr, n, src, dst)
    rng = np.random.default_rng(11)
    for step in range(2):
        _say(f"lds growth batch {step}")
        new = np.arange(3103 + 3000 * step, 3103 + 3000 * (step + 1), dtype=np.int32) % n
        new = new[(new != 1) & (new != 2)]
        dels = rng.choice(a[:50], 20, replace=False)
        b = synth.Batch(
            np.concatenate([np.ones(20, np.int32), dels]).astype(np.int32),
            np.concatenate([dels, np.full(20, 2, np.int32)]).astype(np.int32),
            np.concatenate([np.ones(new.size, np.int32), new, rng.integers(0, n, 40)]).astype(
                np.int32),
            np.concatenate([new, np.full(new.size, 2, np.int32), rng.integers(0, n, 40)]).astype(
                np.int32))
        assert g.apply_batch(b) == o.apply_batch(b)
        assert g.m == o.m
        _same_csr(g, o)


def test_apply_rejects_out_of_range_unchanged(dfpr):
    n = 100
    src, dst = synth.gnm(n, 400, seed=1)
    g, o = _pair(dfpr, n, src, dst)
    before = g.csr(True)
    with pytest.raises(dfpr.DfprError) as e:
        g.apply_batch(_batch([(0, 1)], [(3, n)]))
    assert e.value.code == dfpr.DFPR_E_RANGE
    after = g.csr(True)
    assert np.array_equal(before[1], after[1])
    _same_csr(g, o)


def test_apply_device_arrays(dfpr):
    import torch
    n = 2000
    src, dst = synth.gnm(n, 12000, seed=9)
    g, o = _pair(dfpr, n, src, dst)
    b = synth.random_batch(src, dst, n, 40, 160, seed=4)
    t = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in
         (b.del_src, b.del_dst, b.ins_src, b.ins_dst)]
    torch.cuda.synchronize()
    assert g.apply_batch_device(*t) == o.apply_batch(b) == (40, 160)
    _same_csr(g, o)


# ---------------------------------------------------------------------------
# marking (bit-exact)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_initial_marking_bit_exact(dfpr, seed):
    _say(f"marking seed {seed}")
    n, src, dst = synth.rmat(11, 8, seed=seed)
    g, o = _pair(dfpr, n, src, dst)
    b = synth.random_batch(src, dst, n, 25, 100, seed=seed + 10)
    g.apply_batch(b)
    o.apply_batch(b)
    f_gpu = g.mark_affected(b)
    f_ref = o.mark_initial(b)
    assert np.array_equal(f_gpu, f_ref)
    # marks are cleared afterwards: marking twice gives the same set
    assert np.array_equal(g.mark_affected(b), f_ref)


# ---------------------------------------------------------------------------
# ranks (FP64, 1e-9 L-inf)
# ---------------------------------------------------------------------------

def test_closed_form_star_on_gpu(dfpr):
    n, k = 5000, 1200      # the centre's rows exceed the per-group sizes
    leaves = np.arange(1, k + 1, dtype=np.int32)
    src = np.concatenate([np.zeros(k, np.int32), leaves])
    dst = np.concatenate([leaves, np.zeros(k, np.int32)])
    g = dfpr.Graph(n, src, dst)
    R, st = g.static(dfpr.params(tol=1e-15))
    D = 2 * (k + 1) + 0.85 * (k - 1)
    assert abs(R[0] - (k + 1) / n * (2 + 0.85 * (k - 1)) / D) < 1e-14
    assert np.max(np.abs(R[1:k + 1] - (k + 1) / n * 2 / D)) < 1e-14
    assert np.max(np.abs(R[k + 1:] - 1.0 / n)) < 1e-15


@pytest.mark.parametrize("case", ["c0", "rmat13", "grid"])
def test_static_and_naive_match_oracle(dfpr, case):
    _say(f"static {case}")
    if case == "c0":
        n = 10000
        src, dst = synth.gnm(n, 80000, seed=1)
    elif case == "rmat13":
        n, src, dst = synth.rmat(13, 16, seed=1)
    else:
        n, src, dst = synth.grid2d(60, 0.05, seed=2)
    g, o = _pair(dfpr, n, src, dst)
    R, st = g.static()
    Ro, sto = o.static()
    assert st.converged
    assert np.max(np.abs(R - Ro)) < TOL_RANK
    assert abs(st.iterations - sto.iterations) <= 1
    assert abs(math.fsum(R) - 1.0) < 1e-9
    b = synth.random_batch(src, dst, n, 20, 80, seed=3)
    g.apply_batch(b)
    o.apply_batch(b)
    Rn, stn = g.naive_dynamic()
    Rno, _ = o.naive_dynamic(Ro)
    assert stn.converged
    assert np.max(np.abs(Rn - Rno)) < TOL_RANK
    Rref, _ = o.reference()
    assert np.max(np.abs(Rn - Rref)) < TOL_RANK


def test_dynamic_frontier_config0(dfpr):
    # 10,000 vertices, 80,000 uniform edges + self-loops; one batch of 80
    # (64 new pairs, 16 deleted edges); alpha 0.85, tol 1e-10, tau_f 1e-13
    n = 10000
    src, dst = synth.gnm(n, 80000, seed=1)
    g, o = _pair(dfpr, n, src, dst)
    p = dfpr.params(tol=1e-10, frontier_tol=1e-13)
    R0, _ = g.static(p)
    R0o, _ = o.static()
    nd, ni = synth.batch_counts(80 / o.m, o.m)
    assert (nd, ni) == (16, 64)
    b = synth.random_batch(src, dst, n, nd, ni, seed=1)
    assert g.apply_batch(b) == o.apply_batch(b) == (16, 64)
    assert np.array_equal(g.mark_affected(b), o.mark_initial(b))
    R, st = g.dynamic_frontier(b, p=p)
    Ro, sto, f0, f1, ch = o.dynamic_frontier(b, R0o, frontier_tol=1e-13, return_flags=True,
                                             return_changes=True)
    assert st.converged and sto.converged
    assert st.affected_initial == sto.affected_initial == int(f0.sum())
    assert np.max(np.abs(R - Ro)) < TOL_RANK
    Rref, _ = o.reference()
    assert np.max(np.abs(R - Rref)) < TOL_RANK
    fg = g.affected()
    assert fg.sum() > 0 and np.all(fg >= f0)       # marks only grow
    check_final_marks(fg, f1, ch, *o.csr(out=False), 1e-13, "config 0",
                      st.iterations == sto.iterations)
    # the marking calls after the update do not change which marks the
    # update left: affected() still reports the Dynamic Frontier call's
    g.mark_affected(b)
    g.mark_reachable(b)
    assert np.array_equal(g.affected(), fg)
    # same work as the oracle up to marks that flip near tau_f
    assert abs(st.iterations - sto.iterations) <= 1
    assert abs(st.vertices_processed - sto.vertices_processed) <= 0.02 * sto.vertices_processed


def test_self_loop_only_rows_in_dense_mode(dfpr):
    # Rows whose only in-entry is the self-loop have a schedule bin of their
    # own on the full schedule.  Vertex 0 reaches 5000 vertices, so every
    # batch from it runs in dense mode.  Vertices 5001..5998 have no in-edge
    # but their self-loop; 4000 has one from 0 only.  The batches make 4000
    # and 5500 cross between one and two in-entries both ways (the schedule
    # must follow) and use self-loop-only vertices as sources and deletion
    # targets (they must be processed although no other row points at them).
    n = 6000
    src = np.concatenate([np.zeros(5000, np.int32), np.arange(5001, 5999, dtype=np.int32)])
    dst = np.concatenate([np.arange(1, 5001, dtype=np.int32), np.arange(1, 999, dtype=np.int32)])
    g, o = _pair(dfpr, n, src, dst)
    p = dfpr.params(tol=1e-10, frontier_tol=1e-13)
    g.static(p)
    Ro, _ = o.static()
    batches = [_batch([(0, 4000)], [(0, 5500), (5600, 10)]),
               _batch([(0, 5500)], [(5601, 20), (0, 4000)])]
    for k, b in enumerate(batches):
        _say(f"self-loop rows batch {k}")
        assert g.apply_batch(b) == o.apply_batch(b)
        R, st = g.dynamic_frontier(b, p=p)
        Ro, sto, f0, f1 = o.dynamic_frontier(b, Ro, frontier_tol=1e-13, return_flags=True)
        assert st.converged and sto.converged
        assert st.affected_initial == sto.affected_initial == int(f0.sum())
        assert np.max(np.abs(R - Ro)) < TOL_RANK
        Rref, _ = o.reference()
        assert np.max(np.abs(R - Rref)) < TOL_RANK
        fg = g.affected()
        for v in (4000, 5500, 5600, 5601):
            assert fg[v] == f1[v], v
        assert fg[4000] and fg[5500] and fg[5600 + k]


@pytest.mark.parametrize("cap", [1, 2, 3, 5, 8, 9, 13])
def test_iteration_cap_matches_oracle(dfpr, cap):
    # the host queues iterations in chunks ahead of the device's stop flag;
    # whatever the cap, exactly that many iterations run and the ranks are
    # the oracle's after as many iterations (Static, Naive-dynamic and
    # Dynamic Frontier, all stopped before convergence)
    _say(f"iteration cap {cap}")
    n = 2000
    src, dst = synth.gnm(n, 16000, seed=3)
    g, o = _pair(dfpr, n, src, dst)
    p = dfpr.params(max_iters=cap)
    R, st = g.static(p)
    Ro, sto = o.static(max_iters=cap)
    assert st.iterations == sto.iterations == cap and not st.converged
    assert np.max(np.abs(R - Ro)) < TOL_RANK
    R0, _ = o.static()
    b = synth.random_batch(src, dst, n, 40, 160, seed=4)
    g.apply_batch(b)
    o.apply_batch(b)
    Rn, stn = g.naive_dynamic(prev=R0, p=p)
    Rno, stno = o.naive_dynamic(R0, max_iters=cap)
    assert stn.iterations == stno.iterations == cap
    assert np.max(np.abs(Rn - Rno)) < TOL_RANK
    Rd, std = g.dynamic_frontier(b, prev=R0, p=p)
    Rdo, stdo = o.dynamic_frontier(b, R0, max_iters=cap)
    assert std.iterations == stdo.iterations == cap
    assert np.max(np.abs(Rd - Rdo)) < TOL_RANK


def test_dynamic_frontier_sequence_rmat(dfpr):
    n, src, dst = synth.rmat(13, 16, seed=4)
    g, o = _pair(dfpr, n, src, dst)
    R0, _ = g.static()
    Ro, _ = o.static()
    m = o.m
    counts = [synth.batch_counts(f, m) for f in (1e-4, 1e-3, 1e-2, 1e-4, 1e-3)]
    seq = synth.batch_sequence(src, dst, n, counts, seed=11)
    for i, b in enumerate(seq):
        _say(f"df sequence step {i}, batch {b.size}")
        assert g.apply_batch(b) == o.apply_batch(b)
        R, st = g.dynamic_frontier(b)
        Ro, sto = o.dynamic_frontier(b, Ro)
        assert st.converged
        assert np.max(np.abs(R - Ro)) < TOL_RANK
    Rref, _ = o.reference()
    assert np.max(np.abs(R - Rref)) < TOL_RANK
    _same_csr(g, o)


def test_dynamic_frontier_special_cases(dfpr):
    n = 3000
    src, dst = synth.gnm(n, 20000, seed=8)
    g = dfpr.Graph(n, src, dst)
    R0, _ = g.static()
    # empty batch: previous ranks come back unchanged after one iteration
    R, st = g.dynamic_frontier(synth.Batch.empty())
    assert np.array_equal(R, R0) and st.iterations == 1 and st.converged
    # out-of-range id: error, ranks untouched
    with pytest.raises(dfpr.DfprError):
        g.dynamic_frontier(_batch([], [(0, n)]))
    assert np.array_equal(g.ranks(), R0)
    # tau_f = inf: the final marks are the initial marks
    b = synth.random_batch(src, dst, n, 3, 9, seed=2)
    g.apply_batch(b)
    R1, st = g.dynamic_frontier(b, p=dfpr.params(frontier_tol=math.inf))
    assert st.affected_final == st.affected_initial
    # determinism: same start, same batch -> bitwise equal ranks
    Ra, _ = g.dynamic_frontier(b, prev=R0)
    Rb, _ = g.dynamic_frontier(b, prev=R0)
    assert np.array_equal(Ra, Rb)


def test_untouched_component_bitwise(dfpr):
    nA, nB = 3000, 2000
    sa, da = synth.gnm(nA, 20000, seed=1)
    sb, db = synth.gnm(nB, 12000, seed=2)
    n = nA + nB
    g = dfpr.Graph(n, np.concatenate([sa, sb + nA]), np.concatenate([da, db + nA]))
    R0, _ = g.static()
    b = synth.random_batch(sa, da, nA, 5, 20, seed=3)
    g.apply_batch(b)
    R, st = g.dynamic_frontier(b)
    assert np.array_equal(R[nA:], R0[nA:])
    assert not g.affected()[nA:].any()


def test_dynamic_frontier_device_entry(dfpr):
    import torch
    n, src, dst = synth.rmat(12, 16, seed=6)
    g, o = _pair(dfpr, n, src, dst)
    g.use_torch_stream()
    R0, _ = g.static()
    Ro, _ = o.static()
    b = synth.random_batch(src, dst, n, 10, 40, seed=5)
    t = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in
         (b.del_src, b.del_dst, b.ins_src, b.ins_dst)]
    assert g.apply_batch_device(*t) == o.apply_batch(b)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    st = g.dynamic_frontier_device(*t, out=out)
    torch.cuda.synchronize()
    Ro, _ = o.dynamic_frontier(b, Ro)
    assert np.max(np.abs(out.cpu().numpy() - Ro)) < TOL_RANK
    assert st.converged


# ---------------------------------------------------------------------------
# FP32 precision form
# ---------------------------------------------------------------------------

def test_fp32_form_reaches_fp64_tolerance(dfpr):
    n = 10000
    src, dst = synth.gnm(n, 80000, seed=1)
    g, o = _pair(dfpr, n, src, dst)
    p64 = dfpr.params(frontier_tol=1e-13)
    g.static(p64)
    R0o, _ = o.static()
    b = synth.random_batch(src, dst, n, 16, 64, seed=1)
    g.apply_batch(b)
    o.apply_batch(b)
    p32 = dfpr.params(frontier_tol=1e-13, precision=dfpr.FP32_KAHAN)
    R, st = g.dynamic_frontier(b, p=p32)
    Ro, _ = o.dynamic_frontier(b, R0o, frontier_tol=1e-13)
    assert st.converged and st.refine_sweeps >= 1
    assert np.max(np.abs(R - Ro)) < TOL_RANK
    assert abs(math.fsum(R) - 1.0) < 1e-6


def test_fp32_phase_alone_within_1e6(dfpr):
    # two iterations, both inside the FP32 phase, against the same two
    # iterations in FP64 from the same start
    n, src, dst = synth.rmat(12, 16, seed=3)
    g = dfpr.Graph(n, src, dst)
    g.static()
    R0 = g.ranks()
    b = synth.random_batch(src, dst, n, 20, 80, seed=4)
    g.apply_batch(b)
    R64, s64 = g.dynamic_frontier(b, prev=R0, p=dfpr.params(max_iters=2))
    R32, s32 = g.dynamic_frontier(b, prev=R0, p=dfpr.params(max_iters=2,
                                                            precision=dfpr.FP32_KAHAN))
    assert s32.iterations == 2 and s32.refine_sweeps == 0
    assert np.max(np.abs(R32 - R64)) < 1e-6
    assert np.max(np.abs(R32 - R64)) > 0.0          # the FP32 path really ran


def test_fp32_row_sum_is_compensated(dfpr):
    # Kahan's bound: |computed - exact| <= (2u + N u^2) sum|x|, u = 2^-24
    # (Higham, Accuracy and Stability of Numerical Algorithms, 4.3).  Vertex
    # 0 has in-edges from itself (contribution 1.0) and k leaves
    # (contribution 3e-8 each, just under half an FP32 ulp of 1.0).  Rows of
    # this length are summed by 64 lanes, lane 0 taking positions
    # 0, 64, 128, ...; plain FP32 addition would drop the 15 small terms that
    # follow 1.0 in lane 0, an error above the bound.
    k = 1000
    n = k + 1
    leaves = np.arange(1, k + 1, dtype=np.int32)
    g = dfpr.Graph(n, leaves, np.zeros(k, np.int32))     # in-star, centre 0
    R = np.full(n, 6e-8)
    R[0] = 1.0            # |out(0)| = 1 (self-loop), |out(leaf)| = 2
    g.set_ranks(R)
    x = np.concatenate([[np.float32(1.0)], np.full(k, np.float32(6e-8 / 2))]).astype(np.float32)
    u = 2.0 ** -24
    lane0 = x[::64]
    naive = np.float32(0.0)
    for t in lane0:
        naive = np.float32(naive + t)
    assert abs(float(naive) - math.fsum(lane0.astype(np.float64))) > (2 * u) * float(x.sum())
    p = dfpr.params(tol=0.0, max_iters=1, precision=dfpr.FP32_KAHAN)
    Rn, st = g.dynamic_frontier(synth.Batch(np.zeros(0, np.int32), np.zeros(0, np.int32),
                                            np.array([1], np.int32), np.array([0], np.int32)),
                                p=p)
    assert st.iterations == 1 and st.refine_sweeps == 0
    alpha = 0.85
    exact = (1 - alpha) / n + alpha * math.fsum(x.astype(np.float64))
    bound = alpha * (2 * u + len(x) * u * u) * math.fsum(np.abs(x).astype(np.float64))
    assert abs(Rn[0] - exact) <= bound + 4 * 2.0 ** -53 * exact


# ---------------------------------------------------------------------------
# serving form
# ---------------------------------------------------------------------------

def _serving_workload():
    specs = [("rmat", 10, 1, dfpr_mod_fp64), ("rmat", 11, 2, dfpr_mod_fp32),
             ("rmat", 12, 3, dfpr_mod_fp64), ("gnm", 5000, 4, dfpr_mod_fp64)]
    out = []
    for kind, size, seed, prec in specs:
        if kind == "rmat":
            n, s, d = synth.rmat(size, 16, seed=seed)
        else:
            n = size
            s, d = synth.gnm(n, 8 * n, seed=seed)
        m = s.size + n
        counts = [synth.batch_counts(f, m) for f in (1e-4, 1e-2, 1e-3, 3e-3)]
        out.append((n, s, d, prec, synth.batch_sequence(s, d, n, counts, seed=seed + 100)))
    return out


dfpr_mod_fp64, dfpr_mod_fp32 = 0, 1


def test_serving_results_equal_alone_and_in_the_mix(dfpr):
    work = _serving_workload()
    # alone: each graph's batches one after another through the plain calls
    alone = []
    for n, s, d, prec, batches in work:
        g = dfpr.Graph(n, s, d)
        p = dfpr.params(frontier_tol=1e-13, precision=prec)
        g.static(dfpr.params(frontier_tol=1e-13))
        its = []
        for b in batches:
            g.apply_batch(b)
            _, st = g.dynamic_frontier(b, p=p)
            its.append(st.iterations)
        alone.append((g.ranks(), its))
        g.close()
    # mix: the same requests, all arriving at once, through the server
    graphs = []
    srv = dfpr.Server(max_slots=4)
    for n, s, d, prec, batches in work:
        g = dfpr.Graph(n, s, d)
        g.static(dfpr.params(frontier_tol=1e-13))
        gid = srv.add_graph(g, dfpr.params(frontier_tol=1e-13, precision=prec))
        graphs.append((g, gid))
    rids = []
    for k in range(4):
        for (g, gid), (_, _, _, _, batches) in zip(graphs, work):
            rids.append((gid, k, srv.submit(gid, 0.0, batches[k])))
    st = srv.run()
    assert st["completed"] == len(rids) and st["failed"] == 0
    assert st["max_active"] > 1                    # requests really overlapped
    for gid, k, rid in rids:
        r = srv.result(rid)
        assert r["status"] == 0 and r["converged"]
        assert r["iterations"] == alone[gid][1][k]
    for (g, gid) in graphs:
        assert np.array_equal(g.ranks(), alone[gid][0])


def test_serving_large_lane_in_order_one_at_a_time(dfpr):
    # the same workload with half the graphs moved to the large lane (by
    # lowering its edge threshold): every result still equals the plain
    # calls bitwise, and the large lane runs its requests one at a time, in
    # arrival order, beside the coalesced small lane
    work = _serving_workload()
    alone = []
    for n, s, d, prec, batches in work:
        g = dfpr.Graph(n, s, d)
        p = dfpr.params(frontier_tol=1e-13, precision=prec)
        g.static(dfpr.params(frontier_tol=1e-13))
        for b in batches:
            g.apply_batch(b)
            g.dynamic_frontier(b, p=p)
        alone.append(g.ranks())
        g.close()
    graphs = []
    srv = dfpr.Server(max_slots=4)
    for n, s, d, prec, batches in work:
        g = dfpr.Graph(n, s, d)
        g.static(dfpr.params(frontier_tol=1e-13))
        graphs.append((g, g.m))
    threshold = sorted(m for _, m in graphs)[len(graphs) // 2]
    srv.set_large_edges(threshold)
    large = [m >= threshold for _, m in graphs]
    assert 0 < sum(large) < len(large)
    gids = [srv.add_graph(g, dfpr.params(frontier_tol=1e-13, precision=w[3]))
            for (g, _), w in zip(graphs, work)]
    rids = []
    for k in range(4):
        for gid, w in zip(gids, work):
            rids.append((gid, srv.submit(gid, 0.0, w[4][k])))
    st = srv.run()
    assert st["completed"] == len(rids) and st["failed"] == 0
    for gid, rid in rids:
        r = srv.result(rid)
        assert r["status"] == 0 and r["converged"]
    for (g, _), R in zip(graphs, alone):
        assert np.array_equal(g.ranks(), R)
    # large-lane requests: admitted in submission order (all arrive at 0),
    # each after the previous one finished
    big = [srv.result(rid) for gid, rid in rids if large[gid]]
    for a, b in zip(big, big[1:]):
        assert b["admit_ms"] >= a["done_ms"]
    # the small lane ran beside it
    small = [srv.result(rid) for gid, rid in rids if not large[gid]]
    assert any(s["admit_ms"] < big[-1]["done_ms"] and s["done_ms"] > big[0]["admit_ms"]
               for s in small)


def _hub_graph(n, hubs, fan_in, background, seed):
    # `hubs` vertices of in-degree fan_in (whole-workgroup rows), on top of
    # uniform background edges
    rng = np.random.default_rng(seed)
    hs = np.repeat(np.arange(hubs, dtype=np.int32), fan_in)
    hsrc = rng.integers(hubs, n, size=hs.size, dtype=np.int32)
    bs = rng.integers(0, n, size=background, dtype=np.int32)
    bd = rng.integers(0, n, size=background, dtype=np.int32)
    return np.concatenate([hsrc, bs]), np.concatenate([hs, bd])


@pytest.mark.parametrize("hubs", [7, 8])
def test_wide_kernels_block_rows_match(dfpr, hubs):
    # Full-schedule walks run in 8- or 12-wave workgroups whose 256-thread
    # sub-blocks sum two or three whole-workgroup rows at a time; with 7
    # such rows some sub-blocks have none.  Static against the oracle, and
    # Dynamic Frontier (4-wave class lists, then the 8-wave kernel) against
    # the serving loop's 4-wave kernel, bitwise
    _say(f"wide kernels, {hubs} whole-workgroup rows")
    n = 20000
    src, dst = _hub_graph(n, hubs, 3000, 120000, seed=40 + hubs)
    g, o = _pair(dfpr, n, src, dst)
    R0, s0 = g.static()
    Ro, _ = o.static()
    assert s0.converged and np.max(np.abs(R0 - Ro)) < TOL_RANK
    Rn, _ = g.naive_dynamic(None, p=dfpr.params())
    Rno, _ = o.naive_dynamic(Ro)
    assert np.max(np.abs(Rn - Rno)) < TOL_RANK
    g.set_ranks(R0)
    # a batch touching every hub: the first frontier takes the full schedule
    b = synth.Batch(np.zeros(0, np.int32), np.zeros(0, np.int32),
                    np.arange(hubs, 2 * hubs, dtype=np.int32), np.arange(hubs, dtype=np.int32))
    g2 = dfpr.Graph(n, src, dst)
    g2.static()
    assert g.apply_batch(b) == o.apply_batch(b)
    p = dfpr.params(tol=1e-14, frontier_tol=1e-16)
    Rd, sd = g.dynamic_frontier(b, prev=R0, p=p)
    assert sd.converged and sd.iterations > 12
    Rdo, _ = o.dynamic_frontier(b, Ro, tol=1e-14, frontier_tol=1e-16)
    assert np.max(np.abs(Rd - Rdo)) < TOL_RANK
    srv = dfpr.Server(max_slots=2)
    gid = srv.add_graph(g2, p)
    rid = srv.submit(gid, 0.0, b)
    st = srv.run()
    assert st["completed"] == 1 and srv.result(rid)["converged"]
    assert np.array_equal(g2.ranks(), Rd)
    srv.close()
    g.close()
    g2.close()


def test_serving_budget_limits_concurrency(dfpr):
    n, s, d = synth.rmat(10, 16, seed=5)
    gs = []
    for i in range(3):
        g = dfpr.Graph(n, s, d)
        g.static()
        gs.append(g)
    counts = [synth.batch_counts(1e-3, s.size + n)] * 2
    seq = synth.batch_sequence(s, d, n, counts, seed=6)
    # the resident bytes of the three graphs, from a server with no requests
    probe = dfpr.Server(max_slots=8, hbm_budget_bytes=1 << 40)
    for g in gs:
        probe.add_graph(g)
    resident = probe.run()["peak_bytes"]
    probe.close()
    # room for one request at a time: three graphs, all requests at t = 0
    srv = dfpr.Server(max_slots=8, hbm_budget_bytes=resident + 96 * seq[0].size + 8)
    ids = [srv.add_graph(g) for g in gs]
    rids = [srv.submit(gid, 0.0, seq[i % 2]) for i, gid in enumerate(ids)]
    st = srv.run()
    assert st["completed"] == 3 and st["max_active"] == 1
    assert st["peak_bytes"] <= resident + 96 * seq[0].size + 8
    ends = sorted((srv.result(r)["admit_ms"], srv.result(r)["done_ms"]) for r in rids)
    for (a0, e0), (a1, _) in zip(ends, ends[1:]):
        assert a1 >= e0                                # one at a time
    # a second run serves only the new request
    r4 = srv.submit(ids[0], 0.0, synth.Batch.empty())
    st = srv.run()
    assert st["completed"] == 1 and srv.result(r4)["iterations"] == 1
    # graphs that do not fit the budget are refused
    small = dfpr.Server(max_slots=2, hbm_budget_bytes=1024)
    with pytest.raises(dfpr.DfprError):
        small.add_graph(gs[0])


def test_serving_arrivals_one_writer_and_bad_requests(dfpr):
    n, s, d = synth.rmat(11, 16, seed=7)
    g = dfpr.Graph(n, s, d)
    g.static()
    counts = [synth.batch_counts(1e-3, s.size + n)] * 3
    seq = synth.batch_sequence(s, d, n, counts, seed=8)
    ref = dfpr.Graph(n, s, d)
    ref.static()
    for b in seq:
        ref.apply_batch(b)
        ref.dynamic_frontier(b)
    srv = dfpr.Server(max_slots=4)
    gid = srv.add_graph(g)
    arr = [0.0, 0.0, 30.0]
    bad = _batch([], [(0, n)])
    rids = [srv.submit(gid, arr[0], seq[0]), srv.submit(gid, arr[1], seq[1]),
            srv.submit(gid, 1.0, bad), srv.submit(gid, arr[2], seq[2])]
    st = srv.run()
    assert st["completed"] == 3 and st["failed"] == 1
    res = [srv.result(r) for r in rids]
    assert res[2]["status"] != 0                       # rejected, graph unchanged
    good = [res[0], res[1], res[3]]
    for r, a in zip(good, arr):
        assert r["status"] == 0 and r["admit_ms"] >= a
    for r0, r1 in zip(good, good[1:]):
        assert r1["admit_ms"] >= r0["done_ms"]         # one writer per graph
    assert np.array_equal(g.ranks(), ref.ranks())


# ---------------------------------------------------------------------------
# Dynamic Traversal (comparator)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["gnm", "rmat11", "grid", "dag"])
def test_reachable_set_bit_exact(dfpr, case):
    _say(f"reachable {case}")
    if case == "gnm":
        n = 3000
        src, dst = synth.gnm(n, 6000, seed=21)
    elif case == "rmat11":
        n, src, dst = synth.rmat(11, 4, seed=22)
    elif case == "grid":
        n, src, dst = synth.grid2d(64, 0.05, seed=23)
    else:
        # a forward-only random graph: small reachable sets
        n = 4000
        s0, d0 = synth.gnm(n, 8000, seed=24)
        src, dst = np.minimum(s0, d0), np.maximum(s0, d0)
        keep = src != dst
        src, dst = src[keep], dst[keep]
    g, o = _pair(dfpr, n, src, dst)
    for k, (nd, ni) in enumerate([(0, 1), (2, 6), (20, 80)]):
        # batches drawn against the current edge set
        es, ed = _non_loop_edges(o)
        b = synth.random_batch(es, ed, n, nd, ni, seed=30 + k)
        assert g.apply_batch(b) == o.apply_batch(b)
        assert np.array_equal(g.mark_reachable(b), o.mark_reachable(b))
    assert not g.mark_reachable(synth.Batch.empty()).any()


def _non_loop_edges(o):
    off, idx = o.csr(out=True)
    src = np.repeat(np.arange(o.n, dtype=np.int32), np.diff(off))
    keep = src != idx
    return src[keep], idx[keep].astype(np.int32)


def test_dynamic_traversal_matches_oracle(dfpr):
    n, nA = 5000, 3000
    sa, da = synth.gnm(nA, 20000, seed=25)
    sb, db = synth.gnm(n - nA, 9000, seed=26)
    src = np.concatenate([sa, sb + nA])
    dst = np.concatenate([da, db + nA])
    g, o = _pair(dfpr, n, src, dst)
    p = dfpr.params(frontier_tol=1e-13)
    R0, _ = g.static(p)
    Ro, _ = o.static()
    b = synth.random_batch(sa, da, nA, 4, 16, seed=27)
    g.apply_batch(b)
    o.apply_batch(b)
    R, st = g.dynamic_traversal(b, p=p)
    Rt, sto, ft = o.dynamic_traversal(b, Ro, return_flags=True)
    assert st.converged and abs(st.iterations - sto.iterations) <= 1
    assert st.affected_initial == st.affected_final == int(ft.sum())
    assert np.max(np.abs(R - Rt)) < TOL_RANK
    assert np.array_equal(R[nA:], R0[nA:])           # unreached component untouched
    Rref, _ = o.reference()
    assert np.max(np.abs(R - Rref)) < TOL_RANK


# ---------------------------------------------------------------------------
# asynchronous form (tolerance-only parity: in-place updates race)
# ---------------------------------------------------------------------------

def test_async_form_reaches_the_reference(dfpr):
    n, src, dst = synth.rmat(13, 16, seed=31)
    g, o = _pair(dfpr, n, src, dst)
    pa = dfpr.params(frontier_tol=1e-13, mode=dfpr.ASYNC)
    ps = dfpr.params(frontier_tol=1e-13)
    Ra, sa = g.static(pa)
    Rref, _ = o.reference()
    assert sa.converged and np.max(np.abs(Ra - Rref)) < TOL_RANK
    counts = [synth.batch_counts(f, o.m) for f in (1e-4, 1e-3)]
    for i, b in enumerate(synth.batch_sequence(src, dst, n, counts, seed=32)):
        _say(f"async batch {i}")
        R_prev = g.ranks()
        g.apply_batch(b)
        o.apply_batch(b)
        Rref, _ = o.reference()
        Rs, ss = g.dynamic_frontier(b, p=ps)
        g.set_ranks(R_prev)
        Rd, sd = g.dynamic_frontier(b, p=pa)
        g.set_ranks(R_prev)
        Rt, st_ = g.dynamic_traversal(b, p=pa)
        g.set_ranks(R_prev)
        Rn, sn = g.naive_dynamic(p=pa)
        for R, s_ in ((Rd, sd), (Rt, st_), (Rn, sn)):
            assert s_.converged
            assert np.max(np.abs(R - Rref)) < TOL_RANK
        assert np.max(np.abs(Rd - Rs)) < TOL_RANK
        g.set_ranks(Rd)
    with pytest.raises(dfpr.DfprError):
        g.static(dfpr.params(mode=7))


# ---------------------------------------------------------------------------
# frontier tolerance and batch mixes (against the oracle with the same tau_f)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ftol", [1e-10, 1e-12, 1e-15])
@pytest.mark.parametrize("mix", ["insertions", "deletions"])
def test_frontier_tolerance_and_batch_mix(dfpr, ftol, mix):
    n, src, dst = synth.rmat(12, 16, seed=41)
    g, o = _pair(dfpr, n, src, dst)
    R0, _ = g.static()
    Ro, _ = o.static()
    bsz = 60
    cnt = (0, bsz) if mix == "insertions" else (bsz, 0)
    b = synth.batch_sequence(src, dst, n, [cnt], seed=42)[0]
    assert g.apply_batch(b) == o.apply_batch(b)
    R, st = g.dynamic_frontier(b, p=dfpr.params(frontier_tol=ftol))
    Rd, sto, _, f1, ch = o.dynamic_frontier(b, Ro, frontier_tol=ftol, return_flags=True,
                                            return_changes=True)
    assert st.converged and np.max(np.abs(R - Rd)) < TOL_RANK
    assert abs(st.iterations - sto.iterations) <= 1
    check_final_marks(g.affected(), f1, ch, *o.csr(out=False), ftol, f"{mix} {ftol}",
                      st.iterations == sto.iterations)


# ---------------------------------------------------------------------------
# resident ranks
# ---------------------------------------------------------------------------

def test_resident_ranks_round_trip_and_uniform_reset(dfpr):
    _say("set_ranks / get_ranks round trip, uniform reset")
    n, src, dst = synth.rmat(11, 8, seed=51)
    g = dfpr.Graph(n, src, dst)
    R = np.random.default_rng(52).random(n)
    R /= R.sum()
    g.set_ranks(R)
    assert np.array_equal(g.ranks(), R)
    # NULL restores the uniform start, so Naive-dynamic from the resident
    # ranks repeats the Static computation exactly
    g.set_ranks()
    assert np.array_equal(g.ranks(), np.full(n, 1.0 / n))
    Rn, sn = g.naive_dynamic()
    Rs, ss = g.static()
    assert sn.iterations == ss.iterations and np.array_equal(Rn, Rs)
    with pytest.raises(ValueError):
        g.set_ranks(np.zeros(n - 1))


def test_device_call_rejects_out_of_range_ids(dfpr):
    # ids in device arrays are checked by the device: the call ends with
    # DFPR_E_RANGE before any iteration and the resident ranks stay
    import torch
    _say("device Dynamic Frontier with an id outside [0, n)")
    n, src, dst = synth.rmat(10, 8, seed=61)
    g = dfpr.Graph(n, src, dst)
    R0, _ = g.static()
    bad = [torch.tensor(x, dtype=torch.int32, device="cuda")
           for x in ([], [], [0, 5], [1, n])]
    with pytest.raises(dfpr.DfprError) as e:
        g.dynamic_frontier_device(*bad)
    assert e.value.code == dfpr.DFPR_E_RANGE
    assert np.array_equal(g.ranks(), R0)
    with pytest.raises(ValueError):
        g.dynamic_frontier_device(*bad[:3], bad[3][:1])


def test_stats_split_device_time_by_phase(dfpr):
    _say("per-phase device times in the statistics")
    n, src, dst = synth.rmat(12, 16, seed=81)
    g = dfpr.Graph(n, src, dst)
    _, st = g.static()
    assert st.ms_apply == 0.0 and st.ms_mark >= 0.0 and st.ms_iter > 0.0
    b = synth.random_batch(src, dst, n, 20, 80, seed=82)
    g.apply_batch(b)
    for call in (lambda: g.dynamic_frontier(b), lambda: g.dynamic_traversal(b),
                 lambda: g.dynamic_frontier(b, p=dfpr.params(precision=dfpr.FP32_KAHAN))):
        _, st = call()
        assert st.ms_apply > 0.0 and st.ms_mark > 0.0 and st.ms_iter > 0.0
        assert abs(st.ms_mark + st.ms_iter - st.ms_device) <= 0.01 + 1e-3 * st.ms_device
    g.apply_batch(synth.Batch.empty())
    _, st = g.naive_dynamic()
    assert st.ms_apply == 0.0


def test_checkpoint_and_resume(dfpr, tmp_path):
    # a graph saved after some batches and loaded again continues the same
    # sequence: the same CSR after every batch, ranks within the parity
    # tolerance of the uninterrupted run (the reloaded graph renumbers its
    # vertices, so sums may round differently and a call may stop one
    # iteration apart)
    _say("checkpoint and resume")
    n, src, dst = synth.rmat(12, 16, seed=91)
    counts = [synth.batch_counts(f, src.size + n) for f in (1e-4, 1e-3, 1e-4, 1e-3)]
    seq = synth.batch_sequence(src, dst, n, counts, seed=92)
    g = dfpr.Graph(n, src, dst)
    g.static()
    for b in seq[:2]:
        g.apply_batch(b)
        g.dynamic_frontier(b)
    path = tmp_path / "ckpt.npz"
    g.save(path)
    h = dfpr.Graph.load(path)
    assert np.array_equal(h.ranks(), g.ranks())
    _same_csr_pair(g, h)
    for b in seq[2:]:
        assert g.apply_batch(b) == h.apply_batch(b)
        Rg, sg = g.dynamic_frontier(b)
        Rh, sh = h.dynamic_frontier(b)
        assert sg.converged and sh.converged and abs(sg.iterations - sh.iterations) <= 1
        assert np.max(np.abs(Rg - Rh)) < TOL_RANK
    _same_csr_pair(g, h)


def _same_csr_pair(a, b):
    for out in (True, False):
        x, y = a.csr(out), b.csr(out)
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


@pytest.mark.parametrize("n", [1, 2, 65])
def test_degenerate_graphs_every_method(dfpr, n):
    # one vertex (its self-loop only), two vertices and one edge, and a
    # complete digraph whose rows are one entry longer than a wave: every
    # method against the oracle's reference, and the closed form where
    # there is one (uniform ranks on a vertex-transitive graph)
    _say(f"degenerate graph n={n}")
    if n == 1:
        src = dst = np.zeros(0, np.int32)
        b = _batch([(0, 0)], [])                 # deleting a self-loop changes nothing
    elif n == 2:
        src, dst = np.array([0], np.int32), np.array([1], np.int32)
        b = _batch([(0, 1)], [(1, 0)])
    else:
        u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        keep = u != v
        src, dst = u[keep].astype(np.int32), v[keep].astype(np.int32)
        b = _batch([(0, 1)], [])
    g, o = _pair(dfpr, n, src, dst)
    R0, st = g.static()
    Ro, _ = o.static()
    assert st.converged and np.max(np.abs(R0 - Ro)) < TOL_RANK
    if n != 2:
        assert np.max(np.abs(R0 - 1.0 / n)) < 1e-15
    assert g.apply_batch(b) == o.apply_batch(b)
    _same_csr(g, o)
    Rref, _ = o.reference()
    runs = [("DF", lambda: g.dynamic_frontier(b, p=dfpr.params(frontier_tol=1e-13))),
            ("FP32 form", lambda: g.dynamic_frontier(
                b, p=dfpr.params(frontier_tol=1e-13, precision=dfpr.FP32_KAHAN))),
            ("DT", lambda: g.dynamic_traversal(b)),
            ("naive", lambda: g.naive_dynamic())]
    for name, call in runs:
        g.set_ranks(R0)
        R, s_ = call()
        assert s_.converged, name
        assert np.max(np.abs(R - Rref)) < TOL_RANK, name


def test_mega_row_star(dfpr):
    # a centre with 10^6 in-edges and 10^6 out-edges (bidirectional star):
    # the whole-workgroup row path over thousands of rounds, against the
    # closed form; then a batch at the centre, whose expansion scans its
    # million-entry out-row, against the oracle
    _say("star with 10^6 leaves")
    k = 1_000_000
    n = k + 1
    leaves = np.arange(1, k + 1, dtype=np.int32)
    src = np.concatenate([np.zeros(k, np.int32), leaves])
    dst = np.concatenate([leaves, np.zeros(k, np.int32)])
    g, o = _pair(dfpr, n, src, dst)
    R, st = g.static(dfpr.params(tol=1e-15))
    D = 2 * (k + 1) + 0.85 * (k - 1)
    assert st.converged
    # the centre's sum of 10^6 terms carries rounding up to k u sum|x|
    # (recursive summation, Higham 4.2), sum|x| <= 1
    assert abs(R[0] - (k + 1) / n * (2 + 0.85 * (k - 1)) / D) < k * 2.0 ** -53
    assert np.max(np.abs(R[1:] - (k + 1) / n * 2 / D)) < 1e-14
    Ro, _ = o.static()
    g.set_ranks(Ro)
    b = _batch([(0, 7)], [(5, 9)])
    assert g.apply_batch(b) == o.apply_batch(b) == (1, 1)
    Rd, sd = g.dynamic_frontier(b, p=dfpr.params(frontier_tol=1e-13))
    Rdo, sdo = o.dynamic_frontier(b, Ro, frontier_tol=1e-13)
    assert sd.converged and abs(sd.iterations - sdo.iterations) <= 1
    assert np.max(np.abs(Rd - Rdo)) < TOL_RANK


# ---------------------------------------------------------------------------
# small-frontier loop (Algorithm 1's loop inside one cooperative launch)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_frontier_loop_matches_launch_pairs_and_oracle(dfpr, precision):
    # a localised batch on a grid keeps the frontier small, so the call
    # runs inside the small-frontier loop when asked to; the same call with
    # one launch pair per iteration (the default) must give bitwise the same
    # ranks and marks, and both must match the oracle
    _say(f"small-frontier loop on a grid, {precision}")
    side = 128
    n, src, dst = synth.grid2d(side, 0.05, seed=5)
    g, o = _pair(dfpr, n, src, dst)
    prec = dfpr.FP64 if precision == "fp64" else dfpr.FP32_KAHAN
    R0, _ = g.static(dfpr.params(tol=1e-13))
    Ro, _ = o.static(tol=1e-13)
    b = synth.localized_batch(src, dst, side, 4, 16, seed=6)
    assert g.apply_batch(b) == o.apply_batch(b)
    pa = dfpr.params(frontier_tol=1e-13, precision=prec, loop=dfpr.LOOP_DEVICE)
    pl = dfpr.params(frontier_tol=1e-13, precision=prec)
    Ra, sa = g.dynamic_frontier(b, prev=R0, p=pa)
    fa = g.affected()
    Rl, sl = g.dynamic_frontier(b, prev=R0, p=pl)
    fl = g.affected()
    assert sa.converged and sl.converged
    _say(f"iterations {sa.iterations}, in the small loop {sa.loop_iterations}")
    assert sa.loop_iterations > 0 and sl.loop_iterations == 0
    assert sa.iterations == sl.iterations and sa.refine_sweeps == sl.refine_sweeps
    assert np.array_equal(Ra, Rl) and np.array_equal(fa, fl)
    Rd, sd, _, f1, ch = o.dynamic_frontier(b, Ro, frontier_tol=1e-13, return_flags=True,
                                           return_changes=True)
    assert np.max(np.abs(Ra - Rd)) < TOL_RANK
    if precision == "fp64":
        check_final_marks(fa, f1, ch, *o.csr(out=False), 1e-13, "small loop",
                          sa.iterations == sd.iterations)


def test_small_frontier_loop_hands_over_to_launches(dfpr):
    # on R-MAT the frontier of a one-edge batch outgrows the small loop
    # after a few iterations: the call continues with launch pairs and must
    # still equal the all-launches call bitwise and the oracle within 1e-9
    _say("small-frontier loop hand-over on R-MAT scale 16")
    n, src, dst = synth.rmat(16, 16, seed=7)
    g, o = _pair(dfpr, n, src, dst)
    R0, _ = g.static()
    Ro, _ = o.static()
    b = synth.random_batch(src, dst, n, 0, 1, seed=8)
    assert g.apply_batch(b) == o.apply_batch(b)
    Ra, sa = g.dynamic_frontier(b, prev=R0, p=dfpr.params(loop=dfpr.LOOP_DEVICE))
    Rl, sl = g.dynamic_frontier(b, prev=R0)
    assert sa.converged and sl.converged
    _say(f"iterations {sa.iterations}, in the small loop {sa.loop_iterations}")
    assert 0 < sa.loop_iterations < sa.iterations
    assert sa.iterations == sl.iterations and np.array_equal(Ra, Rl)
    Rd, sd = o.dynamic_frontier(b, Ro)
    assert np.max(np.abs(Ra - Rd)) < TOL_RANK
    with pytest.raises(dfpr.DfprError):
        g.dynamic_frontier(b, p=dfpr.params(loop=5))


# ---------------------------------------------------------------------------
# frontier tolerance on localised batches, and its adaptive choice
# ---------------------------------------------------------------------------

def _adaptive_exponent(marked, out_edges):
    # the rule of dfpr_params.frontier_tol, from the oracle's initial marks
    if marked == 0:
        return 5
    for k, t in ((1, 8), (2, 16), (3, 32), (4, 64)):
        if out_edges <= t * marked:
            return k
    return 5


@pytest.mark.parametrize("ftol", [1e-11, 1e-12, "adaptive"])
def test_localised_grid_batch_frontier_tolerance(dfpr, ftol):
    # tau/10 and tau/100 (the values Section 5.2.4 finds suitable for
    # temporal graphs) and the adaptive choice, on a localised grid batch:
    # ranks within 1e-9 of the oracle run at the same tolerance, final marks
    # as sets; the adaptive choice equals the rule applied to the oracle's
    # initial marks
    _say(f"localised grid batch, frontier tolerance {ftol}")
    side = 96
    n, src, dst = synth.grid2d(side, 0.05, seed=12)
    g, o = _pair(dfpr, n, src, dst)
    R0, _ = g.static(dfpr.params(tol=1e-13))
    Ro, _ = o.static(tol=1e-13)
    b = synth.localized_batch(src, dst, side, 3, 12, seed=13)
    assert g.apply_batch(b) == o.apply_batch(b)
    p = dfpr.params(frontier_tol=dfpr.FTOL_ADAPTIVE if ftol == "adaptive" else ftol)
    R, st = g.dynamic_frontier(b, prev=R0, p=p)
    if ftol == "adaptive":
        f0 = o.mark_initial(b).astype(bool)
        off, _ = o.csr(out=True)
        k = _adaptive_exponent(int(f0.sum()), int(np.diff(off)[f0].sum()))
        _say(f"adaptive: marked {int(f0.sum())}, exponent {k}")
        assert st.frontier_tol_used == 1e-10 / [1.0, 1e1, 1e2, 1e3, 1e4, 1e5][k]
        assert k == 1                      # a grid: every out-degree is at most 6
    else:
        assert st.frontier_tol_used == ftol
    Rd, sd, _, f1, ch = o.dynamic_frontier(b, Ro, frontier_tol=st.frontier_tol_used,
                                           return_flags=True, return_changes=True)
    assert st.converged and np.max(np.abs(R - Rd)) < TOL_RANK
    check_final_marks(g.affected(), f1, ch, *o.csr(out=False), st.frontier_tol_used,
                      f"grid {ftol}", st.iterations == sd.iterations)


def test_adaptive_frontier_tolerance_on_rmat(dfpr):
    # hub-rich neighbourhoods: the rule keeps the accurate tol/1e5
    _say("adaptive frontier tolerance on R-MAT scale 12")
    n, src, dst = synth.rmat(12, 16, seed=14)
    g, o = _pair(dfpr, n, src, dst)
    R0, _ = g.static()
    Ro, _ = o.static()
    b = synth.random_batch(src, dst, n, 4, 16, seed=15)
    assert g.apply_batch(b) == o.apply_batch(b)
    R, st = g.dynamic_frontier(b, p=dfpr.params(frontier_tol=dfpr.FTOL_ADAPTIVE))
    f0 = o.mark_initial(b).astype(bool)
    off, _ = o.csr(out=True)
    k = _adaptive_exponent(int(f0.sum()), int(np.diff(off)[f0].sum()))
    assert st.frontier_tol_used == 1e-10 / [1.0, 1e1, 1e2, 1e3, 1e4, 1e5][k]
    Rd, sd = o.dynamic_frontier(b, Ro, frontier_tol=st.frontier_tol_used)
    assert st.converged and np.max(np.abs(R - Rd)) < TOL_RANK
    with pytest.raises(dfpr.DfprError):
        g.dynamic_frontier(b, p=dfpr.params(frontier_tol=float("nan")))


def _wide_first_frontier_batch(n, src, dst, limit):
    """A deletion-only batch whose claimed sources reach few out-edges (the
    first walk stays on the class lists) while the vertices the marking
    marks have more out-edges than `limit`: deleted edges are sampled from
    existing ones, so their sources lean to hubs.  Found by a seeded search
    on the CPU; returns the batch and the marking's two out-edge sums."""
    outdeg = np.bincount(src, minlength=n) + 1           # with the self-loop
    for seed in range(200):
        for nd in (2, 3, 4):
            b = synth.batch_sequence(src, dst, n, [(nd, 0)], seed=1000 + seed)[0]
            # after the deletions each source has one out-edge fewer
            reach = int(outdeg[np.unique(b.del_src)].sum()) - nd
            if reach + nd > 0.8 * limit:
                continue
            marks = np.zeros(n, bool)
            for u in np.unique(b.del_src):
                marks[_out_row(src, dst, u)] = True
                marks[u] = True
            marks[b.del_dst] = True
            reach0 = int(outdeg[marks].sum())
            if marks.sum() < 0.8 * limit and reach0 > 2 * limit:
                return b, reach, reach0
    raise AssertionError("no batch with a wide first frontier found")


def _out_row(src, dst, u):
    return dst[src == u]


def test_wide_first_frontier_marks_plainly(dfpr):
    # R-MAT scale 16: class-list limit max(4096, n/64) = 4096.  The first
    # iteration walks the class lists, and its expansions mark with plain
    # stores and move the call to the full schedule (the marking's
    # out-edge sum exceeds the limit); ranks and final marks against the
    # oracle as in any other call
    n, src, dst = synth.rmat(16, 16, seed=21)
    limit = max(4096, n // 64)
    b, reach, reach0 = _wide_first_frontier_batch(n, src, dst, limit)
    _say(f"wide first frontier: {b.size} deletions, sources reach {reach}, marks reach {reach0}")
    g, o = _pair(dfpr, n, src, dst)
    p = dfpr.params(tol=1e-10, frontier_tol=1e-13)
    R0, _ = g.static(p)
    R0o, _ = o.static()
    assert g.apply_batch(b) == o.apply_batch(b)
    f0 = o.mark_initial(b)
    assert np.array_equal(g.mark_affected(b), f0)
    R, st = g.dynamic_frontier(b, p=p)
    Ro, sto, _, f1, ch = o.dynamic_frontier(b, R0o, frontier_tol=1e-13, return_flags=True,
                                            return_changes=True)
    assert st.converged and sto.converged
    assert st.affected_initial == int(f0.sum())
    assert np.max(np.abs(R - Ro)) < TOL_RANK
    check_final_marks(g.affected(), f1, ch, *o.csr(out=False), 1e-13, "wide first frontier",
                      st.iterations == sto.iterations)
    # the same call again from the same previous ranks: bitwise equal
    Rd, _ = g.dynamic_frontier(b, prev=R0, p=p)
    assert np.array_equal(R, Rd)
