"""The entry point for callers that cannot allocate
(dfpr_pagerank_dynamic_frontier_device_noalloc) against the existing
device entry point, through the C-ABI: the same ranks, bitwise, and the
same statistics, on two calls in a row, the second with a smaller batch;
after the first call on the device (which places the library's fixed
array there), free device memory unchanged across a call; an oversized
batch refused with nothing changed."""
import sys

import numpy as np
import pytest

from paper_2401_03256_amd import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    sys.stdout.write(f"\n[case] {msg}\n")
    sys.stdout.flush()


def test_noalloc_matches_device_entry_twice():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2401_03256_amd import dfpr
    dfpr.lib()
    n, src, dst = synth.rmat(14, 16, seed=21)
    ga = dfpr.Graph(n, src, dst)      # the existing entry point
    gb = dfpr.Graph(n, src, dst)      # the entry point that allocates nothing
    p = dfpr.params(frontier_tol=1e-13)
    ga.static(p)
    gb.static(p)
    m = ga.m
    counts = [synth.batch_counts(1e-2, m), synth.batch_counts(1e-4, m)]
    seq = synth.batch_sequence(src, dst, n, counts, seed=22)
    assert seq[1].size < seq[0].size
    for k, b in enumerate(seq):
        _say(f"no-allocation entry point, call {k}: batch of {b.size}")
        t = [torch.from_numpy(np.ascontiguousarray(x)).cuda()
             for x in (b.del_src, b.del_dst, b.ins_src, b.ins_dst)]
        assert ga.apply_batch_device(*t) == gb.apply_batch_device(*t)
        ra = torch.empty(n, dtype=torch.float64, device="cuda")
        rb = torch.empty(n, dtype=torch.float64, device="cuda")
        sa = ga.dynamic_frontier_device(*t, out=ra, p=p)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        sb = gb.dynamic_frontier_device(*t, out=rb, p=p, noalloc=True)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        if k > 0:
            assert free1 >= free0, "the no-allocation call took device memory"
        assert sb.converged and sa.converged
        assert (sb.iterations, sb.affected_initial, sb.affected_final, sb.edges_processed) == \
            (sa.iterations, sa.affected_initial, sa.affected_final, sa.edges_processed)
        assert torch.equal(ra, rb)
        assert np.array_equal(ga.affected(), gb.affected())
    # a batch beyond the limit is refused and changes nothing
    big = torch.zeros((1 << 20) + 1, dtype=torch.int32, device="cuda")
    none = torch.zeros(0, dtype=torch.int32, device="cuda")
    before = gb.ranks()
    with pytest.raises(dfpr.DfprError) as e:
        gb.dynamic_frontier_device(none, none, big, big, p=p, noalloc=True)
    assert e.value.code == dfpr.DFPR_E_LIMIT
    assert np.array_equal(gb.ranks(), before)
