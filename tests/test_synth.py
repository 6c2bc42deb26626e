"""The seeded input generators: shapes, set properties and determinism."""
import numpy as np

from paper_2401_03256_amd import synth


def _keys(s, d, n):
    return synth.edge_keys(s, d, n)


def test_gnm_exact_distinct_no_loops_deterministic():
    s, d = synth.gnm(1000, 8000, seed=1)
    assert s.size == 8000 and s.dtype == np.int32
    assert not np.any(s == d)
    assert np.unique(_keys(s, d, 1000)).size == 8000
    s2, d2 = synth.gnm(1000, 8000, seed=1)
    assert np.array_equal(s, s2) and np.array_equal(d, d2)
    s3, _ = synth.gnm(1000, 8000, seed=2)
    assert not np.array_equal(s, s3)


def test_rmat_properties():
    n, s, d = synth.rmat(12, 16, seed=1)
    assert n == 4096
    assert s.min() >= 0 and max(s.max(), d.max()) < n
    assert not np.any(s == d)
    k = _keys(s, d, n)
    assert np.unique(k).size == k.size
    # skew: the lowest ids (many zero bits) carry far more than the mean degree
    indeg = np.bincount(d, minlength=n)
    assert indeg[0] > 20 * indeg.mean()
    # a < 0.25 + ... : the (0,0) quadrant dominates
    assert np.mean(s < n // 2) > 0.7
    n2, s2, d2 = synth.rmat(12, 16, seed=1)
    assert np.array_equal(s, s2) and np.array_equal(d, d2)


def test_grid_counts_and_symmetry():
    side = 64
    n, s, d = synth.grid2d(side, 0.05, seed=3)
    assert n == side * side
    k = set(_keys(s, d, n).tolist())
    assert all((v * n + u) in k for u, v in zip(s[:500], d[:500]))   # bidirectional
    four = 4 * side * (side - 1)
    assert four < s.size <= four + 2 * int(round(0.05 * n))
    assert not np.any(s == d)


def test_batch_counts_rounding():
    assert synth.batch_counts(1e-7, 70_000_000) == (1, 6)
    assert synth.batch_counts(1e-3, 90_000) == (18, 72)
    nd, ni = synth.batch_counts(80 / 90_000, 90_000)
    assert (nd, ni) == (16, 64)
    assert synth.batch_counts(1e-12, 10) == (0, 1)


def test_batch_sequence_is_effective_and_disjoint():
    n = 500
    s, d = synth.gnm(n, 3000, seed=4)
    base = set(_keys(s, d, n).tolist())
    seq = synth.batch_sequence(s, d, n, [(5, 20), (7, 30), (0, 3)], seed=8)
    dels, ins = [], []
    for b, (nd, ni) in zip(seq, [(5, 20), (7, 30), (0, 3)]):
        assert b.del_src.size == nd and b.ins_src.size == ni
        dels += _keys(b.del_src, b.del_dst, n).tolist()
        ins += _keys(b.ins_src, b.ins_dst, n).tolist()
        assert not np.any(b.ins_src == b.ins_dst)
    assert len(set(dels)) == len(dels) and set(dels) <= base
    assert len(set(ins)) == len(ins) and not (set(ins) & base)


def test_localized_batch_stays_in_window():
    side = 64
    n, s, d = synth.grid2d(side, 0.05, seed=1)
    b = synth.localized_batch(s, d, side, 4, 16, seed=2)
    pts = np.concatenate([b.del_src, b.del_dst, b.ins_src, b.ins_dst])
    r, c = pts // side, pts % side
    assert r.max() - r.min() < 10 and c.max() - c.min() < 10
    k = set(_keys(s, d, n).tolist())
    assert all(x in k for x in _keys(b.del_src, b.del_dst, n).tolist())
    assert not any(x in k for x in _keys(b.ins_src, b.ins_dst, n).tolist())


def test_rmat_permuted_is_a_relabelling():
    # the permuted graph is the same edge set under a bijection of the
    # vertex ids: equal sizes and degree multisets, ids moved, still a
    # sorted set without self-loops, and seeded
    n, s, d = synth.rmat(11, 8, seed=5)
    n2, s2, d2 = synth.rmat(11, 8, seed=5, permute=True)
    assert n == n2 and s.size == s2.size
    assert np.array_equal(np.sort(np.bincount(s, minlength=n)), np.sort(np.bincount(s2, minlength=n)))
    assert np.array_equal(np.sort(np.bincount(d, minlength=n)), np.sort(np.bincount(d2, minlength=n)))
    assert not np.array_equal(s, s2)
    keys = s2.astype(np.int64) * n + d2
    assert np.all(np.diff(keys) > 0) and np.all(s2 != d2)
    n3, s3, d3 = synth.rmat(11, 8, seed=5, permute=True)
    assert np.array_equal(s2, s3) and np.array_equal(d2, d3)
