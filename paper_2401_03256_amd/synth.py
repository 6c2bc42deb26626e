"""Seeded synthetic inputs: graphs and batch updates.

This module only draws random edge lists.  It holds none of the PageRank
arithmetic and none of the graph-update logic: adding self-loops, removing
duplicates inside the library and applying a batch are done separately by the
GPU library and by the CPU reference, each in its own code.  Both are fed the
same arrays produced here.

Every generator takes an explicit seed and uses numpy's PCG64, so the same
call gives the same bytes on any machine.

Edge lists are returned as two ``int32`` arrays ``(src, dst)`` holding a
*set* of directed edges ``u -> v`` with ``u != v`` (no duplicates, no
self-loops): the paper adds a self-loop to every vertex itself (Section 3.1,
Section 5.1.3), so the generators leave that to the graph loader.

Batch updates follow Section 5.1.4: insertions are vertex pairs drawn with
equal probability that are not already edges; deletions are existing edges
drawn uniformly; the default mix is 80% insertions and 20% deletions; the
vertex set never changes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Batch",
    "rng_for",
    "gnm",
    "rmat",
    "grid2d",
    "edge_keys",
    "batch_counts",
    "batch_sequence",
    "random_batch",
    "localized_batch",
]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def edge_keys(src: np.ndarray, dst: np.ndarray, n: int) -> np.ndarray:
    """Integer key ``u * n + v`` of each edge (int64); used for set tests."""
    return src.astype(np.int64) * np.int64(n) + dst.astype(np.int64)


def _split_keys(keys: np.ndarray, n: int):
    return (keys // n).astype(np.int32), (keys % n).astype(np.int32)


@dataclass
class Batch:
    """One batch update: deletions ``del_src -> del_dst`` and insertions."""

    del_src: np.ndarray
    del_dst: np.ndarray
    ins_src: np.ndarray
    ins_dst: np.ndarray

    @property
    def size(self) -> int:
        return int(self.del_src.size + self.ins_src.size)

    @staticmethod
    def empty() -> "Batch":
        z = np.zeros(0, np.int32)
        return Batch(z, z.copy(), z.copy(), z.copy())


# ---------------------------------------------------------------------------
# graphs
# ---------------------------------------------------------------------------


def gnm(n: int, m: int, seed: int):
    """Directed G(n, m): ``m`` distinct uniform pairs ``u != v``."""
    if m > n * (n - 1):
        raise ValueError("too many edges for a simple digraph")
    rng = rng_for(seed)
    keys = np.zeros(0, np.int64)
    while keys.size < m:
        need = m - keys.size
        draw = int(need * 1.2) + 16
        u = rng.integers(0, n, draw, dtype=np.int64)
        v = rng.integers(0, n, draw, dtype=np.int64)
        ok = u != v
        new = u[ok] * n + v[ok]
        # keep first occurrences in draw order, so the result does not depend
        # on how many extra draws were made
        _, first = np.unique(new, return_index=True)
        new = new[np.sort(first)]
        new = new[~np.isin(new, keys)]
        keys = np.concatenate([keys, new[:need]])
    keys = np.sort(keys)
    return _split_keys(keys, n)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 1, permute: bool = False):
    """R-MAT graph with ``2**scale`` vertices and ``edge_factor * 2**scale``
    generated edges; self-loops are dropped and duplicates removed.

    At every one of the ``scale`` levels an edge picks the quadrant
    (src bit, dst bit) = (0,0), (0,1), (1,0), (1,1) with probabilities
    a, b, c, d = 1 - a - b - c.  By default vertex ids are not permuted, so
    high-degree vertices sit at ids with many zero bits and ids that share
    their bits share neighbourhoods.  ``permute`` relabels the vertices by a
    seeded uniform permutation (the Graph500 convention), which removes that
    id structure; the edge set is otherwise the same.
    """
    n = 1 << scale
    m_raw = edge_factor * n
    rng = rng_for(seed)
    u = np.zeros(m_raw, np.uint32)
    v = np.zeros(m_raw, np.uint32)
    ta, tab, tabc = np.float32(a), np.float32(a + b), np.float32(a + b + c)
    for level in range(scale):
        r = rng.random(m_raw, dtype=np.float32)
        ubit = r >= tab                      # quadrants c and d
        vbit = ((r >= ta) & (r < tab)) | (r >= tabc)   # quadrants b and d
        u |= ubit.astype(np.uint32) << np.uint32(level)
        v |= vbit.astype(np.uint32) << np.uint32(level)
        del r, ubit, vbit
    keep = u != v
    keys = (u[keep].astype(np.int64) << 32) | v[keep].astype(np.int64)
    del u, v, keep
    keys = np.unique(keys)
    if permute:
        # new label of each vertex, from a stream of its own
        perm = rng_for(seed + (1 << 40)).permutation(n).astype(np.int64)
        keys = (perm[keys >> 32] << 32) | perm[keys & 0xFFFFFFFF]
        keys.sort()
    src = (keys >> 32).astype(np.int32)
    dst = (keys & 0xFFFFFFFF).astype(np.int32)
    return n, src, dst


def grid2d(side: int, diag_frac: float = 0.05, seed: int = 1):
    """``side x side`` grid with bidirectional 4-neighbour edges plus, for a
    seeded ``diag_frac`` of the vertices, a bidirectional edge to one random
    existing diagonal neighbour.  Vertex id = row * side + col."""
    n = side * side
    ids = np.arange(n, dtype=np.int64).reshape(side, side)
    h_a = ids[:, :-1].ravel()
    h_b = ids[:, 1:].ravel()
    v_a = ids[:-1, :].ravel()
    v_b = ids[1:, :].ravel()
    rng = rng_for(seed)
    k = int(round(diag_frac * n))
    pick = rng.choice(n, size=k, replace=False).astype(np.int64)
    r, c = pick // side, pick % side
    dirs = rng.integers(0, 4, k)
    dr = np.where(dirs < 2, -1, 1)
    dc = np.where(dirs % 2 == 0, -1, 1)
    # reflect a direction that leaves the grid, so every pick gets an edge
    dr = np.where((r + dr < 0) | (r + dr >= side), -dr, dr)
    dc = np.where((c + dc < 0) | (c + dc >= side), -dc, dc)
    other = (r + dr) * side + (c + dc)
    src = np.concatenate([h_a, h_b, v_a, v_b, pick, other])
    dst = np.concatenate([h_b, h_a, v_b, v_a, other, pick])
    keys = np.unique(src * n + dst)
    s, d = _split_keys(keys, n)
    return n, s, d


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------


def batch_counts(frac: float, num_edges: int, ins_frac: float = 0.8):
    """Batch of ``max(1, round(frac * |E|))`` edges split into
    ``round(ins_frac * B)`` insertions and the rest deletions.  ``num_edges``
    is |E| including self-loops, as Table 1 counts it."""
    bsz = max(1, int(round(frac * num_edges)))
    ni = int(round(ins_frac * bsz))
    return bsz - ni, ni


def _sample_new_pairs(rng, n, count, exclude_sorted):
    """``count`` distinct uniform pairs ``u != v`` whose key is not in
    ``exclude_sorted`` (sorted int64 keys)."""
    out = np.zeros(0, np.int64)
    while out.size < count:
        need = count - out.size
        draw = int(need * 1.1) + 16
        u = rng.integers(0, n, draw, dtype=np.int64)
        v = rng.integers(0, n, draw, dtype=np.int64)
        key = u * n + v
        ok = u != v
        if exclude_sorted.size:
            pos = np.searchsorted(exclude_sorted, key)
            pos = np.minimum(pos, exclude_sorted.size - 1)
            ok &= exclude_sorted[pos] != key
        key = key[ok]
        _, first = np.unique(key, return_index=True)
        key = key[np.sort(first)]
        if out.size:
            key = key[~np.isin(key, out)]
        out = np.concatenate([out, key[:need]])
    return out


def batch_sequence(src, dst, n, counts, seed, protect_keys=None):
    """A sequence of batches for the base edge set ``(src, dst)``.

    ``counts`` is a list of ``(n_del, n_ins)``.  Deletions are drawn
    uniformly without replacement from the base edges, disjoint across the
    whole sequence; insertions are new uniform pairs, absent from the base
    edge set and distinct across the sequence.  Applied one after another,
    every entry of every batch therefore changes the graph.
    ``protect_keys`` (optional int64 keys) are never deleted.
    """
    rng = rng_for(seed)
    m0 = int(src.size)
    tot_del = int(sum(c[0] for c in counts))
    tot_ins = int(sum(c[1] for c in counts))
    base_keys = edge_keys(src, dst, n)
    order = np.argsort(base_keys, kind="stable")
    sorted_keys = base_keys[order]
    if protect_keys is not None and len(protect_keys):
        allowed = np.flatnonzero(~np.isin(base_keys, protect_keys))
    else:
        allowed = None
    pool = m0 if allowed is None else allowed.size
    if tot_del > pool:
        raise ValueError("not enough edges to delete")
    pick = rng.choice(pool, size=tot_del, replace=False) if tot_del else np.zeros(0, np.int64)
    if allowed is not None:
        pick = allowed[pick]
    new = _sample_new_pairs(rng, n, tot_ins, sorted_keys)
    out = []
    pd = pi = 0
    for nd, ni in counts:
        dsel = pick[pd:pd + nd]
        isel = new[pi:pi + ni]
        pd += nd
        pi += ni
        out.append(Batch(src[dsel].astype(np.int32), dst[dsel].astype(np.int32),
                         (isel // n).astype(np.int32), (isel % n).astype(np.int32)))
    return out


def random_batch(src, dst, n, n_del, n_ins, seed):
    """One uniformly random batch (Section 5.1.4)."""
    return batch_sequence(src, dst, n, [(n_del, n_ins)], seed)[0]


def localized_batch(src, dst, side, n_del, n_ins, seed, max_hop=2):
    """Batch whose endpoints all lie in one seeded square window of a
    ``side x side`` grid graph.  The window holds about ``4 * (n_del + n_ins)``
    vertices; insertions join window cells at Chebyshev distance at most
    ``max_hop`` that are not already joined; deletions are drawn among the
    existing edges with both endpoints inside the window."""
    n = side * side
    rng = rng_for(seed)
    bsz = n_del + n_ins
    w = max(3, int(np.ceil(np.sqrt(4 * max(bsz, 1)))))
    w = min(w, side)
    r0 = int(rng.integers(0, side - w + 1))
    c0 = int(rng.integers(0, side - w + 1))
    sr, sc = src // side, src % side
    dr_, dc_ = dst // side, dst % side
    inwin = ((sr >= r0) & (sr < r0 + w) & (sc >= c0) & (sc < c0 + w) &
             (dr_ >= r0) & (dr_ < r0 + w) & (dc_ >= c0) & (dc_ < c0 + w))
    cand = np.flatnonzero(inwin)
    if n_del > cand.size:
        raise ValueError("window too small for the requested deletions")
    dsel = rng.choice(cand, size=n_del, replace=False) if n_del else np.zeros(0, np.int64)
    keys_sorted = np.sort(edge_keys(src, dst, n))
    ins = np.zeros(0, np.int64)
    while ins.size < n_ins:
        need = n_ins - ins.size
        draw = 2 * need + 16
        ur = rng.integers(r0, r0 + w, draw)
        uc = rng.integers(c0, c0 + w, draw)
        vr = ur + rng.integers(-max_hop, max_hop + 1, draw)
        vc = uc + rng.integers(-max_hop, max_hop + 1, draw)
        ok = (vr >= r0) & (vr < r0 + w) & (vc >= c0) & (vc < c0 + w)
        ok &= (vr != ur) | (vc != uc)
        key = (ur * side + uc).astype(np.int64) * n + (vr * side + vc)
        pos = np.minimum(np.searchsorted(keys_sorted, key), keys_sorted.size - 1)
        ok &= keys_sorted[pos] != key
        key = key[ok]
        _, first = np.unique(key, return_index=True)
        key = key[np.sort(first)]
        if ins.size:
            key = key[~np.isin(key, ins)]
        ins = np.concatenate([ins, key[:need]])
    return Batch(src[dsel].astype(np.int32), dst[dsel].astype(np.int32),
                 (ins // n).astype(np.int32), (ins % n).astype(np.int32))
