"""Dense reference for tiny graphs — TEST INFRASTRUCTURE ONLY.

The PageRank vector is the fixed point of Eq. 1.  Writing Eq. 1 for all
vertices at once gives the linear system

    (I - alpha * P) R = (1 - alpha) / n * 1,   P[v, u] = 1 / |out(u)| if u -> v,

which is solved here with ``numpy.linalg.solve`` (LU) in FP64.  The edge set
(with a self-loop on every vertex, Section 3.1) is built from the raw edge
list with a Python set, independently of the C oracle's CSR code.
"""
from __future__ import annotations

import numpy as np


def edge_set(n, src, dst):
    E = {(int(u), int(v)) for u, v in zip(src, dst)}
    E |= {(v, v) for v in range(n)}
    return E


def pagerank_dense(n, edges, alpha=0.85):
    """Exact PageRank of the edge set ``edges`` (a set of (u, v) pairs that
    already holds every self-loop)."""
    if n > 64:
        raise ValueError("dense reference is for tiny graphs")
    outdeg = np.zeros(n)
    for u, _ in edges:
        outdeg[u] += 1
    P = np.zeros((n, n))
    for u, v in edges:
        P[v, u] += 1.0 / outdeg[u]
    A = np.eye(n) - alpha * P
    b = np.full(n, (1.0 - alpha) / n)
    return np.linalg.solve(A, b)


def csr_from_set(n, edges, out: bool):
    """Sorted CSR (offsets int64, idx int32) of an edge set."""
    rows = [[] for _ in range(n)]
    for u, v in edges:
        if out:
            rows[u].append(v)
        else:
            rows[v].append(u)
    off = np.zeros(n + 1, np.int64)
    idx = []
    for r in range(n):
        rows[r].sort()
        off[r + 1] = off[r] + len(rows[r])
        idx.extend(rows[r])
    return off, np.array(idx, dtype=np.int32)
