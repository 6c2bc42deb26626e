"""CPU reference ("oracle") for Dynamic Frontier PageRank.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
benchmark's CPU-baseline leg import this package; the GPU library never
does, and the two share no code.

``OracleGraph`` wraps the plain C implementation in ``dfpr_oracle.c``
(FP64, sequential per-row sums, OpenMP over vertices); ``brute`` holds a
dense linear-solve reference for tiny graphs.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DFPR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (-O3, OpenMP; no contraction of a
    multiply and an add into one rounding)."""
    import subprocess

    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    src = os.path.join(_HERE, "dfpr_oracle.c")
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-ffp-contract=off", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("final_linf", ctypes.c_double),
        ("affected_initial", ctypes.c_int64),
        ("affected_final", ctypes.c_int64),
        ("vertices_processed", ctypes.c_int64),
        ("edges_processed", ctypes.c_int64),
    ]


@dataclass
class Stats:
    iterations: int
    converged: bool
    final_linf: float
    affected_initial: int
    affected_final: int
    vertices_processed: int
    edges_processed: int


def _stats(s: _Stats) -> Stats:
    return Stats(s.iterations, bool(s.converged), s.final_linf, s.affected_initial,
                 s.affected_final, s.vertices_processed, s.edges_processed)


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_load_graph.argtypes = [_I32, _I64, _P, _P, ctypes.POINTER(_P)]
        L.oracle_free_graph.argtypes = [_P]
        L.oracle_free_graph.restype = None
        L.oracle_graph_info.argtypes = [_P, _P, _P]
        L.oracle_export_csr.argtypes = [_P, ctypes.c_int, _P, _P]
        L.oracle_apply_batch.argtypes = [_P, _I64, _P, _P, _I64, _P, _P, _P]
        L.oracle_pagerank_static.argtypes = [_P, _D, _D, _I32, _P, _P]
        L.oracle_pagerank_naive_dynamic.argtypes = [_P, _D, _D, _I32, _P, _P, _P]
        L.oracle_pagerank_dynamic_frontier.argtypes = [
            _P, _D, _D, _D, _I32, _I64, _P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P]
        L.oracle_mark_initial_csr.argtypes = [_I32, _P, _P, _I64, _P, _P, _I64, _P, _P, _P]
        L.oracle_expand_csr.argtypes = [_I32, _P, _P, _P, _P, _D, _P]
        L.oracle_mark_reachable_csr.argtypes = [_I32, _P, _P, _I64, _P, _P, _I64, _P, _P, _P]
        L.oracle_pagerank_dynamic_traversal.argtypes = [
            _P, _D, _D, _I32, _I64, _P, _P, _I64, _P, _P, _P, _P, _P, _P]
        L.oracle_num_threads.argtypes = []
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_P) if a is not None else None


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


ALPHA = 0.85        # Section 5.1.2
TOL = 1e-10         # Section 5.1.2 (L-inf)
MAX_ITERS = 500     # Section 5.1.2


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(k: int) -> None:
    """Threads of the oracle's parallel loops from now on (results do not
    depend on it)."""
    lib().oracle_set_num_threads(int(k))


class OracleGraph:
    """A graph held by the C oracle (edge set with a self-loop per vertex)."""

    def __init__(self, n, src, dst):
        src, dst = _i32(src), _i32(dst)
        if src.shape != dst.shape:
            raise ValueError("src/dst length mismatch")
        h = _P()
        _check(lib().oracle_load_graph(int(n), int(src.size), _ptr(src), _ptr(dst),
                                       ctypes.byref(h)), "load_graph")
        self._h = h
        self.n = int(n)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().oracle_free_graph(h)
            self._h = None

    @property
    def m(self) -> int:
        m = _I64()
        lib().oracle_graph_info(self._h, None, ctypes.byref(m))
        return int(m.value)

    def csr(self, out: bool):
        off = np.zeros(self.n + 1, np.int64)
        idx = np.zeros(max(self.m, 1), np.int32)
        _check(lib().oracle_export_csr(self._h, 1 if out else 0, _ptr(off), _ptr(idx)),
               "export_csr")
        return off, idx[: self.m]

    def apply_batch(self, batch):
        ds, dd = _i32(batch.del_src), _i32(batch.del_dst)
        is_, id_ = _i32(batch.ins_src), _i32(batch.ins_dst)
        applied = np.zeros(2, np.int64)
        _check(lib().oracle_apply_batch(self._h, ds.size, _ptr(ds), _ptr(dd), is_.size,
                                        _ptr(is_), _ptr(id_), _ptr(applied)), "apply_batch")
        return int(applied[0]), int(applied[1])

    def static(self, alpha=ALPHA, tol=TOL, max_iters=MAX_ITERS):
        R = np.zeros(self.n, np.float64)
        st = _Stats()
        _check(lib().oracle_pagerank_static(self._h, alpha, tol, max_iters, _ptr(R),
                                            ctypes.byref(st)), "static")
        return R, _stats(st)

    def reference(self):
        """Reference Static of Section 5.1.5: tolerance 1e-100, at most 500
        iterations."""
        return self.static(ALPHA, 1e-100, 500)

    def naive_dynamic(self, prev, alpha=ALPHA, tol=TOL, max_iters=MAX_ITERS):
        prev = np.ascontiguousarray(prev, np.float64)
        R = np.zeros(self.n, np.float64)
        st = _Stats()
        _check(lib().oracle_pagerank_naive_dynamic(self._h, alpha, tol, max_iters,
                                                   _ptr(prev), _ptr(R), ctypes.byref(st)),
               "naive_dynamic")
        return R, _stats(st)

    def dynamic_frontier(self, batch, prev, alpha=ALPHA, tol=TOL, frontier_tol=TOL / 1e5,
                         max_iters=MAX_ITERS, return_flags=False, return_changes=False):
        """Dynamic Frontier on the current graph.  return_flags adds the
        initial and final marks; return_changes adds, per vertex, the
        largest rank change over the sweeps that processed it."""
        prev = np.ascontiguousarray(prev, np.float64)
        ds, dd = _i32(batch.del_src), _i32(batch.del_dst)
        is_, id_ = _i32(batch.ins_src), _i32(batch.ins_dst)
        R = np.zeros(self.n, np.float64)
        f0 = np.zeros(self.n, np.uint8)
        f1 = np.zeros(self.n, np.uint8)
        ch = np.zeros(self.n, np.float64) if return_changes else None
        st = _Stats()
        _check(lib().oracle_pagerank_dynamic_frontier(
            self._h, alpha, tol, frontier_tol, max_iters, ds.size, _ptr(ds), _ptr(dd),
            is_.size, _ptr(is_), _ptr(id_), _ptr(prev), _ptr(R), ctypes.byref(st),
            _ptr(f0), _ptr(f1), _ptr(ch)), "dynamic_frontier")
        out = (R, _stats(st))
        if return_flags:
            out += (f0, f1)
        if return_changes:
            out += (ch,)
        return out

    def mark_initial(self, batch):
        off, idx = self.csr(out=True)
        return mark_initial_csr(self.n, off, idx, batch)

    def mark_reachable(self, batch):
        off, idx = self.csr(out=True)
        return mark_reachable_csr(self.n, off, idx, batch)

    def dynamic_traversal(self, batch, prev, alpha=ALPHA, tol=TOL, max_iters=MAX_ITERS,
                          return_flags=False):
        """Dynamic Traversal PageRank (Section 3.3.2) on the current graph."""
        prev = np.ascontiguousarray(prev, np.float64)
        ds, dd = _i32(batch.del_src), _i32(batch.del_dst)
        is_, id_ = _i32(batch.ins_src), _i32(batch.ins_dst)
        R = np.zeros(self.n, np.float64)
        f = np.zeros(self.n, np.uint8)
        st = _Stats()
        _check(lib().oracle_pagerank_dynamic_traversal(
            self._h, alpha, tol, max_iters, ds.size, _ptr(ds), _ptr(dd), is_.size, _ptr(is_),
            _ptr(id_), _ptr(prev), _ptr(R), ctypes.byref(st), _ptr(f)), "dynamic_traversal")
        return (R, _stats(st), f) if return_flags else (R, _stats(st))


def mark_reachable_csr(n, out_off, out_idx, batch):
    """Dynamic Traversal marking (Section 3.3.2) on any out-CSR."""
    off = np.ascontiguousarray(out_off, np.int64)
    idx = _i32(out_idx) if len(out_idx) else np.zeros(1, np.int32)
    ds, dd = _i32(batch.del_src), _i32(batch.del_dst)
    is_, id_ = _i32(batch.ins_src), _i32(batch.ins_dst)
    flags = np.zeros(n, np.uint8)
    _check(lib().oracle_mark_reachable_csr(int(n), _ptr(off), _ptr(idx), ds.size, _ptr(ds),
                                           _ptr(dd), is_.size, _ptr(is_), _ptr(id_),
                                           _ptr(flags)), "mark_reachable_csr")
    return flags


def mark_initial_csr(n, out_off, out_idx, batch):
    """Initial marking (Section 4.1.1) on any out-CSR."""
    off = np.ascontiguousarray(out_off, np.int64)
    idx = _i32(out_idx) if len(out_idx) else np.zeros(1, np.int32)
    ds, dd = _i32(batch.del_src), _i32(batch.del_dst)
    is_, id_ = _i32(batch.ins_src), _i32(batch.ins_dst)
    flags = np.zeros(n, np.uint8)
    _check(lib().oracle_mark_initial_csr(int(n), _ptr(off), _ptr(idx), ds.size, _ptr(ds),
                                         _ptr(dd), is_.size, _ptr(is_), _ptr(id_),
                                         _ptr(flags)), "mark_initial_csr")
    return flags


def expand_csr(n, out_off, out_idx, affected, dr, frontier_tol):
    """Incremental marking (Section 4.1.1) on any out-CSR."""
    off = np.ascontiguousarray(out_off, np.int64)
    idx = _i32(out_idx) if len(out_idx) else np.zeros(1, np.int32)
    aff = np.ascontiguousarray(affected, np.uint8)
    dr = np.ascontiguousarray(dr, np.float64)
    nxt = np.zeros(n, np.uint8)
    _check(lib().oracle_expand_csr(int(n), _ptr(off), _ptr(idx), _ptr(aff), _ptr(dr),
                                   float(frontier_tol), _ptr(nxt)), "expand_csr")
    return nxt
